"""Thin ctypes binding of libfwr (C ABI in include/fwr.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
library.  torch is used for device memory and streams.  If the library is
missing or fails to load this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FWR_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("FWR_LIBRARY") or os.path.join(_HERE, "libfwr.so")

FWR_OK = 0
FWR_E_INVAL = -1
FWR_E_UNSUPPORTED = -2
FWR_E_NOMEM = -3
FWR_E_DEVICE = -4
FWR_E_STATE = -5
FWR_MODEL_FRIED = 0
FWR_MODEL_SINC = 1
MODELS = {"fried": FWR_MODEL_FRIED, "sinc": FWR_MODEL_SINC}

# grid sizes handled by the on-chip kernel (N = 4 t)
ONCHIP_GRIDS = (8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 128)

EXPORTED = ("fwr_plan", "fwr_extend", "fwr_reconstruct", "fwr_destroy", "fwr_set_stream",
            "fwr_plan_launch_info", "fwr_status_string", "fwr_extend_start", "fwr_reconstruct_start",
            "fwr_cnn_create", "fwr_cnn_set_params", "fwr_cnn_get_params", "fwr_cnn_forward",
            "fwr_cnn_backward", "fwr_cnn_get_grads", "fwr_cnn_adam_step", "fwr_cnn_destroy",
            "fwr_reconstruct_group", "fwr_generate", "fwr_cnn_set_stream", "fwr_plan_set_group",
            "fwr_plan_autotune", "fwr_hudgin_extend", "fwr_reconstruct_learned", "fwr_plan_set_schedule",
            "fwr_plan_get_schedule", "fwr_reconstruct_learned_noalloc", "fwr_cnn_loss_grad",
            "fwr_cnn_backward_grad", "fwr_fried_slopes", "fwr_plan_set_wait_limit")
CNN_PARAMS = 47714


class FwrParams(ctypes.Structure):
    _fields_ = [
        ("n_sub", ctypes.c_int32),
        ("n_grid", ctypes.c_int32),
        ("mask", ctypes.POINTER(ctypes.c_uint8)),
        ("n_iter", ctypes.c_int32),
        ("periodic", ctypes.c_int32),
        ("periodic_each_iter", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("noise_var", ctypes.c_double),
        ("r0", ctypes.c_double),
        ("L0", ctypes.c_double),
        ("d", ctypes.c_double),
        ("alpha_map", ctypes.POINTER(ctypes.c_double)),
        ("max_batch", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("d_px", ctypes.c_double),
    ]


class FwrWork(ctypes.Structure):
    _fields_ = [
        ("plan", ctypes.c_void_p),
        ("d_slopes", ctypes.c_void_p),
        ("d_phase", ctypes.c_void_p),
        ("d_start", ctypes.c_void_p),
        ("d_resid", ctypes.c_void_p),
        ("B", ctypes.c_int32),
    ]


class FwrError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Open libfwr.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} not found: build it with `python -m paper_1705_04298_amd.build`")
    lib = ctypes.CDLL(path)
    lib.fwr_plan.argtypes = [ctypes.POINTER(FwrParams), ctypes.POINTER(ctypes.c_void_p)]
    lib.fwr_plan.restype = ctypes.c_int
    for name in ("fwr_extend", "fwr_reconstruct"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        f.restype = ctypes.c_int
    lib.fwr_destroy.argtypes = [ctypes.c_void_p]
    lib.fwr_destroy.restype = ctypes.c_int
    lib.fwr_set_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.fwr_set_stream.restype = ctypes.c_int
    lib.fwr_plan_launch_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.fwr_plan_launch_info.restype = ctypes.c_int
    lib.fwr_status_string.argtypes = [ctypes.c_int32]
    lib.fwr_status_string.restype = ctypes.c_char_p
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    for name in ("fwr_extend_start", "fwr_reconstruct_start"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, vp, vp, i32]
        f.restype = ctypes.c_int
    lib.fwr_cnn_create.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_uint8), i32, f32, i32, vp,
                                   ctypes.POINTER(vp)]
    lib.fwr_cnn_create.restype = ctypes.c_int
    for name in ("fwr_cnn_set_params", "fwr_cnn_get_params", "fwr_cnn_get_grads"):
        f = getattr(lib, name)
        f.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
        f.restype = ctypes.c_int
    lib.fwr_cnn_forward.argtypes = [vp, vp, vp, i32]
    lib.fwr_cnn_forward.restype = ctypes.c_int
    lib.fwr_cnn_backward.argtypes = [vp, vp, vp, i32, ctypes.POINTER(ctypes.c_float)]
    lib.fwr_cnn_backward.restype = ctypes.c_int
    lib.fwr_cnn_loss_grad.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_float)]
    lib.fwr_cnn_loss_grad.restype = ctypes.c_int
    lib.fwr_cnn_backward_grad.argtypes = [vp, vp, i32]
    lib.fwr_cnn_backward_grad.restype = ctypes.c_int
    lib.fwr_cnn_adam_step.argtypes = [vp, f32]
    lib.fwr_cnn_adam_step.restype = ctypes.c_int
    lib.fwr_cnn_set_stream.argtypes = [vp, vp]
    lib.fwr_cnn_set_stream.restype = ctypes.c_int
    lib.fwr_cnn_destroy.argtypes = [vp]
    lib.fwr_cnn_destroy.restype = ctypes.c_int
    lib.fwr_reconstruct_learned.argtypes = [vp, vp, vp, vp, vp, vp, vp, f32, i32, ctypes.POINTER(i32)]
    lib.fwr_reconstruct_learned.restype = ctypes.c_int
    lib.fwr_reconstruct_learned_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, f32, i32, vp]
    lib.fwr_reconstruct_learned_noalloc.restype = ctypes.c_int
    lib.fwr_hudgin_extend.argtypes = [vp, vp, vp, i32]
    lib.fwr_hudgin_extend.restype = ctypes.c_int
    lib.fwr_fried_slopes.argtypes = [vp, vp, vp, vp, i32]
    lib.fwr_fried_slopes.restype = ctypes.c_int
    lib.fwr_plan_set_group.argtypes = [vp, i32]
    lib.fwr_plan_set_group.restype = ctypes.c_int
    lib.fwr_plan_set_schedule.argtypes = [vp, i32]
    lib.fwr_plan_set_schedule.restype = ctypes.c_int
    lib.fwr_plan_set_wait_limit.argtypes = [vp, i32]
    lib.fwr_plan_set_wait_limit.restype = ctypes.c_int
    lib.fwr_plan_get_schedule.argtypes = [vp, ctypes.POINTER(i32)]
    lib.fwr_plan_get_schedule.restype = ctypes.c_int
    lib.fwr_plan_autotune.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.fwr_plan_autotune.restype = ctypes.c_int
    lib.fwr_reconstruct_group.argtypes = [ctypes.POINTER(FwrWork), i32, vp]
    lib.fwr_reconstruct_group.restype = ctypes.c_int
    u64 = ctypes.c_uint64
    lib.fwr_generate.argtypes = [vp, u64, u64, vp, f32, f32, f32, vp, vp, i32]
    lib.fwr_generate.restype = ctypes.c_int
    _lib = lib
    return lib


def fwr_reconstruct_learned(plan, fallback, cnn, d_slopes: int, d_start: int, d_phase: int, d_resid: int,
                            threshold: float, B: int, count=None) -> int:
    return load().fwr_reconstruct_learned(plan, fallback, cnn, ctypes.c_void_p(d_slopes), ctypes.c_void_p(d_start),
                                          ctypes.c_void_p(d_phase), ctypes.c_void_p(d_resid), float(threshold),
                                          B, count)


def fwr_reconstruct_learned_noalloc(plan, fallback, cnn, d_slopes: int, d_start: int, d_phase: int, d_resid: int,
                                    threshold: float, B: int, d_count: int = 0) -> int:
    """The allocation-free learned call; d_count: device int32 address or 0."""
    return load().fwr_reconstruct_learned_noalloc(plan, fallback, cnn, ctypes.c_void_p(d_slopes),
                                                  ctypes.c_void_p(d_start), ctypes.c_void_p(d_phase),
                                                  ctypes.c_void_p(d_resid), float(threshold), B,
                                                  ctypes.c_void_p(d_count or None))


def status_string(status: int) -> str:
    return load().fwr_status_string(int(status)).decode()


# ----------------------------------------------------------------- raw C calls

def fwr_plan(params: FwrParams) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = load().fwr_plan(ctypes.byref(params), ctypes.byref(h))
    if st != FWR_OK:
        raise FwrError(st, "fwr_plan")
    return h


def fwr_extend(plan, d_slopes: int, d_ext: int, B: int) -> int:
    return load().fwr_extend(plan, ctypes.c_void_p(d_slopes), ctypes.c_void_p(d_ext), int(B))


def fwr_reconstruct(plan, d_slopes: int, d_phase: int, B: int) -> int:
    return load().fwr_reconstruct(plan, ctypes.c_void_p(d_slopes), ctypes.c_void_p(d_phase), int(B))


def fwr_extend_start(plan, d_slopes: int, d_start: int, d_ext: int, d_resid: int, B: int) -> int:
    return load().fwr_extend_start(plan, d_slopes or None, d_start or None, d_ext or None, d_resid or None, int(B))


def fwr_reconstruct_start(plan, d_slopes: int, d_start: int, d_phase: int, d_resid: int, B: int) -> int:
    return load().fwr_reconstruct_start(plan, d_slopes or None, d_start or None, d_phase or None,
                                        d_resid or None, int(B))


def fwr_destroy(plan) -> int:
    return load().fwr_destroy(plan)


def fwr_set_stream(plan, stream: int) -> int:
    return load().fwr_set_stream(plan, ctypes.c_void_p(stream))


def fwr_reconstruct_group(items, stream: int) -> int:
    """items: sequence of (plan handle, d_slopes, d_phase, d_start, d_resid, B) device pointers (0 = NULL)."""
    arr = (FwrWork * max(1, len(items)))()
    for i, (h, s, o, st, r, B) in enumerate(items):
        arr[i].plan, arr[i].d_slopes, arr[i].d_phase = h, s or None, o or None
        arr[i].d_start, arr[i].d_resid, arr[i].B = st or None, r or None, int(B)
    return load().fwr_reconstruct_group(arr, len(items), ctypes.c_void_p(stream))


def fwr_generate(plan, seed: int, first_frame: int, d_counter: int, r0: float, L0: float, sigma: float,
                 d_slopes: int, d_phase: int, B: int) -> int:
    return load().fwr_generate(plan, ctypes.c_uint64(seed), ctypes.c_uint64(first_frame), d_counter or None,
                               float(r0), float(L0), float(sigma), d_slopes or None, d_phase or None, int(B))


def fwr_plan_launch_info(plan):
    t, f, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    st = load().fwr_plan_launch_info(plan, ctypes.byref(t), ctypes.byref(f), ctypes.byref(l))
    if st != FWR_OK:
        raise FwrError(st, "fwr_plan_launch_info")
    return t.value, f.value, l.value


# ----------------------------------------------------------------- convenience

def _current_stream() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A reconstruction plan bound to the current device and (by default) torch's current stream.

    Inputs and outputs are torch CUDA float32 tensors, C-contiguous:
    slopes ``[B, 2, n, n]``; phase ``[B, n+1, n+1]``; extended slopes ``[B, 2, N, N]``.
    """

    def __init__(self, n_sub: int, n_grid: int, mask, n_iter: int = 10, periodic: bool = True,
                 periodic_each_iter: bool = False, gamma: float = 1.0, noise_var: float = 0.05 ** 2,
                 r0: float = 0.15, L0: float = 25.0, d: float = 0.2,
                 alpha_map: Optional[np.ndarray] = None, max_batch: int = 4096,
                 stream: Optional[int] = None, model: str = "fried", d_px: float = 0.0):
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        if mask.shape != (n_sub, n_sub):
            raise ValueError(f"mask must be {n_sub}x{n_sub}")
        self._mask = mask
        self._alpha = None if alpha_map is None else np.ascontiguousarray(alpha_map, dtype=np.float64)
        self.n_sub, self.n_grid, self.max_batch = int(n_sub), int(n_grid), int(max_batch)
        self.stream = _current_stream() if stream is None else int(stream)
        p = FwrParams()
        p.n_sub, p.n_grid = self.n_sub, self.n_grid
        p.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        p.n_iter, p.periodic, p.periodic_each_iter = int(n_iter), int(bool(periodic)), int(bool(periodic_each_iter))
        if model not in MODELS:
            raise ValueError(f"model must be one of {sorted(MODELS)}")
        self.model = model
        p.model = MODELS[model]
        p.gamma, p.noise_var, p.r0, p.L0, p.d = float(gamma), float(noise_var), float(r0), float(L0), float(d)
        p.alpha_map = (self._alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                       if self._alpha is not None else None)
        p.max_batch = self.max_batch
        p.stream = self.stream
        p.d_px = float(d_px)
        self._h = fwr_plan(p)

    def _check(self, t, shape, name):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def _start_args(self, start, resid, B):
        sp = rp = 0
        if start is not None:
            self._check(start, (B, 2, self.n_grid, self.n_grid), "start")
            sp = start.data_ptr()
        if resid is not None:
            self._check(resid, (B,), "resid")
            rp = resid.data_ptr()
        return sp, rp

    def reconstruct(self, slopes, out=None, start=None, resid=None):
        """Phase [B, n+1, n+1]; optional start slopes [B, 2, N, N] and residual output [B]."""
        import torch
        B = slopes.shape[0]
        self._check(slopes, (B, 2, self.n_sub, self.n_sub), "slopes")
        if out is None:
            out = torch.empty((B, self.n_sub + 1, self.n_sub + 1), device=slopes.device, dtype=torch.float32)
        self._check(out, (B, self.n_sub + 1, self.n_sub + 1), "out")
        if start is None and resid is None:
            st = fwr_reconstruct(self._h, slopes.data_ptr(), out.data_ptr(), B)
        else:
            sp, rp = self._start_args(start, resid, B)
            st = fwr_reconstruct_start(self._h, slopes.data_ptr(), sp, out.data_ptr(), rp, B)
        if st != FWR_OK:
            raise FwrError(st, "fwr_reconstruct")
        return out

    def extend(self, slopes, out=None, start=None, resid=None):
        """Extended slopes [B, 2, N, N]; optional start slopes and residual output as reconstruct."""
        import torch
        B = slopes.shape[0]
        self._check(slopes, (B, 2, self.n_sub, self.n_sub), "slopes")
        if out is None:
            out = torch.empty((B, 2, self.n_grid, self.n_grid), device=slopes.device, dtype=torch.float32)
        self._check(out, (B, 2, self.n_grid, self.n_grid), "out")
        if start is None and resid is None:
            st = fwr_extend(self._h, slopes.data_ptr(), out.data_ptr(), B)
        else:
            sp, rp = self._start_args(start, resid, B)
            st = fwr_extend_start(self._h, slopes.data_ptr(), sp, out.data_ptr(), rp, B)
        if st != FWR_OK:
            raise FwrError(st, "fwr_extend")
        return out

    def launch_info(self):
        return fwr_plan_launch_info(self._h)

    def hudgin_extend(self, slopes, out=None):
        """The comparison (Hudgin) extension with Eq. 5: extended slopes [B, 2, N, N]."""
        import torch
        B = slopes.shape[0]
        self._check(slopes, (B, 2, self.n_sub, self.n_sub), "slopes")
        if out is None:
            out = torch.empty((B, 2, self.n_grid, self.n_grid), device=slopes.device, dtype=torch.float32)
        self._check(out, (B, 2, self.n_grid, self.n_grid), "out")
        st = load().fwr_hudgin_extend(self._h, ctypes.c_void_p(slopes.data_ptr()), ctypes.c_void_p(out.data_ptr()), B)
        if st != FWR_OK:
            raise FwrError(st, "fwr_hudgin_extend")
        return out

    def fried_slopes(self, phase, noise=None, out=None):
        """The plan's Fried slope model on node phases [B, n+1, n+1] (+ noise [B, 2, n, n]), zero on
        invalid subapertures: slopes [B, 2, n, n] (fwr_fried_slopes)."""
        import torch
        B = phase.shape[0]
        self._check(phase, (B, self.n_sub + 1, self.n_sub + 1), "phase")
        if noise is not None:
            self._check(noise, (B, 2, self.n_sub, self.n_sub), "noise")
        if out is None:
            out = torch.empty((B, 2, self.n_sub, self.n_sub), device=phase.device, dtype=torch.float32)
        self._check(out, (B, 2, self.n_sub, self.n_sub), "out")
        st = load().fwr_fried_slopes(self._h, ctypes.c_void_p(phase.data_ptr()),
                                     ctypes.c_void_p(noise.data_ptr() if noise is not None else 0),
                                     ctypes.c_void_p(out.data_ptr()), B)
        if st != FWR_OK:
            raise FwrError(st, "fwr_fried_slopes")
        return out

    def generate(self, B: int, seed: int, first_frame: int = 0, r0: float = 0.15, L0: float = 25.0,
                 sigma: float = 0.05, counter=None, slopes=None, phase=None, with_phase: bool = False):
        """Synthetic frames on the device (fwr_generate): returns (slopes [B, 2, n, n], phase or None).

        `counter`: optional int64 CUDA tensor of one element, the device frame counter."""
        import torch
        n = self.n_sub
        if slopes is None:
            slopes = torch.empty((B, 2, n, n), device="cuda", dtype=torch.float32)
        self._check(slopes, (B, 2, n, n), "slopes")
        if phase is None and with_phase:
            phase = torch.empty((B, n + 1, n + 1), device="cuda", dtype=torch.float32)
        if phase is not None:
            self._check(phase, (B, n + 1, n + 1), "phase")
        cp = 0
        if counter is not None:
            if not (isinstance(counter, torch.Tensor) and counter.is_cuda and counter.dtype == torch.int64
                    and counter.numel() == 1):
                raise TypeError("counter must be a one-element int64 CUDA tensor")
            cp = counter.data_ptr()
        st = fwr_generate(self._h, seed, first_frame, cp, r0, L0, sigma, slopes.data_ptr(),
                          phase.data_ptr() if phase is not None else 0, B)
        if st != FWR_OK:
            raise FwrError(st, "fwr_generate")
        return slopes, phase

    def set_group(self, frames_per_group: int):
        """Frames per workgroup of the on-chip kernel (fwr_plan_set_group)."""
        st = load().fwr_plan_set_group(self._h, int(frames_per_group))
        if st != FWR_OK:
            raise FwrError(st, "fwr_plan_set_group")

    def set_schedule(self, schedule: int):
        """Radix schedule of the in-lane DFTs, or the multi-pass loop's launch shape (0, 1, 2;
        fwr_plan_set_schedule)."""
        st = load().fwr_plan_set_schedule(self._h, int(schedule))
        if st != FWR_OK:
            raise FwrError(st, "fwr_plan_set_schedule")

    def set_wait_limit(self, polls: int):
        """Watchdog of the persistent multi-pass loop, in polls (fwr_plan_set_wait_limit)."""
        st = load().fwr_plan_set_wait_limit(self._h, int(polls))
        if st != FWR_OK:
            raise FwrError(st, "fwr_plan_set_wait_limit")

    @property
    def schedule(self) -> int:
        v = ctypes.c_int32()
        st = load().fwr_plan_get_schedule(self._h, ctypes.byref(v))
        if st != FWR_OK:
            raise FwrError(st, "fwr_plan_get_schedule")
        return int(v.value)

    def autotune(self, B: Optional[int] = None) -> int:
        """Time every launch shape and radix schedule on B frames, keep the fastest; returns frames per
        workgroup (the schedule: `schedule`)."""
        out = ctypes.c_int32()
        st = load().fwr_plan_autotune(self._h, int(B or self.max_batch), ctypes.byref(out))
        if st != FWR_OK:
            raise FwrError(st, "fwr_plan_autotune")
        return out.value

    def set_stream(self, stream: Optional[int] = None):
        """Rebind the plan to `stream` (default: torch's current stream), e.g. a capture stream."""
        self.stream = _current_stream() if stream is None else int(stream)
        st = fwr_set_stream(self._h, self.stream)
        if st != FWR_OK:
            raise FwrError(st, "fwr_set_stream")

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            fwr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct_group(work, stream: Optional[int] = None):
    """Several (plan, slopes, out, start, resid) items in one fwr_reconstruct_group call.

    `work`: sequence of tuples (Plan, slopes, out, start or None, resid or None); tensors as
    Plan.reconstruct.  Items run concurrently; the call is ordered on `stream` (default: torch's
    current stream)."""
    items = []
    for plan, slopes, out, start, resid in work:
        B = slopes.shape[0]
        plan._check(slopes, (B, 2, plan.n_sub, plan.n_sub), "slopes")
        plan._check(out, (B, plan.n_sub + 1, plan.n_sub + 1), "out")
        sp, rp = plan._start_args(start, resid, B)
        items.append((plan.handle, slopes.data_ptr(), out.data_ptr(), sp, rp, B))
    st = fwr_reconstruct_group(items, _current_stream() if stream is None else int(stream))
    if st != FWR_OK:
        raise FwrError(st, "fwr_reconstruct_group")


class CNN:
    """Learned initial extension (fwr_cnn_* calls).  Parameters are a flat float32 array of
    47714 values: per layer, weights [out][in][3][3] then biases [out]."""

    def __init__(self, n_sub: int, n_grid: int, mask, max_batch: int, input_scale: float = 0.5,
                 training: bool = False, stream: Optional[int] = None):
        mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        self.n_sub, self.n_grid, self.max_batch = int(n_sub), int(n_grid), int(max_batch)
        self.stream = _current_stream() if stream is None else int(stream)
        h = ctypes.c_void_p()
        st = load().fwr_cnn_create(self.n_sub, self.n_grid, mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   self.max_batch, float(input_scale), int(bool(training)), self.stream,
                                   ctypes.byref(h))
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_create")
        self._h = h

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        st = load().fwr_cnn_set_params(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size)
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_set_params")

    def _get(self, fn, what):
        a = np.empty(CNN_PARAMS, dtype=np.float32)
        st = fn(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size)
        if st != FWR_OK:
            raise FwrError(st, what)
        return a

    def get_params(self) -> np.ndarray:
        return self._get(load().fwr_cnn_get_params, "fwr_cnn_get_params")

    def get_grads(self) -> np.ndarray:
        return self._get(load().fwr_cnn_get_grads, "fwr_cnn_get_grads")

    def forward(self, slopes, pred=None):
        import torch
        B = slopes.shape[0]
        if pred is None:
            pred = torch.empty((B, 2, self.n_grid, self.n_grid), device=slopes.device, dtype=torch.float32)
        st = load().fwr_cnn_forward(self._h, slopes.data_ptr(), pred.data_ptr(), B)
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_forward")
        return pred

    def backward(self, pred, target) -> float:
        loss = ctypes.c_float()
        st = load().fwr_cnn_backward(self._h, pred.data_ptr(), target.data_ptr(), pred.shape[0],
                                     ctypes.byref(loss))
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_backward")
        return float(loss.value)

    def loss_grad(self, pred, target, grad=None) -> tuple:
        """fwr_cnn_loss_grad: (loss, dloss/dpred) of the masked MSE for any prediction-shaped map."""
        import torch
        if grad is None:
            grad = torch.empty_like(pred)
        loss = ctypes.c_float()
        st = load().fwr_cnn_loss_grad(self._h, pred.data_ptr(), target.data_ptr(), grad.data_ptr(), pred.shape[0],
                                      ctypes.byref(loss))
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_loss_grad")
        return float(loss.value), grad

    def backward_grad(self, grad):
        """fwr_cnn_backward_grad: parameter gradients from dloss/dpred (after forward on the same batch)."""
        st = load().fwr_cnn_backward_grad(self._h, grad.data_ptr(), grad.shape[0])
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_backward_grad")

    def set_stream(self, stream: Optional[int] = None):
        """Rebind to `stream` (default: torch's current stream), e.g. a capture stream."""
        self.stream = _current_stream() if stream is None else int(stream)
        st = load().fwr_cnn_set_stream(self._h, ctypes.c_void_p(self.stream))
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_set_stream")

    def adam_step(self, lr: float):
        st = load().fwr_cnn_adam_step(self._h, float(lr))
        if st != FWR_OK:
            raise FwrError(st, "fwr_cnn_adam_step")

    def close(self):
        if getattr(self, "_h", None):
            load().fwr_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params_to_flat(params) -> np.ndarray:
    """[(w [O][C][3][3], b [O]), ...] -> flat float32 array in the library's layout."""
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params]).astype(np.float32)


def flat_to_params(flat: np.ndarray, layers):
    out, i = [], 0
    for cin, cout in layers:
        nw = cout * cin * 9
        w = flat[i:i + nw].reshape(cout, cin, 3, 3)
        i += nw
        b = flat[i:i + cout]
        i += cout
        out.append((w.astype(np.float64), b.astype(np.float64)))
    return out
