"""Learned initial extension: training, the learned-start reconstruction with fallback, evaluation.

    python -m paper_1705_04298_amd.learned train --frames 200000 --epochs 3 --out weights.npz
    python -m paper_1705_04298_amd.learned evaluate --weights weights.npz

Everything numeric runs in libfwr (HIP): the CNN forward/backward/Adam kernels
train the network; targets are the plain Gerchberg loop at 50 iterations
(`fwr_extend`, no Eq. 5), i.e. the converged out-of-pupil extension the
network should predict; the reconstruction then starts Algorithm 1 from the
network's prediction (`fwr_reconstruct_start`).  A frame whose in-pupil
residual after the learned start exceeds `threshold` is recomputed from the
zero-padded start with the plain iteration count (the fallback).
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import fwr
from . import inputs as I

N_SUB, N_GRID, D = 40, 80, 0.2
LAYERS = ((3, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 2))
INPUT_SCALE = 0.5


def he_init(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, flattened in the library's parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in LAYERS:
        parts.append(rng.standard_normal(cout * cin * 9) * np.sqrt(2.0 / (cin * 9)))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def _gen_chunk(args):
    count, seed = args
    s, p, _, _ = I.training_frames(count, seed=seed)
    return s, p


def make_frames(count: int, seed0: int, workers: int = 1, chunk: int = 4096):
    jobs = [(min(chunk, count - i), seed0 + k) for k, i in enumerate(range(0, count, chunk))]
    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_gen_chunk, jobs)
    else:
        parts = [_gen_chunk(j) for j in jobs]
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def targets(slopes_dev, chunk: int = 4096, n_iter: int = 50):
    """Converged extension (plain loop, no Eq. 5) of every frame, on the device."""
    import torch
    B = slopes_dev.shape[0]
    plan = fwr.Plan(N_SUB, N_GRID, I.pupil_mask(N_SUB), n_iter=n_iter, periodic=False,
                    max_batch=min(chunk, B))
    out = torch.empty((B, 2, N_GRID, N_GRID), device=slopes_dev.device, dtype=torch.float32)
    for i in range(0, B, chunk):
        plan.extend(slopes_dev[i:i + chunk], out[i:i + chunk])
    torch.cuda.synchronize()
    plan.close()
    return out


def train(frames: int, epochs: int, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          workers: int = 1, log=print, init: np.ndarray | None = None, loop_iters: int = 0):
    """Train the network on `frames` generated frames; returns (params, history).

    loop_iters = 0: loss on the network's prediction itself (out-of-pupil MSE against the
    50-iteration extension).  loop_iters = k > 0: loss on the extension after k iterations of
    Algorithm 1 started from the prediction, i.e. on what the loop makes of the start; its
    gradient with respect to the prediction is the same k-iteration loop run with zero
    measurements on the loss gradient (the loop's out-of-pupil map is symmetric), so the
    network learns the components the loop itself converges slowly on."""
    import torch
    t0 = time.perf_counter()
    slopes, _ = make_frames(frames, seed0=1000 * (seed + 1), workers=workers)
    log(f"[learned] generated {frames} training frames in {time.perf_counter() - t0:.1f} s")
    x = torch.from_numpy(slopes).cuda()
    t0 = time.perf_counter()
    y = targets(x)
    log(f"[learned] targets (plain loop, 50 iterations) in {time.perf_counter() - t0:.2f} s")
    net = fwr.CNN(N_SUB, N_GRID, I.pupil_mask(N_SUB), max_batch=batch, input_scale=INPUT_SCALE, training=True)
    net.set_params(he_init(seed) if init is None else init)
    rng = np.random.default_rng(seed)
    hist = []
    pred = torch.empty((batch, 2, N_GRID, N_GRID), device="cuda", dtype=torch.float32)
    steps_per_epoch = frames // batch
    if loop_iters:
        loop = fwr.Plan(N_SUB, N_GRID, I.pupil_mask(N_SUB), n_iter=loop_iters, periodic=False, max_batch=batch)
        zeros = torch.zeros((batch, 2, N_SUB, N_SUB), device="cuda", dtype=torch.float32)
        ext, gext, gstart = (torch.empty_like(pred) for _ in range(3))
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(frames)).cuda()
        t1 = time.perf_counter()
        tot = 0.0
        for st in range(steps_per_epoch):
            idx = perm[st * batch:(st + 1) * batch]
            xb = x.index_select(0, idx).contiguous()
            yb = y.index_select(0, idx).contiguous()
            net.forward(xb, pred)
            if loop_iters:
                loop.extend(xb, ext, start=pred)           # k iterations from the network's start
                loss, _ = net.loss_grad(ext, yb, gext)      # d loss / d extension
                loop.extend(zeros, gstart, start=gext)      # the loop's adjoint: same loop, no data
                net.backward_grad(gstart)
            else:
                loss = net.backward(pred, yb)
            step_lr = lr * (0.5 ** ep)
            net.adam_step(step_lr)
            tot += loss
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        hist.append({"epoch": ep, "mean_loss": tot / steps_per_epoch, "seconds": dt,
                     "frames_per_s": steps_per_epoch * batch / dt})
        log(f"[learned] epoch {ep} loss {tot / steps_per_epoch:.5f} ({dt:.1f} s, "
            f"{steps_per_epoch * batch / dt:.0f} frames/s)")
    params = net.get_params()
    net.close()
    if loop_iters:
        loop.close()
    return params, hist


class LearnedReconstructor:
    """CNN start + `n_iter` Gerchberg iterations, with the plain-loop fallback
    (`fwr_reconstruct_learned`: one library call).

    `reconstruct(slopes)` returns (phase [B, n+1, n+1], residual [B], number of frames recomputed
    by the plain loop).
    """

    def __init__(self, params: np.ndarray, n_iter: int = 2, plain_iter: int = 10, threshold: float = 0.2,
                 max_batch: int = 4096, periodic: bool = True):
        mask = I.pupil_mask(N_SUB)
        self.net = fwr.CNN(N_SUB, N_GRID, mask, max_batch=max_batch, input_scale=INPUT_SCALE, training=False)
        self.net.set_params(params)
        self.plan = fwr.Plan(N_SUB, N_GRID, mask, n_iter=n_iter, periodic=periodic, max_batch=max_batch)
        self.plain = fwr.Plan(N_SUB, N_GRID, mask, n_iter=plain_iter, periodic=periodic, max_batch=max_batch)
        self.threshold = float(threshold)
        self._start = None

    def reconstruct(self, slopes, out=None):
        import ctypes
        import torch
        B = slopes.shape[0]
        self.plan._check(slopes, (B, 2, N_SUB, N_SUB), "slopes")
        if out is None:
            out = torch.empty((B, N_SUB + 1, N_SUB + 1), device=slopes.device, dtype=torch.float32)
        self.plan._check(out, (B, N_SUB + 1, N_SUB + 1), "out")
        if self._start is None or self._start.shape[0] < B:
            self._start = torch.empty((B, 2, N_GRID, N_GRID), device=slopes.device, dtype=torch.float32)
        resid = torch.empty(B, device=slopes.device, dtype=torch.float32)
        count = ctypes.c_int32()
        st = fwr.fwr_reconstruct_learned(self.plan.handle, self.plain.handle, self.net._h, slopes.data_ptr(),
                                         self._start.data_ptr(), out.data_ptr(), resid.data_ptr(), self.threshold,
                                         B, ctypes.byref(count))
        if st != fwr.FWR_OK:
            raise fwr.FwrError(st, "fwr_reconstruct_learned")
        return out, resid, int(count.value)

    def close(self):
        self.net.close()
        self.plan.close()
        self.plain.close()


def _pupil_nodes():
    return I.pupil_nodes(I.pupil_mask(N_SUB))


def evaluate(params: np.ndarray, frames: int = 4096, seed: int = 99, log=print, steps: int = 20):
    """CNN + k iterations vs the plain loop on held-out frames: residual, error vs truth, frames/s."""
    import torch
    slopes, truth = make_frames(frames, seed0=10_000 + seed)
    x = torch.from_numpy(slopes).cuda()
    mask = I.pupil_mask(N_SUB)
    nodes = _pupil_nodes()

    def err_vs_truth(phase):
        e = (phase - truth)[:, nodes]
        e = e - e.mean(axis=1, keepdims=True)
        return np.sqrt(np.mean(e * e, axis=1))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    res = {"frames": frames}
    net = fwr.CNN(N_SUB, N_GRID, mask, max_batch=frames, input_scale=INPUT_SCALE, training=False)
    net.set_params(params)
    start = net.forward(x)
    for k in (1, 2, 3, 10):
        plan = fwr.Plan(N_SUB, N_GRID, mask, n_iter=k, periodic=True, max_batch=frames)
        for label, st in (("plain", None), ("cnn", start)):
            resid = torch.empty(frames, device="cuda")
            ph = plan.reconstruct(x, start=st, resid=resid)
            torch.cuda.synchronize()
            r = resid.cpu().numpy()
            e = err_vs_truth(ph.cpu().numpy())
            if st is None:
                ms = timed(lambda: plan.reconstruct(x))
            else:
                ms = timed(lambda: (net.forward(x, start), plan.reconstruct(x, start=start)))
            res[f"{label}_{k}"] = {"median_residual": float(np.median(r)), "mean_residual": float(np.mean(r)),
                                   "median_err_rad": float(np.median(e)), "ms_per_batch": ms,
                                   "frames_per_s": frames / ms * 1e3}
            log(f"[learned] {label} + {k} it: residual {np.median(r):.4f}, err {np.median(e):.4f} rad, "
                f"{frames / ms * 1e3:.0f} frames/s")
        plan.close()
    ms_cnn = timed(lambda: net.forward(x, start))
    res["cnn_forward_ms"] = ms_cnn
    flops = frames * 2.0 * N_GRID * N_GRID * sum(9 * cin * cout for cin, cout in LAYERS)
    res["cnn_forward_tflops"] = flops / (ms_cnn / 1e3) / 1e12
    target = res["plain_10"]["median_residual"]
    res["iterations_to_match_plain10"] = next((k for k in (1, 2, 3, 10)
                                              if res[f"cnn_{k}"]["median_residual"] <= target), None)
    # fallback rate of the default learned reconstructor (CNN + 2 iterations, threshold 2x plain-10 level)
    lr = LearnedReconstructor(params, n_iter=2, plain_iter=10, threshold=2.0 * target, max_batch=frames)
    _, resid, nfall = lr.reconstruct(x)
    ms_lr = timed(lambda: lr.reconstruct(x))  # network, 2 iterations, fallback (one host sync per call)
    res["fallback"] = {"threshold": 2.0 * target, "rate": nfall / frames, "ms_per_batch": ms_lr,
                       "frames_per_s": frames / ms_lr * 1e3}
    log(f"[learned] cnn + 2 it + fallback (threshold {2.0 * target:.4f}): {100 * nfall / frames:.1f} % "
        f"recomputed, {frames / ms_lr * 1e3:.0f} frames/s")
    lr.close()
    net.close()
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--frames", type=int, default=200_000)
    t.add_argument("--epochs", type=int, default=3)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--workers", type=int, default=0)
    t.add_argument("--out", required=True)
    t.add_argument("--loop-iters", type=int, default=0,
                   help="loss on the extension after this many loop iterations from the network's start")
    t.add_argument("--init", default=None, help="start from these weights (.npz) instead of He-normal")
    t.add_argument("--evaluate", action="store_true")
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", required=True)
    e.add_argument("--frames", type=int, default=4096)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.cmd == "train":
        workers = args.workers or max(1, min(16, len(os.sched_getaffinity(0))))
        init = np.load(args.init)["params"] if args.init else None
        params, hist = train(args.frames, args.epochs, args.batch, args.lr, workers=workers, log=log,
                             init=init, loop_iters=args.loop_iters)
        np.savez(args.out, params=params, history=json.dumps(hist))
        result = {"history": hist}
        if args.evaluate:
            result["evaluation"] = evaluate(params, log=log)
        print(json.dumps(result), flush=True)
    else:
        params = np.load(args.weights)["params"]
        print(json.dumps(evaluate(params, frames=args.frames, log=log)), flush=True)


if __name__ == "__main__":
    main()
