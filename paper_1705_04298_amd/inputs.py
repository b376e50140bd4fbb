"""Seeded synthetic Shack-Hartmann workloads.

This module simulates the *measurement*, never the reconstruction: it draws
von Karman phase screens, samples Fried-geometry slopes from them and adds
white measurement noise.  Both the HIP path and the FP64 oracle are fed from
here; neither of them is imported by this module and it holds no step of the
reconstruction method (no filter, no transform of the slopes, no iteration).

Workload shapes follow the paper's SPHERE-like system (Table 1: r0 = 15 cm,
D = 8 m, 40x40 lenslets, V-band sensing) and the ELT-scale motivation of
Sec. 1 / Sec. 3.3 (Eq. 8).  The outer scale is 25 m for the synthetic
workloads (the paper's Table 1 quotes 30 m; see the design notes).

Random numbers: frame ``i`` of workload ``c`` is drawn from
``numpy.random.default_rng([170504298, c, i])``: the screen first, then the
noise.  Every array this module returns is float64 unless stated.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

try:  # multi-threaded FFTs make screen synthesis ~8x faster; numpy is the fallback
    import scipy.fft as _sfft

    def _ifft2(a: np.ndarray) -> np.ndarray:
        return _sfft.ifft2(a, workers=-1)
except Exception:  # pragma: no cover - scipy is present in this image
    def _ifft2(a: np.ndarray) -> np.ndarray:
        return np.fft.ifft2(a)

SEED_BASE = 170504298

# Kolmogorov/von Karman PSD prefactor [24/5 Gamma(6/5)]^(5/6) Gamma(11/6)^2 / (2 pi^(11/3)),
# written out so that this module does not depend on the oracle.
_VK_CONST = (
    (24.0 / 5.0 * math.gamma(6.0 / 5.0)) ** (5.0 / 6.0)
    * math.gamma(11.0 / 6.0) ** 2
    / (2.0 * math.pi ** (11.0 / 3.0))
)


def pupil_mask(n: int, supersample: int = 16, obstruction_pct: int = 14) -> np.ndarray:
    """Valid-subaperture mask of an ``n x n`` Shack-Hartmann array.

    Circular pupil of diameter ``n`` lenslets with a central obstruction of
    ``obstruction_pct`` percent of the diameter.  A subaperture is valid when
    strictly more than half of its ``supersample**2`` sample points are lit.
    Everything is decided in integers (sample centres in half-sample units),
    so the result has no floating-point ties: 436 / 1240 / 3168 / 12636 valid
    subapertures for n = 24 / 40 / 64 / 128.

    Returns ``uint8[n, n]``, row index = y, 1 = valid.
    """
    S = int(supersample)
    a = np.arange(n * S, dtype=np.int64)
    u = 2 * a + 1 - n * S                      # sample centre, half-sample units
    U, V = np.meshgrid(u, u)                   # V varies along rows (y)
    r2 = U * U + V * V
    lit = (r2 <= (n * S) ** 2) & (10000 * r2 >= (obstruction_pct * n * S) ** 2)
    count = lit.reshape(n, S, n, S).sum(axis=(1, 3))
    return (2 * count > S * S).astype(np.uint8)


def pupil_nodes(mask: np.ndarray) -> np.ndarray:
    """Fried nodes of the valid subapertures: ``bool[n+1, n+1]``, True at every corner of a
    valid subaperture (the phase points a reconstruction is judged on)."""
    m = np.asarray(mask).astype(bool)
    n = m.shape[0]
    nodes = np.zeros((n + 1, n + 1), dtype=bool)
    for a in (0, 1):
        for b in (0, 1):
            nodes[a:a + n, b:b + n] |= m
    return nodes


def von_karman_psd(kappa2: np.ndarray, r0: float, L0: float) -> np.ndarray:
    """Von Karman phase PSD [rad^2 m^2] at squared spatial frequency ``kappa2`` [m^-2]."""
    return _VK_CONST * r0 ** (-5.0 / 3.0) * (kappa2 + 1.0 / (L0 * L0)) ** (-11.0 / 6.0)


def vk_screen(rng: np.random.Generator, M: int, d: float, r0: float, L0: float) -> np.ndarray:
    """One periodic von Karman phase screen [rad at 500 nm] on an ``M x M`` grid of spacing ``d``.

    Spectral synthesis: complex white Gaussian noise shaped by sqrt(PSD) * dkappa,
    real part of the inverse FFT scaled by M^2.  The piston term is zero.
    """
    f = np.fft.fftfreq(M, d=d)
    kx, ky = np.meshgrid(f, f)
    psd = von_karman_psd(kx * kx + ky * ky, r0, L0)
    psd[0, 0] = 0.0
    dk = 1.0 / (M * d)
    w = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    return np.real(_ifft2(w * np.sqrt(psd) * dk)) * (M * M)


def fried_slopes_from_nodes(phi: np.ndarray):
    """Noise-free Fried-geometry slopes of the ``(n+1) x (n+1)`` node phase ``phi``.

    Each subaperture measures the mean of the two phase differences across it
    (x: along columns, y: along rows), in radians.  Returns (sx, sy), each ``n x n``.
    """
    a = phi[:-1, :-1]
    b = phi[:-1, 1:]
    c = phi[1:, :-1]
    e = phi[1:, 1:]
    sx = 0.5 * ((b - a) + (e - c))
    sy = 0.5 * ((c - a) + (e - b))
    return sx, sy


def sinc_slopes_from_screen(screen: np.ndarray, n: int, delta: float = 0.0):
    """Lenslet-averaged slopes (Eq. 4: the difference of the phase averaged over opposite
    lenslet edges) of the periodic ``M x M`` screen, for the ``n x n`` lenslets whose corner
    nodes are screen samples [0, n] x [0, n].

    Computed on the screen's own grid: a screen mode exp(2 pi i (k' x + l' y) / M) (signed
    k', l') has the x measurement exp(i pi (k' + l') / M) 2i sin(pi k' / M) sinc(l' / M)
    times its value at the lenslet's first corner, y likewise; Nyquist components, whose
    measurement of a real screen is not real, are dropped.  With delta = d_px / d the edge
    averages lie (1 - delta) d apart (pixel-size correction): sin(pi k' (1 - delta) / M).
    Returns (sx, sy), each n x n.
    """
    M = screen.shape[0]
    f = np.fft.fftfreq(M) * M                  # signed integer frequencies
    fx, fy = np.meshgrid(f, f)                 # fx along columns (x), fy along rows (y)
    shift = np.exp(1j * np.pi * (fx + fy) / M)
    hx = shift * 2j * np.sin(np.pi * fx * (1.0 - delta) / M) * np.sinc(fy / M)
    hy = shift * 2j * np.sin(np.pi * fy * (1.0 - delta) / M) * np.sinc(fx / M)
    if M % 2 == 0:
        nyq = (np.abs(fx) == M // 2) | (np.abs(fy) == M // 2)
        hx[nyq] = 0.0
        hy[nyq] = 0.0
    S = np.fft.fft2(screen)
    sx = np.real(np.fft.ifft2(hx * S))[:n, :n]
    sy = np.real(np.fft.ifft2(hy * S))[:n, :n]
    return sx, sy


@dataclasses.dataclass(frozen=True)
class Workload:
    """Geometry and statistics of one synthetic workload."""

    n_sub: int            # lenslets per side
    diameter: float       # telescope diameter [m]
    r0: float = 0.15      # Fried parameter at 500 nm [m]
    L0: float = 25.0      # outer scale [m]
    noise_sigma: float = 0.05  # slope noise [rad]
    screen_size: int = 256     # M, periodic screen side in samples of pitch d
    config_id: int = 1
    model: str = "fried"       # slope measurement: "fried" (corner differences) or "sinc" (Eq. 4)
    d_px_frac: float = 0.0     # sinc model: detector pixel length / lenslet pitch (d - d_px remark)

    @property
    def d(self) -> float:
        return self.diameter / self.n_sub


# The workloads: 40x40 SPHERE-like (single frame and 4096-frame batch), the
# 128x128 ELT-scale case, and the smaller/larger sizes of the uneven mix.
SPHERE_40 = Workload(n_sub=40, diameter=8.0, screen_size=256, config_id=1)
SPHERE_40_BATCH = dataclasses.replace(SPHERE_40, config_id=2)
ELT_128 = Workload(n_sub=128, diameter=39.0, screen_size=512, config_id=3)
MIX_24 = Workload(n_sub=24, diameter=8.0, screen_size=256, config_id=5)
MIX_64 = Workload(n_sub=64, diameter=8.0, screen_size=256, config_id=5)
SPHERE_40_SINC = Workload(n_sub=40, diameter=8.0, screen_size=256, config_id=6, model="sinc")


def frame_rng(config_id: int, index: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(config_id), int(index)])


def make_frame(w: Workload, index: int, noise_sigma: Optional[float] = None,
               r0: Optional[float] = None):
    """Frame ``index`` of workload ``w``.

    Returns ``(slopes, phase)``: ``slopes`` is ``float64[2, n, n]`` (x then y,
    row = y) with zeros on invalid subapertures; ``phase`` is the true
    ``(n+1) x (n+1)`` node phase the slopes were sampled from (before noise).
    """
    rng = frame_rng(w.config_id, index)
    n = w.n_sub
    r0v = w.r0 if r0 is None else r0
    sig = w.noise_sigma if noise_sigma is None else noise_sigma
    scr = vk_screen(rng, w.screen_size, w.d, r0v, w.L0)
    phi = scr[: n + 1, : n + 1].copy()
    if w.model == "sinc":
        sx, sy = sinc_slopes_from_screen(scr, n, w.d_px_frac)
    else:
        sx, sy = fried_slopes_from_nodes(phi)
    noise = rng.standard_normal((2, n, n)) * sig
    m = pupil_mask(n).astype(bool)
    out = np.zeros((2, n, n))
    out[0] = np.where(m, sx + noise[0], 0.0)
    out[1] = np.where(m, sy + noise[1], 0.0)
    return out, phi


def make_batch(w: Workload, count: int, start: int = 0, dtype=np.float32) -> np.ndarray:
    """``count`` consecutive frames as one ``[count, 2, n, n]`` array (C order)."""
    out = np.empty((count, 2, w.n_sub, w.n_sub), dtype=dtype)
    for i in range(count):
        out[i] = make_frame(w, start + i)[0]
    return out


def random_mask(n: int, seed: int, keep: float = 0.6) -> np.ndarray:
    """Arbitrary (non-circular) ``uint8`` mask for edge-case tests."""
    rng = np.random.default_rng([SEED_BASE, 99, seed])
    return (rng.random((n, n)) < keep).astype(np.uint8)


def random_slopes(B: int, n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """White ``float64[B, 2, n, n]`` slopes for small-grid tests (not turbulence-like)."""
    rng = np.random.default_rng([SEED_BASE, 98, seed])
    return rng.standard_normal((B, 2, n, n)) * scale


# ---------------------------------------------------------------------------
# Training frames for the learned initial extension
# ---------------------------------------------------------------------------

LEARNED_SCREEN = 1024   # one screen gives (1024 // 41)^2 = 576 disjoint 41x41 node windows
LEARNED_CONFIG = 4


def training_frames(count: int, n: int = 40, diameter: float = 8.0, seed: int = 0,
                    r0_range=(0.08, 0.20), sigma_range=(0.0, 0.1), L0: float = 25.0):
    """``count`` frames with per-frame r0 ~ U(r0_range) and noise sigma ~ U(sigma_range).

    Phases are disjoint (n+1) x (n+1) windows of large periodic von Karman screens
    drawn at r0 = 0.15 m and rescaled by (0.15 / r0)^(5/6) (the PSD scales as
    r0^(-5/3)).  Returns ``(slopes float32[count, 2, n, n], phase float32[count, n+1, n+1],
    r0 float64[count], sigma float64[count])``; slopes are zero on invalid subapertures.
    """
    d = diameter / n
    per = (LEARNED_SCREEN // (n + 1)) ** 2
    m = pupil_mask(n).astype(bool)
    slopes = np.zeros((count, 2, n, n), dtype=np.float32)
    phase = np.zeros((count, n + 1, n + 1), dtype=np.float32)
    rng = np.random.default_rng([SEED_BASE, LEARNED_CONFIG, seed])
    r0 = rng.uniform(*r0_range, count)
    sig = rng.uniform(*sigma_range, count)
    side = LEARNED_SCREEN // (n + 1)
    i = 0
    s = 0
    while i < count:
        scr = vk_screen(frame_rng(LEARNED_CONFIG, 1_000_000 * (seed + 1) + s), LEARNED_SCREEN, d, 0.15, L0)
        s += 1
        for w in range(per):
            if i >= count:
                break
            a, b = divmod(w, side)
            phi = scr[a * (n + 1):(a + 1) * (n + 1), b * (n + 1):(b + 1) * (n + 1)] * (0.15 / r0[i]) ** (5.0 / 6.0)
            sx, sy = fried_slopes_from_nodes(phi)
            noise = rng.standard_normal((2, n, n)) * sig[i]
            slopes[i, 0] = np.where(m, sx + noise[0], 0.0)
            slopes[i, 1] = np.where(m, sy + noise[1], 0.0)
            phase[i] = phi
            i += 1
    return slopes, phase, r0, sig
