"""FP64 CPU oracle for the modified-Gerchberg slope extension and Fourier reconstruction.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the CPU-baseline leg of the benchmark may import or call this module.  The
product path (the HIP library and its Python binding) never does, and shares
no code, table or constant with it.

What it computes (Bond et al., "Iterative wave-front reconstruction in the
Fourier domain"):

* Sec. 2, Eq. 1 -- slopes are a linear filter G of the phase plus noise.  The
  discrete model used here is the Fried geometry: a subaperture measures the
  mean of the two phase differences across its four corner nodes.
* Sec. 2, Eq. 2 -- phase estimate = R_x S_x + R_y S_y, then inverse transform.
* Sec. 2, Eq. 3 -- Wiener filter R = G* / (|G|^2 + gamma W_eta / W_phi);
  gamma = 0 is least squares (used inside the loop, Sec. 3.3), gamma = 1 the
  MMSE filter (used for the final reconstruction, Sec. 3.3).
* Sec. 3.2, Eq. 5 -- periodicity: the last column of s_x is minus the sum of
  the rest of its row, the last row of s_y minus the sum of the rest of its
  column.
* Sec. 3.3, Algorithm 1 -- for each iteration: (1) transform both slope maps,
  (2) reconstruct the phase with the LSQ filter and re-derive slopes with G,
  (3) inverse transform, (4) put the measured slopes back inside the pupil.
  After the loop, (5) optionally enforce Eq. 5.
* Sec. 4.1 -- zero iterations means the measurement padded with zeros.

Readings where the paper is silent (each listed in the design notes):
  * G is the Fried model (the paper's own filter is only referenced), or the
    lenslet-averaging (sinc) model of Eq. 4 read on the DFT grid (`sinc_model`);
  * the pupil sits centred in the padded grid, offset (N - n) / 2;
  * out-of-pupil start values are zero;
  * Eq. 5 is applied once, after the loop (optionally after every iteration);
    the "N-th" column / row of Eq. 5 is index N-1 of the padded grid;
  * 0/0 in the filters: the frequencies where |G| = 0 by construction (DC and,
    for even N, the (N/2, N/2) waffle frequency) are set to zero by index;
  * W_eta / W_phi = sigma^2 d^2 / Phi_vK(kappa) in DFT units;
  * the real part is taken after every inverse transform.

DFT convention: X[l, k] = sum_{m, n} x[m, n] exp(-2 pi i (l m + k n) / N); the
row index m and frequency l are y, the column index n and frequency k are x.
The inverse carries 1 / N^2.  numpy.fft.fft2 / ifft2 are used as the
transform primitive (pinned against a brute-force matrix DFT in the tests).
"""
from __future__ import annotations

import math
from typing import NamedTuple, Optional

import numpy as np


# ---------------------------------------------------------------------------
# Transforms (library primitive)
# ---------------------------------------------------------------------------

def dft2(x: np.ndarray) -> np.ndarray:
    """Forward 2-D DFT with the convention above (Algorithm 1 step 1, "TF")."""
    return np.fft.fft2(np.asarray(x, dtype=np.float64))


def idft2(X: np.ndarray) -> np.ndarray:
    """Inverse 2-D DFT, 1/N^2 normalisation (Algorithm 1 step 3, "TF^-1")."""
    return np.fft.ifft2(X)


# ---------------------------------------------------------------------------
# Measurement model and filters (Sec. 2)
# ---------------------------------------------------------------------------

def frequency_indices(N: int):
    """Integer frequency grids (l, k) with l along rows (y) and k along columns (x)."""
    idx = np.arange(N)
    k, l = np.meshgrid(idx, idx)
    return l, k


def fried_model(N: int):
    """Fourier transfer functions G_x, G_y of the Fried slope model (Eq. 1 / Eq. 4 reading).

    s_x[m, n] = (phi[m, n+1] - phi[m, n] + phi[m+1, n+1] - phi[m+1, n]) / 2 and
    s_y[m, n] = (phi[m+1, n] - phi[m, n] + phi[m+1, n+1] - phi[m, n+1]) / 2 on the
    periodic N x N grid give, with theta_k = 2 pi k / N,
        G_x = (e^{i theta_k} - 1)(1 + e^{i theta_l}) / 2,
        G_y = (e^{i theta_l} - 1)(1 + e^{i theta_k}) / 2.
    """
    l, k = frequency_indices(N)
    ek = np.exp(2j * np.pi * k / N)
    el = np.exp(2j * np.pi * l / N)
    Gx = 0.5 * (ek - 1.0) * (1.0 + el)
    Gy = 0.5 * (el - 1.0) * (1.0 + ek)
    return Gx, Gy


def sinc_model(N: int, delta: float = 0.0):
    """Fourier transfer functions of the lenslet-averaging model of Eq. 4 (sinc reading).

    A subaperture measures the difference of the phase averaged over its two opposite
    edges (Sec. 2, Eq. 4: comb sampling x (box average convolved with the gradient)).
    For a grid mode exp(2 pi i (k' n + l' m) / N) of the node phase, interpolated as the
    same continuous mode, the x measurement of cell (m, n) is the node value times
        G_x = exp(i pi (k' + l') / N) 2i sin(pi k' / N) sinc(l' / N),
    sinc(u) = sin(pi u) / (pi u), with signed frequencies k', l' in [-N/2, N/2); G_y swaps
    the roles of k' and l'.  The slopes of a real phase must be real, so the transfer
    function is the Hermitian part of this expression on the DFT grid; it equals the
    expression off the Nyquist lines and vanishes on them (even N), where the expression is
    anti-Hermitian.

    Pixel-size correction (the remark after Eq. 4: the difference is effectively taken over
    d - d_px): with delta = d_px / d the two edge averages lie (1 - delta) d apart, centred on
    the lenslet, each still averaged over the full edge length d, and the measurement stays a
    phase difference in radians:
        G_x = exp(i pi (k' + l') / N) 2i sin(pi k' (1 - delta) / N) sinc(l' / N).
    """
    l, k = frequency_indices(N)
    ks = np.where(k < (N + 1) // 2, k, k - N).astype(np.float64)
    ls = np.where(l < (N + 1) // 2, l, l - N).astype(np.float64)
    shift = np.exp(1j * np.pi * (ks + ls) / N)
    Gx = shift * 2j * np.sin(np.pi * ks * (1.0 - delta) / N) * np.sinc(ls / N)
    Gy = shift * 2j * np.sin(np.pi * ls * (1.0 - delta) / N) * np.sinc(ks / N)
    if N % 2 == 0:
        nyq = (l == N // 2) | (k == N // 2)
        Gx = np.where(nyq, 0.0, Gx)
        Gy = np.where(nyq, 0.0, Gy)
    return Gx, Gy


def sinc_singular_set(N: int) -> np.ndarray:
    """Where the sinc model's |G|^2 vanishes, by index: (0, 0) and, for even N, the Nyquist
    row and column."""
    S = np.zeros((N, N), dtype=bool)
    S[0, 0] = True
    if N % 2 == 0:
        S[N // 2, :] = True
        S[:, N // 2] = True
    return S


def slope_model(name: str, N: int, delta: float = 0.0):
    """(G_x, G_y, singular set) of the named model: "fried" or "sinc" (delta = d_px / d)."""
    if name == "fried":
        if delta != 0.0:
            raise ValueError("the pixel-size correction belongs to the lenslet-averaging model")
        Gx, Gy = fried_model(N)
        return Gx, Gy, singular_set(N)
    if name == "sinc":
        Gx, Gy = sinc_model(N, delta)
        return Gx, Gy, sinc_singular_set(N)
    raise ValueError(f"unknown slope model {name!r}")


def singular_set(N: int) -> np.ndarray:
    """Boolean N x N map of the frequencies where |G|^2 vanishes for the Fried model.

    Decided by index, never by value: (0, 0) always, and (N/2, N/2) when N is even.
    """
    S = np.zeros((N, N), dtype=bool)
    S[0, 0] = True
    if N % 2 == 0:
        S[N // 2, N // 2] = True
    return S


def wiener_reconstructor(Gx: np.ndarray, Gy: np.ndarray, gamma: float = 0.0,
                         ratio: Optional[np.ndarray] = None, singular: Optional[np.ndarray] = None):
    """Eq. 3: R_{x,y} = G*_{x,y} / (|G_x|^2 + |G_y|^2 + gamma W_eta/W_phi).

    ``ratio`` is W_eta / W_phi on the DFT grid (ignored when gamma == 0).
    Where the denominator is zero by construction (the singular set of the model,
    ``singular``, default the Fried one, with no regularisation) the filter is zero.
    """
    N = Gx.shape[0]
    den = np.abs(Gx) ** 2 + np.abs(Gy) ** 2
    if gamma != 0.0:
        if ratio is None:
            raise ValueError("gamma != 0 needs the noise-to-signal ratio")
        den = den + gamma * ratio
        zero = den == 0.0
    else:
        zero = singular_set(N) if singular is None else singular
    safe = np.where(zero, 1.0, den)
    Rx = np.where(zero, 0.0, np.conj(Gx) / safe)
    Ry = np.where(zero, 0.0, np.conj(Gy) / safe)
    return Rx, Ry


def von_karman_psd(kappa2: np.ndarray, r0: float, L0: float) -> np.ndarray:
    """Von Karman phase PSD [rad^2 m^2]: c r0^(-5/3) (kappa^2 + L0^-2)^(-11/6).

    c = [24/5 Gamma(6/5)]^(5/6) Gamma(11/6)^2 / (2 pi^(11/3)) ~= 0.022896
    (textbook turbulence constant; the paper gives r0 and L0 in Table 1).
    """
    c = ((24.0 / 5.0) * math.gamma(1.2)) ** (5.0 / 6.0) * math.gamma(11.0 / 6.0) ** 2 \
        / (2.0 * math.pi ** (11.0 / 3.0))
    return c * r0 ** (-5.0 / 3.0) * (kappa2 + L0 ** -2) ** (-11.0 / 6.0)


def noise_to_signal(N: int, d: float, r0: float, L0: float, noise_var: float) -> np.ndarray:
    """W_eta / W_phi of Eq. 3 on the N x N DFT grid.

    White slope noise of variance sigma^2 has DFT power N^2 sigma^2; a phase of
    PSD Phi sampled at pitch d has DFT power N^2 Phi / d^2.  Their ratio is
    sigma^2 d^2 / Phi(kappa), with kappa = (k', l') / (N d) for the signed
    frequency indices k', l' in [-N/2, N/2).
    """
    f = np.fft.fftfreq(N, d=d)          # signed k' / (N d)
    kx, ky = np.meshgrid(f, f)
    return noise_var * d * d / von_karman_psd(kx * kx + ky * ky, r0, L0)


# ---------------------------------------------------------------------------
# Geometry (Algorithm 1 input; Sec. 4 extension window)
# ---------------------------------------------------------------------------

def pupil_offset(n: int, N: int) -> int:
    if N <= n or (N - n) % 2:
        raise ValueError("padded grid must exceed the lenslet array by an even count")
    return (N - n) // 2


def pupil_on_grid(mask: np.ndarray, N: int) -> np.ndarray:
    """P: the valid-subaperture indicator placed centred on the N x N grid."""
    n = mask.shape[0]
    o = pupil_offset(n, N)
    P = np.zeros((N, N), dtype=bool)
    P[o:o + n, o:o + n] = np.asarray(mask).astype(bool)
    return P


def padded_measurement(slopes: np.ndarray, mask: np.ndarray, N: int):
    """s^0_x, s^0_y: measured slopes inside the pupil, zeros elsewhere (Sec. 4.1)."""
    n = mask.shape[0]
    o = pupil_offset(n, N)
    P = pupil_on_grid(mask, N)
    s0x = np.zeros((N, N))
    s0y = np.zeros((N, N))
    s0x[o:o + n, o:o + n] = slopes[0]
    s0y[o:o + n, o:o + n] = slopes[1]
    s0x[~P] = 0.0
    s0y[~P] = 0.0
    return s0x, s0y, P


# ---------------------------------------------------------------------------
# Algorithm 1 and Eq. 5
# ---------------------------------------------------------------------------

def enforce_periodicity(sx: np.ndarray, sy: np.ndarray):
    """Eq. 5: s_x(m, N) = -sum_{n<N} s_x(m, n);  s_y(N, n) = -sum_{m<N} s_y(m, n)."""
    sx = sx.copy()
    sy = sy.copy()
    sx[:, -1] = -np.sum(sx[:, :-1], axis=1)
    sy[-1, :] = -np.sum(sy[:-1, :], axis=0)
    return sx, sy


def hudgin_extend(s0x: np.ndarray, s0y: np.ndarray, P: np.ndarray):
    """The comparison extension of Sec. 3.2 ("Hudgin extension"): the x slopes are extended up
    and down each column and the y slopes left and right along each row by repeating the slope
    at the edge of the pupil; then Eq. 5 is imposed (the paper always does with this method).

    Reading where the paper is silent (central obstruction): every cell outside the pupil takes
    the slope of the nearest in-pupil cell of its column (x) or row (y), the one above or to the
    left on a tie; a line without in-pupil cells stays zero.  Returns (s_x, s_y) on the grid.
    """
    N = P.shape[0]
    sx = np.array(s0x, dtype=np.float64)
    sy = np.array(s0y, dtype=np.float64)
    for c in range(N):  # columns: x slopes
        valid = np.flatnonzero(P[:, c])
        if valid.size == 0:
            sx[:, c] = 0.0
            continue
        for m in range(N):
            if not P[m, c]:
                dist = np.abs(valid - m)
                sx[m, c] = s0x[valid[np.argmin(dist)], c]  # argmin takes the first (upper) on a tie
    for r in range(N):  # rows: y slopes
        valid = np.flatnonzero(P[r, :])
        if valid.size == 0:
            sy[r, :] = 0.0
            continue
        for n in range(N):
            if not P[r, n]:
                dist = np.abs(valid - n)
                sy[r, n] = s0y[r, valid[np.argmin(dist)]]
    return enforce_periodicity(sx, sy)


def reconstruct_hudgin(slopes: np.ndarray, mask: np.ndarray, p: Params) -> np.ndarray:
    """Hudgin extension followed by the final reconstruction (Eq. 2 with the Eq. 3 filter);
    the (n+1) x (n+1) node window, as `reconstruct`."""
    s0x, s0y, P = padded_measurement(slopes, mask, p.n_grid)
    sx, sy = hudgin_extend(s0x, s0y, P)
    Rx, Ry = final_filters(p)
    phi = fourier_reconstruct(sx, sy, Rx, Ry)
    o = pupil_offset(p.n_sub, p.n_grid)
    return phi[o:o + p.n_sub + 1, o:o + p.n_sub + 1]


class GerchbergResult(NamedTuple):
    sx: np.ndarray
    sy: np.ndarray
    residuals: list          # in-pupil residual before each replacement (see below)


def gerchberg(s0x: np.ndarray, s0y: np.ndarray, P: np.ndarray, Gx: np.ndarray,
              Gy: np.ndarray, Rx: np.ndarray, Ry: np.ndarray, n_iter: int,
              periodic: bool = True, periodic_each_iter: bool = False,
              start: Optional[tuple] = None) -> GerchbergResult:
    """Algorithm 1: extend the measured slopes beyond the pupil.

    ``start`` optionally replaces the zero out-of-pupil start values (the
    measured values inside the pupil are always imposed).  ``residuals[i]``
    is ||P (s^{i+1} - s^0)|| / ||P s^0|| computed from the filtered slopes of
    iteration i+1 before step 4 puts the measurement back.
    """
    Pbar = ~P
    if start is None:
        sx = s0x.copy()
        sy = s0y.copy()
    else:
        sx = np.where(P, s0x, start[0])
        sy = np.where(P, s0y, start[1])
    norm0 = math.sqrt(float(np.sum(s0x[P] ** 2) + np.sum(s0y[P] ** 2)))
    residuals = []
    for _ in range(n_iter):
        # 1: Fourier transform
        Sx = dft2(sx)
        Sy = dft2(sy)
        # 2: phase reconstruction (LSQ filter), then gradient computation
        Phi = Rx * Sx + Ry * Sy
        Sx_i = Gx * Phi
        Sy_i = Gy * Phi
        # 3: inverse transform
        sx_i = np.real(idft2(Sx_i))
        sy_i = np.real(idft2(Sy_i))
        if norm0 > 0.0:
            r = math.sqrt(float(np.sum((sx_i - s0x)[P] ** 2) + np.sum((sy_i - s0y)[P] ** 2)))
            residuals.append(r / norm0)
        else:
            residuals.append(0.0)
        # 4: measured values inside the pupil, extrapolated ones outside
        sx = s0x * P + sx_i * Pbar
        sy = s0y * P + sy_i * Pbar
        if periodic_each_iter:
            sx, sy = enforce_periodicity(sx, sy)
    # 5: periodic condition on the final slopes
    if periodic:
        sx, sy = enforce_periodicity(sx, sy)
    return GerchbergResult(sx, sy, residuals)


def fourier_reconstruct(sx: np.ndarray, sy: np.ndarray, Rx: np.ndarray, Ry: np.ndarray) -> np.ndarray:
    """Eq. 2: phi_hat = Re TF^-1 (R_x TF(s_x) + R_y TF(s_y))."""
    return np.real(idft2(Rx * dft2(sx) + Ry * dft2(sy)))


# ---------------------------------------------------------------------------
# Whole frame
# ---------------------------------------------------------------------------

class Params(NamedTuple):
    n_sub: int
    n_grid: int
    n_iter: int = 10
    periodic: bool = True
    periodic_each_iter: bool = False
    gamma: float = 1.0
    noise_var: float = 0.05 ** 2
    r0: float = 0.15
    L0: float = 25.0
    d: float = 0.2
    model: str = "fried"   # slope model: "fried" or "sinc"
    d_px: float = 0.0      # detector pixel length [m] (sinc model: difference over d - d_px)


def final_filters(p: Params):
    Gx, Gy, S = slope_model(p.model, p.n_grid, p.d_px / p.d)
    ratio = None
    if p.gamma != 0.0:
        ratio = noise_to_signal(p.n_grid, p.d, p.r0, p.L0, p.noise_var)
    return wiener_reconstructor(Gx, Gy, p.gamma, ratio, S)


def extend(slopes: np.ndarray, mask: np.ndarray, p: Params, start=None) -> GerchbergResult:
    """Padded measurement -> Algorithm 1 (steps 1-5) -> extended slopes on the N x N grid."""
    s0x, s0y, P = padded_measurement(slopes, mask, p.n_grid)
    Gx, Gy, S = slope_model(p.model, p.n_grid, p.d_px / p.d)
    Rx, Ry = wiener_reconstructor(Gx, Gy, 0.0, singular=S)
    return gerchberg(s0x, s0y, P, Gx, Gy, Rx, Ry, p.n_iter, p.periodic,
                     p.periodic_each_iter, start)


def reconstruct(slopes: np.ndarray, mask: np.ndarray, p: Params, start=None) -> np.ndarray:
    """Extension followed by the final (MMSE when gamma = 1) reconstruction.

    Returns the (n+1) x (n+1) phase on the Fried nodes of the lenslet array,
    i.e. grid nodes [o, o+n] x [o, o+n].
    """
    ext = extend(slopes, mask, p, start)
    Rx, Ry = final_filters(p)
    phi = fourier_reconstruct(ext.sx, ext.sy, Rx, Ry)
    o = pupil_offset(p.n_sub, p.n_grid)
    n = p.n_sub
    return phi[o:o + n + 1, o:o + n + 1]


def reconstruct_batch(slopes: np.ndarray, mask: np.ndarray, p: Params) -> np.ndarray:
    """Frame by frame over ``slopes[B, 2, n, n]``; returns ``[B, n+1, n+1]`` float64."""
    out = np.empty((slopes.shape[0], p.n_sub + 1, p.n_sub + 1))
    for b in range(slopes.shape[0]):
        out[b] = reconstruct(np.asarray(slopes[b], dtype=np.float64), mask, p)
    return out


def extend_batch(slopes: np.ndarray, mask: np.ndarray, p: Params) -> np.ndarray:
    """Frame by frame; returns the extended slopes ``[B, 2, N, N]`` float64."""
    N = p.n_grid
    out = np.empty((slopes.shape[0], 2, N, N))
    for b in range(slopes.shape[0]):
        r = extend(np.asarray(slopes[b], dtype=np.float64), mask, p)
        out[b, 0] = r.sx
        out[b, 1] = r.sy
    return out
