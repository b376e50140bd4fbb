"""Brute-force real-space constructions used to pin the oracle.

Nothing here imports the oracle.  Every operator is built entry by entry from
its definition on the periodic N x N grid (row index = y, column index = x),
so that a dropped term, a wrong sign or a transposed index in the oracle's
Fourier-domain formulas shows up as a mismatch.
"""
from __future__ import annotations

import numpy as np


def dft_matrix_2d(N: int) -> np.ndarray:
    """(N^2 x N^2) matrix of X[l,k] = sum_{m,n} x[m,n] exp(-2 pi i (l m + k n)/N), built by loops."""
    F = np.zeros((N * N, N * N), dtype=complex)
    for l in range(N):
        for k in range(N):
            for m in range(N):
                for n in range(N):
                    F[l * N + k, m * N + n] = np.exp(-2j * np.pi * (l * m + k * n) / N)
    return F


def fried_stencil_slopes(phi: np.ndarray):
    """Fried slopes of a periodic phase, written as explicit loops over cells."""
    N = phi.shape[0]
    sx = np.zeros((N, N))
    sy = np.zeros((N, N))
    for m in range(N):
        for n in range(N):
            a = phi[m, n]
            b = phi[m, (n + 1) % N]
            c = phi[(m + 1) % N, n]
            d = phi[(m + 1) % N, (n + 1) % N]
            sx[m, n] = 0.5 * ((b - a) + (d - c))
            sy[m, n] = 0.5 * ((c - a) + (d - b))
    return sx, sy


def fried_matrix(N: int) -> np.ndarray:
    """Dense (2 N^2 x N^2) Fried measurement matrix: rows [s_x; s_y], columns = nodes."""
    G = np.zeros((2 * N * N, N * N))
    for j in range(N * N):
        e = np.zeros(N * N)
        e[j] = 1.0
        sx, sy = fried_stencil_slopes(e.reshape(N, N))
        G[: N * N, j] = sx.ravel()
        G[N * N:, j] = sy.ravel()
    return G


def slope_projector(N: int) -> np.ndarray:
    """G pinv(G): orthogonal projector onto the slope fields that are gradients of a phase."""
    G = fried_matrix(N)
    return G @ np.linalg.pinv(G)


def circulant_from_kernel(a: np.ndarray) -> np.ndarray:
    """Dense matrix of y[m,n] = sum_{m',n'} a[(m-m') % N, (n-n') % N] x[m',n']."""
    N = a.shape[0]
    A = np.zeros((N * N, N * N))
    for m in range(N):
        for n in range(N):
            for mp in range(N):
                for nq in range(N):
                    A[m * N + n, mp * N + nq] = a[(m - mp) % N, (n - nq) % N]
    return A


def waffle(N: int) -> np.ndarray:
    m, n = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    return (-1.0) ** (m + n)


def remove_piston_waffle(phi: np.ndarray) -> np.ndarray:
    """Project out the Fried null space {piston, global waffle} (orthogonal projection)."""
    N = phi.shape[0]
    w = waffle(N)
    out = phi - phi.mean()
    out = out - w * np.sum(out * w) / np.sum(w * w)
    return out
