"""The fact the HIP kernels' window pruning rests on, checked in FP64 against the oracle.

Through Algorithm 1 without start values or per-iteration Eq. 5, the adjoint field
q = G_x^T s_x + G_y^T s_y of the slopes that enter each step vanishes outside the
(n+1) x (n+1) node window, and a loop that transforms only window-supported q gives the
oracle's extension.  (With start values it does not vanish: the pruning is not used then.)
"""
import numpy as np
import pytest

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I


def _adjoint(sx, sy, Gx, Gy):
    return np.real(O.idft2(np.conj(Gx) * O.dft2(sx) + np.conj(Gy) * O.dft2(sy)))


def _window(n, N):
    o = (N - n) // 2
    w = np.zeros((N, N), dtype=bool)
    w[o:o + n + 1, o:o + n + 1] = True
    return w


@pytest.mark.parametrize("n,N,seed", [(12, 24, 1), (10, 16, 2), (8, 20, 3)])
def test_adjoint_field_stays_in_the_window(n, N, seed):
    mask = I.random_mask(n, seed=seed)
    slopes = I.random_slopes(1, n, seed=seed)[0]
    s0x, s0y, P = O.padded_measurement(slopes, mask, N)
    Gx, Gy = O.fried_model(N)
    Rx, Ry = O.wiener_reconstructor(Gx, Gy)
    W = _window(n, N)
    sx, sy = s0x.copy(), s0y.copy()
    for _ in range(6):
        q = _adjoint(sx, sy, Gx, Gy)
        assert np.abs(q[~W]).max() <= 1e-12 * np.abs(q).max()
        # steps 1-4 of Algorithm 1
        Phi = Rx * O.dft2(sx) + Ry * O.dft2(sy)
        sx_new = np.where(P, s0x, np.real(O.idft2(Gx * Phi)))
        sy_new = np.where(P, s0y, np.real(O.idft2(Gy * Phi)))
        assert np.abs(sx_new - sx).max() > 0.0  # the loop moves
        sx, sy = sx_new, sy_new


def test_start_values_leave_the_window():
    n, N = 12, 24
    mask = I.random_mask(n, seed=7)
    slopes = I.random_slopes(1, n, seed=7)[0]
    s0x, s0y, P = O.padded_measurement(slopes, mask, N)
    Gx, Gy = O.fried_model(N)
    rng = np.random.default_rng(7)
    sx = np.where(P, s0x, rng.standard_normal((N, N)))
    sy = np.where(P, s0y, rng.standard_normal((N, N)))
    q = _adjoint(sx, sy, Gx, Gy)
    assert np.abs(q[~_window(n, N)]).max() > 0.1 * np.abs(q).max()


@pytest.mark.parametrize("periodic", [False, True])
def test_window_pruned_loop_gives_the_oracle_extension(periodic):
    """phi from window-supported q only (its values outside the window are never used in the
    loop), then the slopes of the last phi everywhere: the oracle's extended slopes."""
    n, N, n_iter = 12, 24, 7
    mask = I.random_mask(n, seed=11)
    slopes = I.random_slopes(1, n, seed=11)[0]
    s0x, s0y, P = O.padded_measurement(slopes, mask, N)
    Gx, Gy = O.fried_model(N)
    Rx, Ry = O.wiener_reconstructor(Gx, Gy)
    L = np.abs(Gx) ** 2 + np.abs(Gy) ** 2
    S = O.singular_set(N)
    Linv = np.where(S, 0.0, 1.0 / np.where(S, 1.0, L))
    W = _window(n, N)
    q = np.where(W, _adjoint(s0x, s0y, Gx, Gy), 0.0)
    for it in range(n_iter):
        Phi = Linv * O.dft2(q)
        if it == n_iter - 1:
            break
        # model slopes of phi on the window's cells only, measurement inside the pupil
        gx = np.real(O.idft2(Gx * Phi))
        gy = np.real(O.idft2(Gy * Phi))
        sx = np.where(P, s0x, gx)
        sy = np.where(P, s0y, gy)
        q = np.where(W, _adjoint(sx, sy, Gx, Gy), 0.0)
    ex = np.where(P, s0x, np.real(O.idft2(Gx * Phi)))
    ey = np.where(P, s0y, np.real(O.idft2(Gy * Phi)))
    if periodic:
        ex, ey = O.enforce_periodicity(ex, ey)
    ref = O.gerchberg(s0x, s0y, P, Gx, Gy, Rx, Ry, n_iter, periodic=periodic)
    scale = np.abs(ref.sx).max()
    assert np.abs(ex - ref.sx).max() <= 1e-12 * scale
    assert np.abs(ey - ref.sy).max() <= 1e-12 * scale
