"""The lenslet-averaging (sinc) slope model of Eq. 4 in the FP64 oracle (CPU only).

Pins: the transfer function equals the continuous Shack-Hartmann measurement of single
Fourier modes computed by Gauss-Legendre quadrature over the lenslet edges; its real-space
kernel is real and it vanishes exactly on its singular set; under this model the loop keeps
the measurement, its residual does not increase, a true extension is a fixed point, Eq. 5
zeroes the line sums, and the LSQ final filter recovers a band-limited phase up to piston.
"""
import numpy as np
import pytest

from oracle import fwr_oracle as O


def _quadrature_slopes(kp, lp, N, m, n):
    """x and y edge-average differences of the mode exp(2 pi i (k' x + l' y) / N) (d = 1)
    over cell (m, n): lenslet x in [n, n + 1], y in [m, m + 1]."""
    t, w = np.polynomial.legendre.leggauss(40)
    u = 0.5 * (t + 1.0)  # nodes on [0, 1]
    w = 0.5 * w
    mode = lambda x, y: np.exp(2j * np.pi * (kp * x + lp * y) / N)
    sx = np.sum(w * (mode(n + 1.0, m + u) - mode(n + 0.0, m + u)))
    sy = np.sum(w * (mode(n + u, m + 1.0) - mode(n + u, m + 0.0)))
    return sx, sy


@pytest.mark.parametrize("N", [16, 20])
def test_transfer_function_matches_quadrature(N):
    Gx, Gy = O.sinc_model(N)
    rng = np.random.default_rng(N)
    half = N // 2
    for _ in range(12):
        kp, lp = rng.integers(-half + 1, half, size=2)
        m, n = rng.integers(0, N, size=2)
        sx, sy = _quadrature_slopes(kp, lp, N, m, n)
        node = np.exp(2j * np.pi * (kp * n + lp * m) / N)
        assert abs(sx - Gx[lp % N, kp % N] * node) < 1e-12
        assert abs(sy - Gy[lp % N, kp % N] * node) < 1e-12


@pytest.mark.parametrize("N", [8, 10, 16])
def test_real_kernel_and_singular_set(N):
    Gx, Gy = O.sinc_model(N)
    for G in (Gx, Gy):
        assert np.abs(np.fft.ifft2(G).imag).max() < 1e-15
    g2 = np.abs(Gx) ** 2 + np.abs(Gy) ** 2
    S = O.sinc_singular_set(N)
    assert np.all(g2[S] == 0.0) and np.all(g2[~S] > 1e-6)


def _bandlimited_phase(N, seed):
    """Real periodic phase without DC or Nyquist content."""
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    F[0, 0] = 0.0
    if N % 2 == 0:
        F[N // 2, :] = 0.0
        F[:, N // 2] = 0.0
    return np.real(np.fft.ifft2(F)) * N


def _model_slopes(phi):
    Gx, Gy = O.sinc_model(phi.shape[0])
    P = np.fft.fft2(phi)
    return np.real(np.fft.ifft2(Gx * P)), np.real(np.fft.ifft2(Gy * P))


def test_loop_invariants_under_the_sinc_model():
    n, N = 8, 16
    mask = (np.random.default_rng(3).random((n, n)) < 0.8).astype(np.uint8)
    p = O.Params(n_sub=n, n_grid=N, n_iter=6, periodic=False, model="sinc")
    slopes = np.random.default_rng(4).standard_normal((2, n, n))
    r = O.extend(slopes, mask, p)
    o = (N - n) // 2
    m = mask.astype(bool)
    assert np.array_equal(r.sx[o:o + n, o:o + n][m], slopes[0][m])
    assert np.array_equal(r.sy[o:o + n, o:o + n][m], slopes[1][m])
    assert all(b <= a + 1e-12 for a, b in zip(r.residuals, r.residuals[1:]))
    rp = O.extend(slopes, mask, p._replace(periodic=True))
    assert np.abs(rp.sx.sum(axis=1)).max() < 1e-12 and np.abs(rp.sy.sum(axis=0)).max() < 1e-12


def test_true_extension_is_a_fixed_point():
    n, N = 8, 16
    phi = _bandlimited_phase(N, 5)
    sx, sy = _model_slopes(phi)
    o = (N - n) // 2
    mask = np.ones((n, n), dtype=np.uint8)
    mask[3:5, 3:5] = 0
    slopes = np.stack([sx[o:o + n, o:o + n], sy[o:o + n, o:o + n]]) * mask
    p = O.Params(n_sub=n, n_grid=N, n_iter=4, periodic=False, model="sinc")
    r = O.extend(slopes, mask, p, start=(sx, sy))
    assert np.abs(r.sx - sx).max() < 1e-10 and np.abs(r.sy - sy).max() < 1e-10


def test_lsq_recovers_a_bandlimited_phase():
    N = 16
    phi = _bandlimited_phase(N, 6)
    sx, sy = _model_slopes(phi)
    Gx, Gy = O.sinc_model(N)
    Rx, Ry = O.wiener_reconstructor(Gx, Gy, 0.0, singular=O.sinc_singular_set(N))
    rec = O.fourier_reconstruct(sx, sy, Rx, Ry)
    assert np.abs(rec - (phi - phi.mean())).max() < 1e-12


def test_sinc_floor_is_the_nyquist_content():
    """Why the lenslet-averaging model's open-loop error floor lies above the Fried model's on the
    same screens: its transfer function vanishes on the Nyquist row and column (R18), so the
    reconstruction has no content there.  Noiseless frames, a 40 x 40 square aperture padded to
    80 x 80, screens periodic on the grid (so generator and model agree), 50 iterations.  Per
    frame, the sinc error against the true phase is the root sum of squares of its error against
    the truth without Nyquist lines and of the Nyquist-line content itself; over the frames (median)
    the error against the Nyquist-free truth matches the Fried model's error against the truth."""
    from paper_1705_04298_amd import inputs as I
    N, n = 80, 40
    rows = []
    for idx in range(8):
        scr = I.vk_screen(np.random.default_rng([7, idx]), N, 0.2, 0.15, 25.0)
        F = np.fft.fft2(scr)
        F[N // 2, :] = 0.0
        F[:, N // 2] = 0.0
        nyq_free = np.real(np.fft.ifft2(F))[:n + 1, :n + 1]
        truth = scr[:n + 1, :n + 1]

        def err(ph, ref):
            e = ph - ref
            e = e - e.mean()
            return float(np.sqrt(np.mean(e * e)))

        out = {}
        for model in ("fried", "sinc"):
            sx, sy = I.fried_slopes_from_nodes(truth) if model == "fried" else I.sinc_slopes_from_screen(scr, n)
            p = O.Params(n_sub=n, n_grid=N, n_iter=50, periodic=True, gamma=1.0, noise_var=1e-6,
                         r0=0.15, L0=25.0, d=0.2, model=model)
            out[model] = O.reconstruct(np.stack([sx, sy]), np.ones((n, n), np.uint8), p)
        s, sn = err(out["sinc"], truth), err(out["sinc"], nyq_free)
        q = err(truth, nyq_free)                               # Nyquist-line content of the truth
        assert abs(s - np.hypot(sn, q)) < 0.1 * s, (idx, s, sn, q)
        assert q > 0.75 * s                                    # most of the sinc error
        rows.append((err(out["fried"], truth), s, sn))
    f, s, sn = np.median(np.array(rows), axis=0)
    assert s > 1.5 * f
    assert abs(sn - f) < 0.25 * f, (sn, f)


def _quadrature_slopes_dpx(kp, lp, N, m, n, delta):
    """As _quadrature_slopes with the edge averages (1 - delta) apart, centred on the lenslet."""
    t, w = np.polynomial.legendre.leggauss(40)
    u = 0.5 * (t + 1.0)
    w = 0.5 * w
    mode = lambda x, y: np.exp(2j * np.pi * (kp * x + lp * y) / N)
    a, b = 0.5 * delta, 1.0 - 0.5 * delta
    sx = np.sum(w * (mode(n + b, m + u) - mode(n + a, m + u)))
    sy = np.sum(w * (mode(n + u, m + b) - mode(n + u, m + a)))
    return sx, sy


@pytest.mark.parametrize("N,delta", [(16, 1.0 / 6.0), (20, 0.25)])
def test_pixel_size_correction_matches_quadrature(N, delta):
    """The d - d_px remark after Eq. 4: the difference of the two edge averages taken (d - d_px)
    apart (Table 1's 6 pixels per lenslet: d_px = d / 6), each over the full edge, by
    Gauss-Legendre quadrature of single Fourier modes."""
    Gx, Gy = O.sinc_model(N, delta)
    rng = np.random.default_rng(N + 1)
    half = N // 2
    for _ in range(12):
        kp, lp = rng.integers(-half + 1, half, size=2)
        m, n = rng.integers(0, N, size=2)
        sx, sy = _quadrature_slopes_dpx(kp, lp, N, m, n, delta)
        node = np.exp(2j * np.pi * (kp * n + lp * m) / N)
        assert abs(sx - Gx[lp % N, kp % N] * node) < 1e-12
        assert abs(sy - Gy[lp % N, kp % N] * node) < 1e-12
    # delta = 0 is the model without the correction; the singular set does not change
    assert np.array_equal(O.sinc_model(N, 0.0)[0], O.sinc_model(N)[0])
    g2 = np.abs(Gx) ** 2 + np.abs(Gy) ** 2
    S = O.sinc_singular_set(N)
    assert np.all(g2[S] == 0.0) and np.all(g2[~S] > 1e-6)


def test_pixel_size_correction_of_the_input_generator():
    """The generator's lenslet-averaged slopes with the correction equal the model applied to a
    screen periodic on the grid (single-mode consistency of inputs.sinc_slopes_from_screen)."""
    from paper_1705_04298_amd import inputs as I
    N, n, delta = 32, 16, 1.0 / 6.0
    scr = I.vk_screen(np.random.default_rng(3), N, 0.2, 0.15, 25.0)
    sx, sy = I.sinc_slopes_from_screen(scr, n, delta)
    Gx, Gy = O.sinc_model(N, delta)
    F = np.fft.fft2(scr)
    wx = np.real(np.fft.ifft2(Gx * F))[:n, :n]
    wy = np.real(np.fft.ifft2(Gy * F))[:n, :n]
    assert np.allclose(sx, wx, atol=1e-12) and np.allclose(sy, wy, atol=1e-12)
