"""The seeded workload generator: geometry, statistics and reproducibility."""
import json
import os

import numpy as np

from paper_1705_04298_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_mask_counts_have_no_ties():
    """Integer >50 %-lit rule: fixed valid counts, and no subaperture exactly half lit."""
    with open(os.path.join(GOLDEN, "mask_counts.json")) as f:
        want = json.load(f)["valid_subapertures"]
    for n_str, count in want.items():
        n = int(n_str)
        m = I.pupil_mask(n)
        assert int(m.sum()) == count
        assert np.array_equal(m, m[::-1, :]) and np.array_equal(m, m[:, ::-1])
        assert np.array_equal(m, m.T)


def test_frames_are_reproducible_and_independent():
    a, pa = I.make_frame(I.SPHERE_40, 11)
    b, pb = I.make_frame(I.SPHERE_40, 11)
    c, _ = I.make_frame(I.SPHERE_40, 12)
    assert np.array_equal(a, b) and np.array_equal(pa, pb)
    assert not np.allclose(a, c)
    batch = I.make_batch(I.SPHERE_40, 3, start=10, dtype=np.float64)
    assert np.array_equal(batch[1], a)


def test_slopes_are_fried_differences_plus_noise_inside_pupil_only():
    s, phi = I.make_frame(I.SPHERE_40, 4)
    m = I.pupil_mask(40).astype(bool)
    assert np.all(s[:, ~m] == 0.0)
    clean, _ = I.make_frame(I.SPHERE_40, 4, noise_sigma=0.0)
    noise = (s - clean)[:, m]
    assert 0.04 < noise.std() < 0.06
    # x slope of a subaperture = mean of the two horizontal differences of its corners
    i, j = 20, 3
    assert m[i, j]
    want = 0.5 * ((phi[i, j + 1] - phi[i, j]) + (phi[i + 1, j + 1] - phi[i + 1, j]))
    assert np.isclose(clean[0, i, j], want, rtol=1e-12)


def test_screen_structure_function_matches_von_karman():
    """Phase structure function of the screens against the von Karman one,
    D(r) = 4 pi int_0^kc Phi(kappa) [1 - J0(2 pi kappa r)] kappa dkappa (numerical
    quadrature; kc = 1/(2d) is the grid's band limit), within sampling error."""
    from scipy import integrate, special
    w = I.SPHERE_40
    kc = 1.0 / (2.0 * w.d)

    def d_vk(r):
        f = lambda k: 4 * np.pi * I.von_karman_psd(k * k, w.r0, w.L0) \
            * (1 - special.j0(2 * np.pi * k * r)) * k
        return integrate.quad(f, 0.0, kc, limit=800)[0]

    acc = {2: [], 4: [], 8: []}
    for i in range(12):
        scr = I.vk_screen(I.frame_rng(90, i), w.screen_size, w.d, w.r0, w.L0)
        for lag in acc:
            acc[lag].append(np.mean((np.roll(scr, -lag, axis=1) - scr) ** 2))
    for lag, vals in acc.items():
        ratio = np.mean(vals) / d_vk(lag * w.d)
        assert 0.9 < ratio < 1.1, (lag, ratio)
