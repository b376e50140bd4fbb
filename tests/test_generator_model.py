"""The host model of the device frame generator, pinned to published values (CPU only)."""
import numpy as np

from paper_1705_04298_amd import inputs as I
from _philox import box_muller, philox4x32_10, reference_frames


def test_philox_known_answers():
    # known-answer vectors published with Philox4x32-10 (Random123 distribution)
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        assert tuple(int(x) for x in philox4x32_10(ctr, key)) == want


def test_box_muller_moments():
    w = philox4x32_10((np.arange(200_000), 7, 0, 0), (1, 2))
    a, b = box_muller(w[0], w[1])
    for x in (a, b):
        assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
    assert abs(np.mean(a * b)) < 0.01


def test_reference_frames_statistics():
    """Screen pairs from the model have the von Karman phase-difference variance of a periodic
    N x N screen: D(r) = sum over the grid spectrum of 2 a^2 (1 - cos(kappa . r)) per screen."""
    n, N, d = 24, 48, 8.0 / 24
    mask = I.pupil_mask(n)
    B = 64
    _, ph = reference_frames(n, N, d, mask, 99, 0, B, 0.15, 25.0, 0.0, I.von_karman_psd)
    f = np.fft.fftfreq(N, d=d)
    kx, ky = np.meshgrid(f, f)
    a2 = I.von_karman_psd(kx * kx + ky * ky, 0.15, 25.0) / (N * d) ** 2
    a2[0, 0] = 0.0
    for lag in (1, 4):
        # Re (and Im) of sum a (g0 + i g1) e^{i theta}: phase differences at lag r have variance
        # sum a^2 |e^{i kappa r} - 1|^2 = sum 2 a^2 (1 - cos kappa r)
        want = np.sum(2 * a2 * (1 - np.cos(2 * np.pi * kx * lag * d)))
        got = np.mean((ph[:, :, lag:] - ph[:, :, :-lag]) ** 2)
        assert abs(got / want - 1) < 0.15, (lag, got, want)
