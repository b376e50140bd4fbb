"""Host model of the device frame generator's random numbers, for tests only.

Philox4x32-10 written from its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011: two 32x32->64-bit
multiplies per round, Weyl key schedule, ten rounds), vectorised over numpy
uint64 arrays, and the Box-Muller mapping the library documents for
`fwr_generate`.  It shares no code with the library.
"""
import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (broadcastable) of uint32 counter words; key: 2 ints. Returns 4 uint64 arrays."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _LO for x in ctr)
    k0, k1 = np.uint64(key[0]) & _LO, np.uint64(key[1]) & _LO
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = (p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & _LO, (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & _LO
        k0 = (k0 + _W0) & _LO
        k1 = (k1 + _W1) & _LO
    return c0, c1, c2, c3


def box_muller(a, b):
    """Two standard normals per word pair: u1 in (0, 1], u2 in [0, 1), in float64."""
    u1 = ((np.asarray(a, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 1.0) / 2.0 ** 24
    u2 = (np.asarray(b, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) / 2.0 ** 24
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)


def reference_frames(n, N, d, mask, seed, first_frame, B, r0, L0, sigma, psd):
    """Frames first_frame .. first_frame+B-1 of the documented generator, in float64.

    `psd(kappa2, r0, L0)` is the von Karman phase PSD.  Returns (slopes [B, 2, n, n],
    phase [B, n+1, n+1])."""
    o = (N - n) // 2
    key = (seed & 0xFFFFFFFF, seed >> 32)
    f = np.fft.fftfreq(N, d=d)
    kx, ky = np.meshgrid(f, f)               # [l, k]: ky along rows (l), kx along columns (k)
    amp = np.sqrt(psd(kx * kx + ky * ky, r0, L0)) / (N * d)
    amp[0, 0] = 0.0
    l, k = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    m = np.asarray(mask).astype(bool)
    slopes = np.zeros((B, 2, n, n))
    phase = np.zeros((B, n + 1, n + 1))
    idx = np.arange(n * n).reshape(n, n)
    for b in range(B):
        f_ = first_frame + b
        p = f_ // 2
        w = philox4x32_10((p & 0xFFFFFFFF, p >> 32, l * N + k, 0), key)
        g0, g1 = box_muller(w[0], w[1])
        field = np.fft.ifft2((g0 + 1j * g1) * amp) * (N * N)
        scr = field.real if f_ % 2 == 0 else field.imag
        phi = scr[o:o + n + 1, o:o + n + 1]
        a, bb, c, e = phi[:-1, :-1], phi[:-1, 1:], phi[1:, :-1], phi[1:, 1:]
        sx = 0.5 * ((bb - a) + (e - c))
        sy = 0.5 * ((c - a) + (e - bb))
        wn = philox4x32_10((p & 0xFFFFFFFF, p >> 32, idx, 1), key)
        nx, ny = box_muller(wn[0], wn[1]) if f_ % 2 == 0 else box_muller(wn[2], wn[3])
        slopes[b, 0] = np.where(m, sx + sigma * nx, 0.0)
        slopes[b, 1] = np.where(m, sy + sigma * ny, 0.0)
        phase[b] = phi
    return slopes, phase
