"""Pins of the FP64 CNN oracle (learned initial extension)."""
import numpy as np
import pytest

from oracle import cnn as C

RNG = np.random.default_rng(42)


def test_conv_matches_library_correlation():
    """The 3x3 'same' convolution is scipy's 2-D cross-correlation summed over input channels."""
    from scipy.signal import correlate2d
    x = RNG.standard_normal((2, 3, 7, 9))
    w = RNG.standard_normal((4, 3, 3, 3))
    b = RNG.standard_normal(4)
    y = C.conv3x3(x, w, b)
    for bi in range(2):
        for o in range(4):
            want = b[o] + sum(correlate2d(x[bi, c], w[o, c], mode="same", boundary="fill")
                              for c in range(3))
            assert np.allclose(y[bi, o], want, atol=1e-12)


def test_conv_explicit_sum_at_a_border_pixel():
    x = RNG.standard_normal((1, 2, 5, 5))
    w = RNG.standard_normal((1, 2, 3, 3))
    y = C.conv3x3(x, w, np.zeros(1))
    i, j = 0, 4   # corner: only taps with i+u-1 >= 0 and j+v-1 <= 4 contribute
    acc = 0.0
    for c in range(2):
        for u in range(3):
            for v in range(3):
                ii, jj = i + u - 1, j + v - 1
                if 0 <= ii < 5 and 0 <= jj < 5:
                    acc += w[0, c, u, v] * x[0, c, ii, jj]
    assert np.isclose(y[0, 0, i, j], acc, atol=1e-13)


def _loss(params, x, target, outside):
    acts = C.forward(x, params)
    return C.masked_mse(acts[-1], target, outside)[0]


def test_gradients_match_central_differences():
    """Backward pass vs central finite differences on a tiny network (8x8 grid, 4 channels)."""
    layers = ((3, 4), (4, 4), (4, 2))
    params = C.init_params(3, layers)
    params = [(w, RNG.standard_normal(b.shape) * 0.1) for w, b in params]
    x = RNG.standard_normal((2, 3, 8, 8))
    target = RNG.standard_normal((2, 2, 8, 8))
    outside = (RNG.random((8, 8)) < 0.6).astype(np.float64)
    acts = C.forward(x, params)
    loss, g = C.masked_mse(acts[-1], target, outside)
    grads = C.backward(acts, params, g)
    eps = 1e-6
    for li, (w, b) in enumerate(params):
        for idx in [(0, 0, 1, 1), (1, 2, 0, 2), (w.shape[0] - 1, w.shape[1] - 1, 2, 0)]:
            wp = w.copy(); wp[idx] += eps
            wm = w.copy(); wm[idx] -= eps
            pp = list(params); pp[li] = (wp, b)
            pm = list(params); pm[li] = (wm, b)
            num = (_loss(pp, x, target, outside) - _loss(pm, x, target, outside)) / (2 * eps)
            assert np.isclose(grads[li][0][idx], num, rtol=1e-5, atol=1e-9), (li, idx)
        for o in range(b.shape[0]):
            bp = b.copy(); bp[o] += eps
            bm = b.copy(); bm[o] -= eps
            pp = list(params); pp[li] = (w, bp)
            pm = list(params); pm[li] = (w, bm)
            num = (_loss(pp, x, target, outside) - _loss(pm, x, target, outside)) / (2 * eps)
            assert np.isclose(grads[li][1][o], num, rtol=1e-5, atol=1e-9), (li, o)


def test_input_gradient_matches_central_differences():
    layers = ((3, 4), (4, 2))
    params = C.init_params(5, layers)
    x = RNG.standard_normal((1, 3, 6, 6))
    target = RNG.standard_normal((1, 2, 6, 6))
    outside = np.ones((6, 6))
    acts = C.forward(x, params)
    _, g = C.masked_mse(acts[-1], target, outside)
    # input gradient through the first layer
    g1 = g
    w1, _ = params[1]
    g1 = C.conv3x3_backward(acts[1], w1, g1)[0] * (acts[1] > 0)
    gx = C.conv3x3_backward(acts[0], params[0][0], g1)[0]
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (0, 2, 3, 4), (0, 1, 5, 5)]:
        xp = x.copy(); xp[idx] += eps
        xm = x.copy(); xm[idx] -= eps
        num = (_loss(params, xp, target, outside) - _loss(params, xm, target, outside)) / (2 * eps)
        assert np.isclose(gx[idx], num, rtol=1e-5, atol=1e-9)


def test_parameter_count():
    n = sum(cout * cin * 9 + cout for cin, cout in C.LAYERS)
    assert n == 47714


def test_adam_two_steps_by_hand():
    """Adam (Kingma & Ba, Algorithm 1), values worked out by hand for two steps.

    Element 0 sees g = 2 twice: the bias-corrected moments are 2 and 4 after either step, so
    each step moves lr * 2 / (2 + eps).  Element 1 sees g = 1 then g = -1: after step 2,
    m = 0.9 * 0.1 - 0.1 = -0.01, m^ = -0.01 / (1 - 0.81) = -1/19, v = 0.999 * 0.001 + 0.001
    = 0.001999, v^ = 0.001999 / (1 - 0.998001) = 1, so step 2 moves +lr / 19 / (1 + eps).
    Element 2 has g = 0 throughout and stays put.  A missing bias correction, a swapped
    beta, or eps inside the square root would move these values well beyond the tolerance."""
    lr, eps = 1e-3, 1e-8
    theta0 = np.array([0.5, -0.25, 3.0])
    state = {}
    th1 = C.adam_step(theta0, np.array([2.0, 1.0, 0.0]), state, lr)
    assert state["t"] == 1
    want1 = np.array([0.5 - lr * 2 / (2 + eps), -0.25 - lr * 1 / (1 + eps), 3.0])
    assert np.allclose(th1, want1, rtol=0, atol=1e-15)
    th2 = C.adam_step(th1, np.array([2.0, -1.0, 0.0]), state, lr)
    want2 = np.array([want1[0] - lr * 2 / (2 + eps), want1[1] + lr / 19 / (1 + eps), 3.0])
    assert np.allclose(th2, want2, rtol=0, atol=1e-15)
    # raw moments: m = 0.9 * 0.2 + 0.2 = 0.38 and v = 0.999 * 0.004 + 0.004 = 0.007996 for g = 2
    assert np.allclose(state["m"], [0.38, -0.01, 0.0], rtol=0, atol=1e-15)
    assert np.allclose(state["v"], [0.007996, 0.001999, 0.0], rtol=0, atol=1e-15)


def test_adam_first_step_is_lr_times_sign():
    """A property of Adam's first step (Kingma & Ba, Sec. 2.1): with bias correction the first
    update has magnitude lr (up to eps) whatever the gradient's scale."""
    g = np.sign(np.random.default_rng(8).standard_normal(50)) * np.logspace(-3, 3, 50)  # |g| >= 1e-3
    th = C.adam_step(np.zeros(50), g, {}, 0.01)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-4, atol=0)  # eps / |g| <= 1e-5
