"""FP64 CPU oracle for the learned initial extension (a small CNN).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg); never used
by the product path.  This part is not in the paper: a network predicts the
out-of-pupil slopes that Algorithm 1 starts from (instead of the zero padding
of Sec. 4.1); the Gerchberg loop always runs after it.

Network: seven 3x3 convolutions with zero "same" padding on the N x N grid,
channels 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2, a bias per output channel
and ReLU after every layer but the last.  Input channels: padded x slopes,
padded y slopes (both times a fixed input scale), pupil indicator.  Output:
the x and y slopes (times the same scale) on the whole grid; only the values
outside the pupil are used.  Loss: mean squared error over the out-of-pupil
cells of both output channels.

Convolution (cross-correlation, as in every CNN framework):
    y[b, o, i, j] = bias[o] + sum_{c, u, v} w[o, c, u, v] x[b, c, i + u - 1, j + v - 1]
with x = 0 outside the grid.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((3, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 2))


def conv3x3(x: np.ndarray, w: np.ndarray, bias: np.ndarray) -> np.ndarray:
    """x [B, C, H, W], w [O, C, 3, 3], bias [O] -> [B, O, H, W] (float64)."""
    B, C, H, W = x.shape
    O = w.shape[0]
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.broadcast_to(bias.reshape(1, O, 1, 1), (B, O, H, W)).astype(np.float64).copy()
    for u in range(3):
        for v in range(3):
            patch = xp[:, :, u:u + H, v:v + W]                 # x[b, c, i+u-1, j+v-1]
            y += np.einsum("oc,bchw->bohw", w[:, :, u, v], patch)
    return y


def conv3x3_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray):
    """Gradients of sum(gy * conv3x3(x, w, b)) w.r.t. x, w and b."""
    B, C, H, W = x.shape
    O = w.shape[0]
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w, dtype=np.float64)
    for u in range(3):
        for v in range(3):
            patch = xp[:, :, u:u + H, v:v + W]
            gw[:, :, u, v] = np.einsum("bohw,bchw->oc", gy, patch)
            gxp[:, :, u:u + H, v:v + W] += np.einsum("oc,bohw->bchw", w[:, :, u, v], gy)
    gb = gy.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:-1, 1:-1], gw, gb


def init_params(seed: int = 0, layers=LAYERS):
    """He-normal weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in layers:
        std = np.sqrt(2.0 / (cin * 9))
        params.append((rng.standard_normal((cout, cin, 3, 3)) * std, np.zeros(cout)))
    return params


def forward(x: np.ndarray, params, act_round=None):
    """Returns the list of layer outputs (post-activation; the last is linear).

    `act_round` (optional) is applied to every hidden layer's output before the next layer
    reads it: the precision an implementation stores its activations in (None = FP64)."""
    acts = [x]
    h = x
    for li, (w, b) in enumerate(params):
        z = conv3x3(h, w, b)
        h = np.maximum(z, 0.0) if li < len(params) - 1 else z
        if act_round is not None and li < len(params) - 1:
            h = act_round(h)
        acts.append(h)
    return acts


def masked_mse(pred: np.ndarray, target: np.ndarray, outside: np.ndarray):
    """Mean over the out-of-pupil cells (outside = 1) of both channels; returns (loss, dloss/dpred)."""
    m = outside.astype(np.float64)
    count = pred.shape[0] * pred.shape[1] * m.sum()
    diff = (pred - target) * m
    return float(np.sum(diff * diff) / count), 2.0 * diff / count


def backward(acts, params, gout: np.ndarray, grad_round=None):
    """Backpropagate dloss/d(output) through the network; returns [(gw, gb)] per layer.

    `grad_round` (optional) is applied to the gradient with respect to every hidden layer's
    pre-activation (after its ReLU), the precision an implementation stores it in."""
    grads = [None] * len(params)
    g = gout
    for li in range(len(params) - 1, -1, -1):
        w, _ = params[li]
        if li < len(params) - 1:
            g = g * (acts[li + 1] > 0.0)       # ReLU of this layer
            if grad_round is not None:
                g = grad_round(g)
        gx, gw, gb = conv3x3_backward(acts[li], w, g)
        grads[li] = (gw, gb)
        g = gx
    return grads


def features(slopes_grid: np.ndarray, pupil: np.ndarray, scale: float) -> np.ndarray:
    """Network input [B, 3, N, N] from padded slopes [B, 2, N, N] and the pupil indicator [N, N]."""
    B, _, N, _ = slopes_grid.shape
    x = np.empty((B, 3, N, N))
    x[:, 0:2] = slopes_grid * scale
    x[:, 2] = pupil.astype(np.float64)
    return x


def adam_step(params, grads, state, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba, "Adam: a method for stochastic optimization", Algorithm 1).

    `params` and `grads` are flat float64 arrays of the same length; `state` is a dict that
    holds the step count t and the first and second moment estimates m and v (empty on the
    first call).  With t the number of the step being taken:
        m <- beta1 m + (1 - beta1) g,       v <- beta2 v + (1 - beta2) g^2,
        m^ = m / (1 - beta1^t),             v^ = v / (1 - beta2^t),
        theta <- theta - lr m^ / (sqrt(v^) + eps).
    Returns the new parameters; `state` is updated in place.
    """
    g = np.asarray(grads, dtype=np.float64)
    theta = np.asarray(params, dtype=np.float64)
    if not state:
        state["t"] = 0
        state["m"] = np.zeros_like(g)
        state["v"] = np.zeros_like(g)
    state["t"] += 1
    t = state["t"]
    state["m"] = beta1 * state["m"] + (1.0 - beta1) * g
    state["v"] = beta2 * state["v"] + (1.0 - beta2) * g * g
    m_hat = state["m"] / (1.0 - beta1 ** t)
    v_hat = state["v"] / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps)
