"""Noise propagation of the FP64 oracle (Sec. 4.1): exact values from its dense operator.

Pins: the Monte-Carlo average of the oracle on white noise agrees with the dense-operator value
(the operator view is the reconstruction itself), and the trends the paper reports for the error
propagation coefficient hold exactly: more iterations propagate more noise, and Eq. 5 adds a
little at the same iteration count.
"""
import numpy as np

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I
from _noiseprop import exact_coefficient


def _p(n, k, per):
    return O.Params(n_sub=n, n_grid=2 * n, n_iter=k, periodic=per, d=8.0 / n)


def test_monte_carlo_matches_the_dense_operator():
    n = 8
    mask = I.pupil_mask(n)
    p = _p(n, 5, True)
    exact = exact_coefficient(mask, p)
    rng = np.random.default_rng(5)
    nodes = I.pupil_nodes(mask)
    acc = []
    for _ in range(300):
        s = rng.standard_normal((2, n, n)) * mask
        ph = O.reconstruct(s, mask, p)[nodes]
        acc.append(np.mean((ph - ph.mean()) ** 2))
    mc = float(np.mean(acc))
    assert abs(mc / exact - 1) < 0.1, (mc, exact)


def test_trends_of_the_paper():
    n = 8
    mask = I.pupil_mask(n)
    iters = (0, 1, 2, 5, 10)
    plain = [exact_coefficient(mask, _p(n, k, False)) for k in iters]
    per = [exact_coefficient(mask, _p(n, k, True)) for k in iters]
    assert all(a < b for a, b in zip(plain, plain[1:])), plain
    assert all(a < b for a, b in zip(per, per[1:])), per
    assert all(b > a for a, b in zip(plain, per)), (plain, per)
