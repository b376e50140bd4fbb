"""Exact noise propagation of the FP64 oracle, for tests only.

The reconstruction is linear in the slopes: applying the oracle to each unit slope vector of a
valid subaperture gives its dense operator R, and for white slope noise of variance sigma^2 the
expected piston-removed energy on the pupil nodes is sigma^2 ||C R||_F^2 (C removes the mean over
the pupil nodes).  The coefficient divides by the number of pupil nodes and sigma^2.
"""
import numpy as np

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I


def dense_operator(mask, p: O.Params) -> np.ndarray:
    n = p.n_sub
    cols = []
    for comp in (0, 1):
        for i, j in np.argwhere(np.asarray(mask).astype(bool)):
            s = np.zeros((2, n, n))
            s[comp, i, j] = 1.0
            cols.append(O.reconstruct(s, mask, p).ravel())
    return np.stack(cols, axis=1)


def exact_coefficient(mask, p: O.Params) -> float:
    R = dense_operator(mask, p)
    nodes = I.pupil_nodes(mask).ravel()
    Rp = R[nodes]
    Rp = Rp - Rp.mean(axis=0, keepdims=True)
    return float((Rp ** 2).sum() / nodes.sum())
