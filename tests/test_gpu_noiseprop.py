"""Noise propagation of the GPU path against the oracle's exact value (needs an MI355X)."""
import sys

import pytest

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I
from _noiseprop import exact_coefficient

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def NP():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_04298_amd import fwr, noiseprop
    fwr.load()
    return noiseprop


@pytest.mark.parametrize("n,n_iter,periodic", [(8, 0, False), (8, 2, True), (12, 10, True), (12, 10, False)])
def test_gpu_coefficient_matches_exact(NP, n, n_iter, periodic):
    print(f"[gpu] noise propagation n={n} it={n_iter} periodic={periodic}", flush=True)
    sys.stdout.flush()
    exact = exact_coefficient(I.pupil_mask(n), O.Params(n_sub=n, n_grid=2 * n, n_iter=n_iter, periodic=periodic,
                                                        d=8.0 / n))
    # 16384 frames: the relative standard error is a few 1e-3
    got = NP.coefficient(n, 2 * n, n_iter, periodic, frames=16384, sigma=0.5)
    assert abs(got / exact - 1) < 0.02, (got, exact)
