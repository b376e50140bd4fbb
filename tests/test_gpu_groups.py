"""Frames per workgroup of the on-chip kernel, and the autotuner (needs an MI355X).

Every launch shape must give the same bits as one frame pair per workgroup (the
arithmetic of a pair does not depend on its neighbours in the workgroup), and the
last, partly filled workgroup must leave the frames past the batch untouched.
"""
import sys

import numpy as np
import pytest

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_04298_amd import fwr
    fwr.load()
    return fwr


GRIDS = [(8, 4), (12, 6), (16, 8), (20, 10), (24, 12), (32, 16), (40, 20), (48, 24), (64, 32), (80, 40),
         (80, 78)]


def _outputs(F, plan, x, start, N, n):
    B = x.shape[0]
    phase = torch.full((B + 1, n + 1, n + 1), 7.0, device="cuda")  # one guard frame past the batch
    ext = torch.full((B + 1, 2, N, N), 7.0, device="cuda")
    resid = torch.full((B + 1,), 7.0, device="cuda")
    plan.reconstruct(x, phase[:B])
    plan.extend(x, ext[:B], start=start, resid=resid[:B])
    with_start = plan.reconstruct(x, start=start)
    torch.cuda.synchronize()
    assert bool((phase[B] == 7.0).all()) and bool((ext[B] == 7.0).all()) and float(resid[B]) == 7.0
    return phase[:B].clone(), ext[:B].clone(), resid[:B].clone(), with_start


@pytest.mark.parametrize("N,n", GRIDS)
def test_group_sizes_give_the_same_bits(F, N, n):
    B = 11
    mask = I.random_mask(n, seed=500 + N + n)
    slopes = I.random_slopes(B, n, seed=600 + N + n).astype(np.float32)
    plan = F.Plan(n, N, mask, n_iter=4, periodic=True, max_batch=B, d=8.0 / n)
    x = torch.from_numpy(slopes).cuda()
    start = torch.from_numpy(np.random.default_rng(N).standard_normal((B, 2, N, N)).astype(np.float32)).cuda()
    plan.set_group(2)
    ref = _outputs(F, plan, x, start, N, n)
    tried = []
    for fpg in (4, 8, 16):
        try:
            plan.set_group(fpg)
        except F.FwrError as e:
            assert e.status == F.FWR_E_UNSUPPORTED
            continue
        tried.append(fpg)
        _flush(f"[gpu] group N={N} n={n} frames/group={fpg}")
        got = _outputs(F, plan, x, start, N, n)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), (N, n, fpg)
        assert plan.launch_info()[1] == fpg
    if N <= 80 and 2 * n <= N:
        assert tried, "no group size above one pair is available"
    # and against the oracle, for the first and the last frame (partly filled workgroup)
    p = O.Params(n_sub=n, n_grid=N, n_iter=4, periodic=True, gamma=1.0, noise_var=0.05 ** 2, r0=0.15,
                 L0=25.0, d=8.0 / n)
    for b in (0, B - 1):
        want = O.reconstruct(slopes[b].astype(np.float64), mask, p)
        got = ref[0][b].cpu().numpy().astype(np.float64)
        err = np.sqrt(np.mean((got - want) ** 2) / np.mean(want ** 2))
        assert err <= 1e-5, (N, n, b, err)
    with pytest.raises(F.FwrError):
        plan.set_group(3)
    plan.close()


def test_autotune_picks_a_valid_group(F):
    _flush("[gpu] autotune")
    mask = I.pupil_mask(40)
    plan = F.Plan(40, 80, mask, n_iter=10, periodic=True, max_batch=512)
    x, _ = plan.generate(512, 99)
    plan.set_group(2)
    want = plan.reconstruct(x)
    fpg = plan.autotune(512)
    assert fpg in (2, 4) and plan.launch_info()[1] == fpg
    assert torch.equal(plan.reconstruct(x), want)
    # a later plan of the same shape starts from the tuned choice
    other = F.Plan(40, 80, mask, n_iter=10, periodic=True, max_batch=64)
    assert other.launch_info()[1] == fpg
    other.close()
    plan.close()
