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
    assert fpg in (2, 4) and plan.launch_info()[1] == fpg and plan.schedule in (0, 1)
    got = plan.reconstruct(x)
    if plan.schedule == 0:
        assert torch.equal(got, want)
    else:  # the other radix schedule rounds differently
        assert float(((got - want) ** 2).mean() / (want ** 2).mean()) ** 0.5 <= 2e-5
    # a later plan of the same shape starts from the tuned choice
    other = F.Plan(40, 80, mask, n_iter=10, periodic=True, max_batch=64)
    assert other.launch_info()[1] == fpg and other.schedule == plan.schedule
    other.close()
    plan.close()


SCHED_GRIDS = [(24, 12), (32, 16), (40, 20), (48, 24), (64, 32), (80, 40), (128, 64)]


def _rel(got, want):
    return np.sqrt(np.mean((got - want) ** 2) / np.mean(want ** 2))


@pytest.mark.parametrize("N,n", SCHED_GRIDS)
def test_second_radix_schedule_matches_oracle(F, N, n):
    """Radix schedule 1 (Cooley-Tukey, radix 5/3/2 first) against the oracle, and the same bits for
    every frames-per-workgroup choice under it."""
    _flush(f"[gpu] radix schedule 1 N={N} n={n}")
    mask = I.pupil_mask(n)
    d = 8.0 / n
    plan = F.Plan(n, N, mask, n_iter=10, periodic=True, max_batch=5, d=d)
    plan.set_schedule(0)
    x, _ = plan.generate(5, 1234)
    p0 = plan.reconstruct(x).clone()
    plan.set_schedule(1)
    assert plan.schedule == 1
    p1 = plan.reconstruct(x).clone()
    torch.cuda.synchronize()
    s64 = x.cpu().numpy().astype(np.float64)
    p = O.Params(n_sub=n, n_grid=N, n_iter=10, periodic=True, d=d)
    for b in range(5):
        want = O.reconstruct(s64[b], mask, p)
        assert _rel(p0[b].cpu().numpy().astype(np.float64), want) <= 1e-5, (0, b)
        assert _rel(p1[b].cpu().numpy().astype(np.float64), want) <= 1e-5, (1, b)
    for fpg in (2, 4, 8, 16):
        try:
            plan.set_group(fpg)
        except F.FwrError:
            continue
        assert torch.equal(plan.reconstruct(x), p1), fpg
    plan.close()


def test_grouped_call_keeps_each_plans_schedule(F):
    _flush("[gpu] radix schedule in a grouped call")
    items = []
    for n, sched in ((20, 1), (40, 0), (64, 1)):
        plan = F.Plan(n, 2 * n, I.pupil_mask(n), n_iter=4, periodic=True, max_batch=3, d=8.0 / n)
        plan.set_schedule(sched)
        x, _ = plan.generate(3, 77)
        items.append((plan, x, torch.empty((3, n + 1, n + 1), device="cuda"), None, None))
    F.reconstruct_group(items)
    torch.cuda.synchronize()
    for plan, x, o, _, _ in items:
        assert torch.equal(o, plan.reconstruct(x)), plan.n_sub
        plan.close()


def test_grouped_call_with_a_persistent_loop_plan(F):
    """A multi-pass plan on schedule 2 (the persistent loop) in a grouped call: beside other items it
    runs one launch per pass, alone in a group the persistent loop; every way gives the bits of the
    plan's own call (the two loop shapes do the same arithmetic)."""
    _flush("[gpu] grouped call, persistent multi-pass loop")
    mp = F.Plan(128, 256, I.pupil_mask(128), n_iter=5, periodic=True, max_batch=6, d=39.0 / 128)
    mp.set_schedule(2)
    xm = torch.from_numpy(I.random_slopes(6, 128, seed=5).astype(np.float32)).cuda()
    ref = mp.reconstruct(xm)
    oc = F.Plan(24, 48, I.pupil_mask(24), n_iter=5, periodic=True, max_batch=4, d=8.0 / 24)
    xo = torch.from_numpy(I.random_slopes(4, 24, seed=6).astype(np.float32)).cuda()
    om = torch.empty_like(ref)
    oo = torch.empty((4, 25, 25), device="cuda")
    F.reconstruct_group([(oc, xo, oo, None, None), (mp, xm, om, None, None)])
    torch.cuda.synchronize()
    assert torch.equal(om, ref) and torch.equal(oo, oc.reconstruct(xo))
    om.zero_()
    F.reconstruct_group([(mp, xm, om, None, None)])
    torch.cuda.synchronize()
    assert torch.equal(om, ref)
    mp.set_schedule(0)
    assert torch.equal(mp.reconstruct(xm), ref)
    mp.close()
    oc.close()


def test_grouped_call_mixes_slope_models_and_paths(F):
    """A group of a lenslet-averaging (sinc) plan, a Fried on-chip plan and a multi-pass plan gives
    the bits of the individual calls."""
    _flush("[gpu] grouped call, mixed models")
    items = []
    for n, N, model in ((40, 80, "sinc"), (24, 48, "fried"), (128, 256, "fried")):
        plan = F.Plan(n, N, I.pupil_mask(n), n_iter=3, periodic=True, max_batch=3, d=8.0 / n, model=model)
        x = torch.from_numpy(I.random_slopes(3, n, seed=n).astype(np.float32)).cuda()
        items.append((plan, x, torch.empty((3, n + 1, n + 1), device="cuda"), None, None))
    F.reconstruct_group(items)
    torch.cuda.synchronize()
    for plan, x, o, _, _ in items:
        assert torch.equal(o, plan.reconstruct(x)), (plan.n_sub, plan.model)
        plan.close()


def test_schedule_choices_outside_the_windowed_kernel(F):
    _flush("[gpu] radix schedule errors")
    cases = [F.Plan(40, 80, I.pupil_mask(40), max_batch=2, model="sinc"),      # Fourier-domain kernel
             F.Plan(78, 80, I.pupil_mask(78), max_batch=2),                    # not 2x padded
             F.Plan(10, 20, I.pupil_mask(10), max_batch=2),                    # T = 5: one schedule
             F.Plan(40, 80, I.pupil_mask(40), max_batch=2, periodic_each_iter=True),
             F.Plan(128, 256, I.pupil_mask(128), max_batch=2, model="sinc")]   # multi-pass, sinc
    for plan in cases:
        plan.set_schedule(0)
        with pytest.raises(F.FwrError) as e:
            plan.set_schedule(1)
        assert e.value.status == F.FWR_E_UNSUPPORTED
        assert plan.schedule == 0
        plan.close()
    plan = F.Plan(40, 80, I.pupil_mask(40), max_batch=2)
    with pytest.raises(F.FwrError) as e:
        plan.set_schedule(3)
    assert e.value.status == F.FWR_E_INVAL
    with pytest.raises(F.FwrError) as e:  # the persistent loop is a multi-pass launch shape
        plan.set_schedule(2)
    assert e.value.status == F.FWR_E_UNSUPPORTED
    assert plan.schedule == 0
    plan.close()
    # the Fried multi-pass plan takes its three launch shapes (column passes of 16 or 64 threads
    # per line, the persistent loop)
    mp = F.Plan(128, 256, I.pupil_mask(128), max_batch=2)
    for sched in (2, 1, 0):
        mp.set_schedule(sched)
        assert mp.schedule == sched
    mp.close()
