"""Process-wide launch state, argument checks of the grouped call and the fallback's treatment
of non-finite residuals (needs an MI355X)."""
import os
import sys

import numpy as np
import pytest

from oracle import cnn as C
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


def test_dynamic_lds_limit_survives_a_smaller_plan(F):
    """The dynamic-LDS limit of a kernel is process-wide: a plan made later for a smaller shape
    must not lower it under an earlier plan's launches (on-chip kernel N = 80 with n = 78 then
    n = 40, Fourier-domain kernel likewise, Hudgin kernel N = 128 then N = 80, network N = 80
    then N = 48).  The first objects' results are compared bit for bit with what they gave
    before the smaller ones existed, and the on-chip phase with the oracle."""
    _flush("[gpu] dynamic LDS limits across plans")
    big = []
    for n, N, model in ((78, 80, "fried"), (78, 80, "sinc"), (64, 128, "fried")):
        mask = I.pupil_mask(n)
        plan = F.Plan(n, N, mask, n_iter=3, periodic=True, max_batch=3, d=8.0 / n, model=model)
        x = torch.from_numpy(I.random_slopes(3, n, seed=n + N).astype(np.float32)).cuda()
        big.append((plan, x, mask, plan.reconstruct(x).clone(), plan.hudgin_extend(x).clone()))
    net = F.CNN(40, 80, I.pupil_mask(40), max_batch=2, input_scale=0.5)
    net.set_params(F.params_to_flat(C.init_params(3)))
    xn = torch.from_numpy(I.random_slopes(2, 40, seed=5).astype(np.float32)).cuda()
    pred = net.forward(xn).clone()
    torch.cuda.synchronize()
    small = [F.Plan(n, N, I.pupil_mask(n), n_iter=3, periodic=True, max_batch=3, d=8.0 / n, model=model)
             for n, N, model in ((40, 80, "fried"), (40, 80, "sinc"), (40, 80, "fried"))]
    small_net = F.CNN(24, 48, I.pupil_mask(24), max_batch=2, input_scale=0.5)
    for plan, x, mask, phase, ext in big:
        assert torch.equal(plan.reconstruct(x), phase), (plan.n_sub, plan.n_grid, plan.model)
        assert torch.equal(plan.hudgin_extend(x), ext), (plan.n_sub, plan.n_grid, plan.model)
    assert torch.equal(net.forward(xn), pred)
    plan, x, mask, phase, _ = big[0]
    p = O.Params(n_sub=78, n_grid=80, n_iter=3, periodic=True, d=8.0 / 78)
    got = phase.cpu().numpy().astype(np.float64)
    for b in range(3):
        want = O.reconstruct(x[b].cpu().numpy().astype(np.float64), mask, p)
        assert np.sqrt(np.mean((got[b] - want) ** 2) / np.mean(want ** 2)) < 1e-5
    for h in [b[0] for b in big] + small + [net, small_net]:
        h.close()


def test_grouped_call_checks_every_item_first(F):
    """fwr_reconstruct_group validates all items before it enqueues anything: with a bad item
    last (B above its plan's max_batch, or a start on the multi-pass grid), the call fails
    and the earlier items' outputs are untouched."""
    _flush("[gpu] grouped call argument checks")
    ok = F.Plan(24, 48, I.pupil_mask(24), n_iter=3, periodic=True, max_batch=4, d=8.0 / 24)
    bad = F.Plan(40, 80, I.pupil_mask(40), n_iter=3, periodic=True, max_batch=2, d=0.2)
    mp = F.Plan(128, 256, I.pupil_mask(128), n_iter=2, periodic=True, max_batch=2, d=39.0 / 128)
    x1 = torch.from_numpy(I.random_slopes(4, 24, seed=1).astype(np.float32)).cuda()
    o1 = torch.full((4, 25, 25), 7.0, device="cuda")
    x2 = torch.zeros((3, 2, 40, 40), device="cuda")
    o2 = torch.full((3, 41, 41), 7.0, device="cuda")
    with pytest.raises(F.FwrError) as e:
        F.reconstruct_group([(ok, x1, o1, None, None), (bad, x2, o2, None, None)])
    assert e.value.status == F.FWR_E_INVAL
    x3 = torch.zeros((2, 2, 128, 128), device="cuda")
    o3 = torch.full((2, 129, 129), 7.0, device="cuda")
    st3 = torch.zeros((2, 2, 256, 256), device="cuda")
    with pytest.raises(F.FwrError) as e:
        F.reconstruct_group([(ok, x1, o1, None, None), (mp, x3, o3, st3, None)])
    assert e.value.status == F.FWR_E_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((o1 == 7.0).all()) and bool((o2 == 7.0).all()) and bool((o3 == 7.0).all())
    # the same items, valid, then run
    F.reconstruct_group([(ok, x1, o1, None, None), (mp, x3, o3, None, None)])
    torch.cuda.synchronize()
    assert torch.equal(o1, ok.reconstruct(x1)) and torch.equal(o3, mp.reconstruct(x3))
    for h in (ok, bad, mp):
        h.close()


def test_fallback_recomputes_frames_with_non_finite_residual(F):
    """A network with a NaN bias gives a NaN start, hence NaN residuals: every frame must fall back
    to the plain loop, and the phases then equal the plain loop's bit for bit."""
    from paper_1705_04298_amd import learned as L
    _flush("[gpu] fallback on NaN residuals")
    params = np.load(os.path.join(os.path.dirname(L.__file__), "weights", "cnn_40x40_fried.npz"))["params"]
    params = params.copy()
    params[-1] = np.nan                        # the last bias of the output layer
    B = 6
    slopes, _ = L.make_frames(B, seed0=91_000)
    x = torch.from_numpy(slopes).cuda()
    lr = L.LearnedReconstructor(params, n_iter=2, plain_iter=10, threshold=1e9, max_batch=B)
    ph, resid, nfall = lr.reconstruct(x)
    torch.cuda.synchronize()
    assert bool(torch.isnan(resid).all())
    assert nfall == B
    plain = F.Plan(40, 80, I.pupil_mask(40), n_iter=10, periodic=True, max_batch=B)
    assert torch.equal(ph, plain.reconstruct(x))
    lr.close()
    plain.close()


def test_non_finite_frame_in_learned_call_is_isolated(F):
    """A NaN measured slope in frame 2: the network's start for that frame is non-finite around
    the cell, the frame's phases and residual are NaN and it falls back to the plain loop (NaN
    again).  Frames outside its pair are bit for bit those of the call with that slope zero;
    its partner (frame 3) equals them to rounding (the two share complex transforms)."""
    from paper_1705_04298_amd import learned as L
    _flush("[gpu] learned call with a non-finite frame")
    params = np.load(os.path.join(os.path.dirname(L.__file__), "weights", "cnn_40x40_fried.npz"))["params"]
    B = 6
    slopes, _ = L.make_frames(B, seed0=92_000)
    cell = (20, 3)
    assert I.pupil_mask(40)[cell] == 1
    bad, ref = slopes.copy(), slopes.copy()
    bad[2, 0][cell] = np.nan
    ref[2, 0][cell] = 0.0
    lr = L.LearnedReconstructor(params, n_iter=2, plain_iter=10, threshold=1e9, max_batch=B)
    outs = []
    for s in (bad, ref):
        ph, resid, nfall = lr.reconstruct(torch.from_numpy(np.ascontiguousarray(s)).cuda())
        torch.cuda.synchronize()
        outs.append((ph.cpu().numpy().copy(), resid.cpu().numpy().copy(), nfall))
    (pb, rb, nb), (pr, rr, nr) = outs
    assert nr == 0 and nb == 1
    assert np.isnan(pb[2]).all() and np.isnan(rb[2])
    for b in (0, 1, 4, 5):
        assert np.array_equal(pb[b], pr[b]) and rb[b] == rr[b]
    e = np.sqrt(np.mean((pb[3] - pr[3]) ** 2) / np.mean(pr[3] ** 2))
    assert e < 1e-5 and abs(rb[3] - rr[3]) <= 1e-4 * rr[3], (e, rb[3], rr[3])
    lr.close()
