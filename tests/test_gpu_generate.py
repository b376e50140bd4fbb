"""Device frame generator, grouped launch and graph replays (needs an MI355X).

The generator is checked against the host model of its documented definition
(Philox4x32-10 + Box-Muller + spectral synthesis in float64); grouped launches
against the same plans called one by one (bit for bit); captured graphs against
eager calls replay by replay (bit for bit); frames from the generator through the
library against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I
from _philox import reference_frames

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x0123456789ABCDEF


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


def _plan(F, n, n_iter=10, max_batch=8, periodic=True):
    d = 8.0 / n if n < 128 else 39.0 / 128
    return F.Plan(n, 2 * n, I.pupil_mask(n), n_iter=n_iter, periodic=periodic, d=d, max_batch=max_batch), d


@pytest.mark.parametrize("n", [24, 40, 64, 128])
def test_generator_matches_host_model(F, n):
    _flush(f"[gpu] generator n={n}")
    plan, d = _plan(F, n, max_batch=3)
    B, first = 3, 10
    sl, ph = plan.generate(B, SEED, first_frame=first, r0=0.12, L0=25.0, sigma=0.07, with_phase=True)
    torch.cuda.synchronize()
    got_s, got_p = sl.cpu().numpy(), ph.cpu().numpy()
    want_s, want_p = reference_frames(n, 2 * n, d, I.pupil_mask(n), SEED, first, B, 0.12, 25.0, 0.07,
                                      I.von_karman_psd)
    # FP32 synthesis vs float64: errors of a few 1e-7 of the screen's rms per operation; the
    # slopes inherit the phase's absolute error
    for b in range(B):
        scale = np.sqrt(np.mean(want_p[b] ** 2))
        assert np.abs(got_p[b] - want_p[b]).max() <= 1e-4 * scale, (b, np.abs(got_p[b] - want_p[b]).max(), scale)
        assert np.abs(got_s[b] - want_s[b]).max() <= 2e-4 * scale
        assert np.array_equal(got_s[b] == 0, want_s[b] == 0)
    plan.close()


def test_generator_counter_and_batch_independence(F):
    _flush("[gpu] generator counter")
    plan, _ = _plan(F, 40, max_batch=8)
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    a, _ = plan.generate(4, SEED, counter=counter)
    b, _ = plan.generate(4, SEED, counter=counter)
    whole, _ = plan.generate(8, SEED)
    part, _ = plan.generate(2, SEED, first_frame=6)
    torch.cuda.synchronize()
    assert int(counter.item()) == 8
    assert torch.equal(torch.cat([a, b]), whole)
    assert torch.equal(part, whole[6:])
    with pytest.raises(F.FwrError):
        plan.generate(2, SEED, first_frame=3)  # odd first frame
    # an odd batch moves the counter on to the next pair: frames 0-2, then 4-6
    counter.zero_()
    c, _ = plan.generate(3, SEED, counter=counter)
    d, _ = plan.generate(3, SEED, counter=counter)
    torch.cuda.synchronize()
    assert int(counter.item()) == 8
    assert torch.equal(c, whole[:3]) and torch.equal(d, whole[4:7])
    plan.close()


def test_generated_frames_match_oracle(F):
    _flush("[gpu] generated frames vs oracle")
    for n in (24, 40):
        plan, d = _plan(F, n, max_batch=2)
        sl, _ = plan.generate(2, SEED, first_frame=100)
        phase = plan.reconstruct(sl).cpu().numpy().astype(np.float64)
        s64 = sl.cpu().numpy().astype(np.float64)
        p = O.Params(n_sub=n, n_grid=2 * n, d=d, r0=0.15, L0=25.0, noise_var=0.05 ** 2)
        for b in range(2):
            want = O.reconstruct(s64[b], I.pupil_mask(n), p)
            err = np.linalg.norm(phase[b] - want) / np.linalg.norm(want)
            assert err <= 1e-5, (n, b, err)
        plan.close()


def _mix(F, B=(6, 4, 2, 2)):
    plans, ins, outs, starts = [], [], [], []
    for n, b in zip((24, 40, 64, 128), B):
        plan, _ = _plan(F, n, n_iter=10 if n < 128 else 20, max_batch=b)
        sl, _ = plan.generate(b, SEED + n)
        plans.append(plan)
        ins.append(sl)
        outs.append(torch.empty((b, n + 1, n + 1), device="cuda"))
        starts.append(torch.randn((b, 2, 2 * n, 2 * n), device="cuda") if n == 40 else None)
    return plans, ins, outs, starts


def test_group_matches_individual_calls(F):
    _flush("[gpu] group launch")
    plans, ins, outs, starts = _mix(F)
    resid = torch.empty(ins[1].shape[0], device="cuda")
    F.reconstruct_group([(p, x, o, s, resid if s is not None else None)
                         for p, x, o, s in zip(plans, ins, outs, starts)])
    torch.cuda.synchronize()
    for p, x, o, s in zip(plans, ins, outs, starts):
        r = torch.empty(x.shape[0], device="cuda")
        want = p.reconstruct(x, start=s, resid=r if s is not None else None)
        torch.cuda.synchronize()
        assert torch.equal(o, want), p.n_sub
        if s is not None:
            assert torch.equal(resid, r)
    with pytest.raises(F.FwrError):  # one plan twice
        F.reconstruct_group([(plans[0], ins[0], outs[0], None, None)] * 2)
    F.reconstruct_group([])
    for p in plans:
        p.close()


def test_graph_replays_match_eager(F):
    _flush("[gpu] graph capture")
    B = (6, 4, 2, 2)
    plans, ins, outs, starts = _mix(F, B)
    counters = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in plans]
    work = [(p, x, o, s, None) for p, x, o, s in zip(plans, ins, outs, starts)]

    def step():
        for p, x, c in zip(plans, ins, counters):
            p.generate(x.shape[0], SEED, counter=c, slopes=x)
        F.reconstruct_group(work)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up: creates the group's streams and events outside capture
        for p in plans:
            p.set_stream()
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for p in plans:
            p.set_stream()
        step()
    for p in plans:
        p.set_stream()
    torch.cuda.synchronize()
    for c in counters:
        c.zero_()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in outs]
        assert [int(c.item()) for c in counters] == [(rep + 1) * b for b in B]
        # eager equivalent of replay `rep` (with eager work between replays): frames rep*b .. of
        # each plan's sequence
        for i, (p, s, b) in enumerate(zip(plans, starts, B)):
            xs, _ = p.generate(b, SEED, first_frame=rep * b)
            want = p.reconstruct(xs, start=s)
            torch.cuda.synchronize()
            assert torch.equal(got[i], want), (rep, p.n_sub)
    for p in plans:
        p.close()
