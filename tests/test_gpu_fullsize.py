"""Parity at the benchmark sizes, in the launch configurations that bench.py times: whole batches
on the GPU, sampled frames against the FP64 oracle (needs an MI355X).

  * 128 frames of 128x128 subapertures padded to 256x256, 20 iterations (multi-pass path);
  * the mixed closed-loop step: 2048 x 24x24, 2048 x 40x40 (network start), 512 x 64x64 and
    64 x 128x128 frames, padded 2x, 10 iterations, generated on the device; the network's frames
    on a branch of their own beside one grouped call for the others; captured in a HIP graph and
    replayed.
"""
import os
import sys

import numpy as np
import pytest

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REL_TOL = 1e-5
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def rel_rms(got, want):
    return np.sqrt(np.mean((got - want) ** 2) / max(np.mean(want ** 2), 1e-300))


@pytest.mark.parametrize("schedule", [0, 2])
def test_elt128_batch_of_128_sampled(F, schedule):
    """Both launch shapes the autotuner picks between at this size (launch per pass, persistent loop)."""
    _flush(f"[gpu] 128 x 128x128 -> 256x256, 20 iterations, schedule {schedule}")
    B, n, N = 128, 128, 256
    rng = np.random.default_rng(12)
    base = I.make_batch(I.ELT_128, 8, start=40, dtype=np.float32)
    scales = rng.uniform(0.5, 1.5, B).astype(np.float32)
    slopes = np.stack([base[b % 8] * scales[b] for b in range(B)])
    mask = I.pupil_mask(n)
    p = O.Params(n_sub=n, n_grid=N, n_iter=20, periodic=True, gamma=1.0, noise_var=0.05 ** 2, r0=0.15,
                 L0=25.0, d=39.0 / n)
    plan = F.Plan(n, N, mask, n_iter=20, periodic=True, gamma=1.0, noise_var=p.noise_var, r0=p.r0, L0=p.L0,
                  d=p.d, max_batch=B)
    plan.set_schedule(schedule)
    got = plan.reconstruct(torch.from_numpy(slopes).cuda()).cpu().numpy().astype(np.float64)
    plan.close()
    for b in (0, 61, 126, 127):
        want = O.reconstruct(slopes[b].astype(np.float64), mask, p)
        assert rel_rms(got[b], want) <= REL_TOL, b


MIXED = ((24, 2048, 8.0 / 24), (40, 2048, 8.0 / 40), (64, 512, 8.0 / 64), (128, 64, 39.0 / 128))


def test_mixed_step_graph_replays_sampled(F):
    from paper_1705_04298_amd import learned as L
    _flush("[gpu] mixed closed-loop step, graph replays")
    seed = 0x5EED_0517
    plans, xs, outs, ctrs, starts, net = [], [], [], [], [], None
    for n, B, d in MIXED:
        plans.append(F.Plan(n, 2 * n, I.pupil_mask(n), n_iter=10, periodic=True, gamma=1.0, noise_var=0.05 ** 2,
                            r0=0.15, L0=25.0, d=d, max_batch=B))
        xs.append(torch.empty((B, 2, n, n), device="cuda"))
        outs.append(torch.empty((B, n + 1, n + 1), device="cuda"))
        ctrs.append(torch.zeros(1, dtype=torch.int64, device="cuda"))
        starts.append(None)
        if n == L.N_SUB:
            net = F.CNN(n, 2 * n, I.pupil_mask(n), max_batch=B, input_scale=L.INPUT_SCALE)
            net.set_params(np.load(os.path.join(ROOT, "paper_1705_04298_amd", "weights",
                                                "cnn_40x40_fried.npz"))["params"])
            starts[-1] = torch.empty((B, 2, 2 * n, 2 * n), device="cuda")
    work = [(p, x, o, s, None) for p, x, o, s in zip(plans, xs, outs, starts)]
    learned = [w for w in work if w[3] is not None]
    others = [w for w in work if w[3] is None]
    branch = torch.cuda.Stream()

    def step():  # as bench.py times it: the network's frames on a branch beside the grouped loops
        for p, x, c in zip(plans, xs, ctrs):
            p.generate(x.shape[0], seed, counter=c, slopes=x, r0=0.15, L0=25.0, sigma=0.05)
        main = torch.cuda.current_stream()
        branch.wait_stream(main)
        with torch.cuda.stream(branch):
            net.set_stream()
            for p, x, o, s, _ in learned:
                p.set_stream()
                net.forward(x, s)
                p.reconstruct(x, o, start=s)
        net.set_stream()
        for p, _, _, _, _ in learned:
            p.set_stream()
        F.reconstruct_group(others)
        main.wait_stream(branch)

    def rebind():
        for p in plans:
            p.set_stream()
        net.set_stream()

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rebind()
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rebind()
        step()
    rebind()
    rng = np.random.default_rng(3)
    for replay in range(2):
        g.replay()
        torch.cuda.synchronize()
        _flush(f"[gpu] replay {replay} done")
        for (n, B, d), x, o, s in zip(MIXED, xs, outs, starts):
            mask = I.pupil_mask(n)
            p = O.Params(n_sub=n, n_grid=2 * n, n_iter=10, periodic=True, gamma=1.0, noise_var=0.05 ** 2,
                         r0=0.15, L0=25.0, d=d)
            for b in (int(rng.integers(B)), B - 1):
                s64 = x[b].cpu().numpy().astype(np.float64)
                st = None
                if s is not None:
                    sb = s[b].cpu().numpy().astype(np.float64)
                    st = (sb[0], sb[1])
                want = O.reconstruct(s64, mask, p, start=st)
                got = o[b].cpu().numpy().astype(np.float64)
                assert rel_rms(got, want) <= REL_TOL, (replay, n, b)
    # replays draw fresh frames: the device counters moved on by two batches after the eager step
    assert all(int(c.item()) == 3 * B for c, (_, B, _) in zip(ctrs, MIXED))
    for p in plans:
        p.close()
    net.close()
