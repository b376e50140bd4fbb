"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances: the reconstructed phase must match the oracle to a relative rms
error <= 1e-5 per frame (float32 path vs float64 oracle); extended slopes to
1e-5 of the frame's rms slope; measured in-pupil slopes bit for bit.
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


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fwr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_04298_amd import fwr as F
    F.load()
    return F


def rel_rms(got, want):
    den = np.sqrt(np.mean(want ** 2))
    return np.sqrt(np.mean((got - want) ** 2)) / max(den, 1e-300)


def run_case(F, slopes, mask, p: O.Params, what="reconstruct", schedule=None):
    n, N = p.n_sub, p.n_grid
    plan = F.Plan(n, N, mask, n_iter=p.n_iter, periodic=p.periodic,
                  periodic_each_iter=p.periodic_each_iter, gamma=p.gamma, noise_var=p.noise_var,
                  r0=p.r0, L0=p.L0, d=p.d, max_batch=max(1, slopes.shape[0]))
    if schedule is not None:
        plan.set_schedule(schedule)
    x = torch.from_numpy(np.ascontiguousarray(slopes, dtype=np.float32)).cuda()
    if what == "reconstruct":
        out = plan.reconstruct(x)
    else:
        out = plan.extend(x)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.float64)
    plan.close()
    return res


def check_reconstruct(F, slopes, mask, p, tag, schedule=None):
    _flush(f"[gpu] reconstruct {tag} n={p.n_sub} N={p.n_grid} B={slopes.shape[0]} it={p.n_iter} "
           f"per={p.periodic} each={p.periodic_each_iter} gamma={p.gamma} schedule={schedule}")
    got = run_case(F, slopes, mask, p, schedule=schedule)
    s32 = slopes.astype(np.float32).astype(np.float64)  # the oracle sees the same float32 inputs
    for b in range(slopes.shape[0]):
        want = O.reconstruct(s32[b], mask, p)
        if np.all(want == 0):
            assert np.abs(got[b]).max() < 1e-6
            continue
        e = rel_rms(got[b], want)
        assert e <= REL_TOL, (tag, b, e)


SPHERE = dict(n_sub=40, n_grid=80, d=0.2, r0=0.15, L0=25.0, noise_var=0.05 ** 2)
ELT = dict(n_sub=128, n_grid=256, d=39.0 / 128, r0=0.15, L0=25.0, noise_var=0.05 ** 2)


def test_sphere40_periodic_10_iterations(fwr):
    """The 40x40 SPHERE-like frame, 10 iterations, Eq. 5 after the loop, MMSE final filter."""
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40, 5, dtype=np.float64)   # odd batch: the last pair is half empty
    check_reconstruct(fwr, slopes, mask, O.Params(n_iter=10, periodic=True, **SPHERE), "sphere")


@pytest.mark.parametrize("n_iter,periodic,each", [(0, False, False), (0, True, False), (1, False, False),
                                                  (2, True, False), (3, False, False), (4, True, True)])
def test_sphere40_variants(fwr, n_iter, periodic, each):
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40, 2, start=20, dtype=np.float64)
    check_reconstruct(fwr, slopes, mask,
                      O.Params(n_iter=n_iter, periodic=periodic, periodic_each_iter=each, **SPHERE),
                      "variant")


def test_lsq_final_filter(fwr):
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40, 2, start=30, dtype=np.float64)
    check_reconstruct(fwr, slopes, mask, O.Params(n_iter=5, periodic=True, gamma=0.0, **SPHERE), "lsq")


@pytest.mark.parametrize("N,n", [(8, 4), (8, 6), (12, 6), (16, 8), (16, 2), (20, 10), (24, 12),
                                 (32, 16), (40, 20), (48, 24), (64, 32), (80, 78), (128, 64),
                                 (256, 128), (256, 250), (256, 252), (256, 254)])
def test_grid_sizes(fwr, N, n):
    """Every grid size (on-chip N <= 128, multi-pass N = 256), random masks, white slopes;
    includes n = N - 2 (thin border; at N = 256 the stencil's reach then wraps round the grid)."""
    mask = I.random_mask(n, seed=N * 1000 + n)
    slopes = I.random_slopes(3, n, seed=N + n)
    p = O.Params(n_sub=n, n_grid=N, n_iter=6, periodic=True, gamma=1.0, noise_var=0.01, r0=0.15,
                 L0=25.0, d=8.0 / n)
    check_reconstruct(fwr, slopes, mask, p, f"grid{N}")


@pytest.mark.parametrize("N,n", [(8, 6), (16, 2), (24, 12), (48, 24), (80, 78), (128, 64), (128, 126)])
@pytest.mark.parametrize("periodic,each", [(False, False), (True, True)])
def test_grid_sizes_other_eq5_modes(fwr, N, n, periodic, each):
    """Without Eq. 5, and with Eq. 5 after every iteration, on thin borders and odd windows."""
    mask = I.random_mask(n, seed=N * 1001 + n)
    slopes = I.random_slopes(3, n, seed=N + 2 * n)
    p = O.Params(n_sub=n, n_grid=N, n_iter=4, periodic=periodic, periodic_each_iter=each, gamma=1.0,
                 noise_var=0.01, r0=0.15, L0=25.0, d=8.0 / n)
    check_reconstruct(fwr, slopes, mask, p, f"grid{N}")


@pytest.mark.parametrize("periodic,each,n_iter", [(False, False, 5), (True, True, 3), (True, False, 1)])
@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_thin_border_multipass(fwr, periodic, each, n_iter, schedule):
    """N = 256 with a one-cell border (n = 254, o = 1): the stencil's reach wraps round the grid and
    node row N-1 is a window row; every launch shape (column passes of 16 and 64 threads per line,
    the loop as one persistent launch)."""
    mask = I.random_mask(254, seed=254)
    slopes = I.random_slopes(2, 254, seed=7)
    p = O.Params(n_sub=254, n_grid=256, n_iter=n_iter, periodic=periodic, periodic_each_iter=each, gamma=1.0,
                 noise_var=0.01, r0=0.15, L0=25.0, d=39.0 / 254)
    check_reconstruct(fwr, slopes, mask, p, "thin256", schedule=schedule)


@pytest.mark.parametrize("periodic", [False, True])
def test_extend_matches_oracle_and_keeps_measurement(fwr, periodic):
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40, 3, start=40, dtype=np.float32)
    p = O.Params(n_iter=7, periodic=periodic, **SPHERE)
    _flush(f"[gpu] extend periodic={periodic}")
    got = run_case(fwr, slopes, mask, p, what="extend")
    s64 = slopes.astype(np.float64)
    o = 20
    for b in range(3):
        ref = O.extend(s64[b], mask, p)
        scale = np.sqrt(np.mean(ref.sx ** 2 + ref.sy ** 2))
        assert np.abs(got[b, 0] - ref.sx).max() <= 10 * REL_TOL * scale
        assert np.abs(got[b, 1] - ref.sy).max() <= 10 * REL_TOL * scale
        m = mask.astype(bool)
        # measured slopes come back bit for bit
        assert np.array_equal(got[b, 0, o:o + 40, o:o + 40][m].astype(np.float32), slopes[b, 0][m])
        assert np.array_equal(got[b, 1, o:o + 40, o:o + 40][m].astype(np.float32), slopes[b, 1][m])
        if periodic:
            assert np.abs(got[b, 0].sum(axis=1)).max() < 1e-3 * scale * 80
            assert np.abs(got[b, 1].sum(axis=0)).max() < 1e-3 * scale * 80


def test_out_of_pupil_values_are_ignored(fwr):
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40, 2, start=50, dtype=np.float32)
    g = slopes.copy()
    g[:, :, mask == 0] = 123.0
    p = O.Params(n_iter=3, periodic=True, **SPHERE)
    assert np.array_equal(run_case(fwr, slopes, mask, p), run_case(fwr, g, mask, p))


def test_bitwise_deterministic(fwr):
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40, 6, start=60, dtype=np.float32)
    p = O.Params(n_iter=10, periodic=True, **SPHERE)
    a = run_case(fwr, slopes, mask, p)
    b = run_case(fwr, slopes, mask, p)
    assert np.array_equal(a, b)


def _isolation_case(case):
    """(slopes, mask, params, what, bad cell) of one isolation case."""
    if case.startswith("multipass"):
        mask = I.pupil_mask(128)
        slopes = I.make_batch(I.ELT_128, 5, start=40, dtype=np.float32)
        p = O.Params(n_iter=3, periodic=True, **ELT)
        cell = (64, 3)
    else:
        mask = I.pupil_mask(40)
        slopes = I.make_batch(I.SPHERE_40, 5, start=70, dtype=np.float32)
        p = O.Params(n_iter=4, periodic=True, periodic_each_iter=case == "each", **SPHERE)
        cell = (20, 3)
    assert mask[cell] == 1  # a valid subaperture (the centre is obstructed)
    return slopes, mask, p, "extend" if case.endswith("extend") else "reconstruct", cell


@pytest.mark.parametrize("case", ["win", "each", "extend", "multipass", "multipass_extend"])
@pytest.mark.parametrize("which,value", [(2, np.nan), (3, np.inf), (4, -np.inf)])
def test_non_finite_frame_is_isolated(fwr, case, which, value):
    """Frames share a complex field in pairs (2i real, 2i+1 imaginary).  A frame with a
    non-finite in-pupil slope gets an all-NaN output; every other frame, its partner included,
    is bit for bit what it is when that slope is zero.  Frame 4 of the 5 has no partner."""
    slopes, mask, p, what, cell = _isolation_case(case)
    _flush(f"[gpu] isolation {case} frame={which} value={value}")
    bad = slopes.copy()
    bad[which, 1 if which == 3 else 0][cell] = value
    ref = slopes.copy()
    ref[which, 1 if which == 3 else 0][cell] = 0.0
    got = run_case(fwr, bad, mask, p, what)
    want = run_case(fwr, ref, mask, p, what)
    assert np.isnan(got[which]).all()
    others = [b for b in range(slopes.shape[0]) if b != which]
    assert np.array_equal(got[others], want[others])
    assert np.isfinite(got[others]).all()


def test_non_finite_outside_the_pupil_is_ignored(fwr):
    """Slopes of cells outside the pupil are not read: a NaN there changes nothing."""
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40, 4, start=75, dtype=np.float32)
    p = O.Params(n_iter=4, periodic=True, **SPHERE)
    assert mask[0, 0] == 0
    bad = slopes.copy()
    bad[1, 0, 0, 0] = np.nan
    assert np.array_equal(run_case(fwr, bad, mask, p), run_case(fwr, slopes, mask, p))


def test_abi_errors(fwr):
    F = fwr
    mask = I.pupil_mask(40)
    plan = F.Plan(40, 80, mask, max_batch=4)
    x = torch.zeros((5, 2, 40, 40), device="cuda")
    y = torch.zeros((5, 41, 41), device="cuda")
    assert F.fwr_reconstruct(plan._h, x.data_ptr(), y.data_ptr(), 5) == F.FWR_E_INVAL
    assert F.fwr_reconstruct(plan._h, 0, y.data_ptr(), 2) == F.FWR_E_INVAL
    assert F.fwr_reconstruct(plan._h, x.data_ptr(), 0, 2) == F.FWR_E_INVAL
    assert F.fwr_reconstruct(plan._h, 0, 0, 0) == F.FWR_OK          # empty batch is a no-op
    assert F.fwr_reconstruct(plan._h, x.data_ptr(), y.data_ptr(), -1) == F.FWR_E_INVAL
    assert F.fwr_extend(None, x.data_ptr(), y.data_ptr(), 1) == F.FWR_E_STATE
    plan.close()
    with pytest.raises(F.FwrError):
        F.Plan(40, 81, mask)          # N - n odd
    with pytest.raises(F.FwrError):
        F.Plan(40, 40, mask)          # N <= n
    with pytest.raises(F.FwrError) as e:
        F.Plan(40, 84, mask)          # not a supported grid size
    assert e.value.status == F.FWR_E_UNSUPPORTED


@pytest.mark.parametrize("n,N", [(40, 80), (128, 256)])
def test_calls_are_ordered_on_the_plans_stream(fwr, n, N):
    """A plan bound to a side stream reads its input after earlier work on that stream and
    before later work on it; the result equals the null-stream result bit for bit."""
    F = fwr
    _flush(f"[gpu] side stream n={n} N={N}")
    mask = I.pupil_mask(n)
    cfg = SPHERE if n == 40 else ELT
    slopes = (I.make_batch(I.SPHERE_40, 4, start=90, dtype=np.float32) if n == 40
              else I.make_batch(I.ELT_128, 2, start=7, dtype=np.float32))
    p = O.Params(n_iter=5, periodic=True, **cfg)
    want = run_case(F, slopes, mask, p)
    B = slopes.shape[0]
    src = torch.from_numpy(slopes).cuda()
    x = torch.zeros_like(src)
    y = torch.full((B, n + 1, n + 1), -1.0, device="cuda")
    big = torch.ones(1 << 26, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    plan = F.Plan(n, N, mask, n_iter=5, periodic=True, gamma=p.gamma, noise_var=p.noise_var, r0=p.r0,
                  L0=p.L0, d=p.d, max_batch=B, stream=s.cuda_stream)
    with torch.cuda.stream(s):
        for _ in range(16):           # keeps the stream busy before the input is written
            big.mul_(1.0)
        x.copy_(src)
        plan.reconstruct(x, y)
        x.zero_()                     # overwriting the input afterwards must not reach the result
        got = y.clone()
    s.synchronize()
    plan.close()
    assert np.array_equal(got.cpu().numpy().astype(np.float64), want)


def test_full_batch_sampled(fwr):
    """4096 frames in one launch (the batched workload); 12 frames checked against the oracle."""
    mask = I.pupil_mask(40)
    B = 4096
    rng = np.random.default_rng(5)
    base = I.make_batch(I.SPHERE_40_BATCH, 64, dtype=np.float32)
    # tile 64 distinct generated frames with per-frame sign/scale changes (keeps generation fast)
    slopes = np.empty((B, 2, 40, 40), dtype=np.float32)
    scales = rng.uniform(0.5, 1.5, B).astype(np.float32)
    for b in range(B):
        slopes[b] = base[b % 64] * scales[b]
    p = O.Params(n_iter=10, periodic=True, **SPHERE)
    _flush("[gpu] full batch 4096")
    got = run_case(fwr, slopes, mask, p)
    for b in rng.choice(B, 12, replace=False):
        want = O.reconstruct(slopes[b].astype(np.float64), mask, p)
        assert rel_rms(got[b], want) <= REL_TOL, b




@pytest.mark.parametrize("n_iter,periodic,each", [(20, True, False), (0, True, False), (3, False, False),
                                                  (2, True, True)])
def test_elt128_multipass(fwr, n_iter, periodic, each):
    """128x128 subapertures, D = 39 m, padded to 256x256 (multi-pass through HBM)."""
    mask = I.pupil_mask(128)
    slopes = I.make_batch(I.ELT_128, 3, dtype=np.float64)
    check_reconstruct(fwr, slopes, mask,
                      O.Params(n_iter=n_iter, periodic=periodic, periodic_each_iter=each, **ELT), "elt")


@pytest.mark.parametrize("n_iter,periodic,each", [(20, True, False), (3, False, False), (2, True, True)])
def test_elt128_column_pass_64_threads_per_line(fwr, n_iter, periodic, each):
    """The column pass's second launch shape (schedule 1: one wave per 256-point line, quads of
    lanes doing the 16-point sub-transforms) against the oracle (the two shapes round differently:
    each is held to the oracle's tolerance, not to the other)."""
    mask = I.pupil_mask(128)
    slopes = I.make_batch(I.ELT_128, 3, start=11, dtype=np.float64)
    p = O.Params(n_iter=n_iter, periodic=periodic, periodic_each_iter=each, **ELT)
    check_reconstruct(fwr, slopes, mask, p, "elt-q", schedule=1)


@pytest.mark.parametrize("n_iter,periodic,each", [(20, True, False), (3, False, False), (2, True, True)])
def test_elt128_persistent_loop(fwr, n_iter, periodic, each):
    """Schedule 2: the loop's column passes and fused row steps as one persistent launch whose
    workgroups hand the spectra to one another (per-pair counts) against the oracle; with Eq. 5 after
    every iteration the plan keeps the launch-per-pass loop."""
    mask = I.pupil_mask(128)
    slopes = I.make_batch(I.ELT_128, 5, start=17, dtype=np.float64)
    p = O.Params(n_iter=n_iter, periodic=periodic, periodic_each_iter=each, **ELT)
    check_reconstruct(fwr, slopes, mask, p, "elt-persistent", schedule=2)


@pytest.mark.parametrize("n,periodic,n_iter", [(100, True, 7), (200, True, 5), (250, False, 4), (252, True, 3),
                                              (64, True, 9)])
def test_persistent_loop_other_windows(fwr, n, periodic, n_iter):
    """The persistent loop on other lenslet counts of the 256 x 256 grid (window row blocks and the
    stencil's reach of other sizes: 4 to 16 row blocks per step), random masks, against the oracle
    and bit for bit against the launch-per-pass loop."""
    mask = I.random_mask(n, seed=n + 17)
    slopes = I.random_slopes(5, n, seed=n + 18)
    p = O.Params(n_sub=n, n_grid=256, n_iter=n_iter, periodic=periodic, gamma=1.0, noise_var=0.01, r0=0.15,
                 L0=25.0, d=39.0 / n)
    check_reconstruct(fwr, slopes, mask, p, f"persistent n={n}", schedule=2)
    a = run_case(fwr, slopes, mask, p, schedule=0)
    b = run_case(fwr, slopes, mask, p, schedule=2)
    assert np.array_equal(a, b)


def test_persistent_loop_watchdog(fwr):
    """A wait limit of one poll makes the persistent loop give up as soon as an item finds its pair's
    previous step unfinished (forced from the host; every kernel still ends normally): the call's
    frames are then all NaN, never partly computed, and the next call with the default limit is
    exact again (the start pass clears the error word)."""
    B = 128
    mask = I.pupil_mask(128)
    slopes = I.make_batch(I.ELT_128, 8, start=21, dtype=np.float32)
    x = torch.from_numpy(np.ascontiguousarray(np.concatenate([slopes] * (B // 8)))).cuda()
    p = O.Params(n_iter=20, periodic=True, **ELT)
    plan = fwr.Plan(128, 256, mask, n_iter=20, periodic=True, gamma=p.gamma, noise_var=p.noise_var, r0=p.r0,
                    L0=p.L0, d=p.d, max_batch=B)
    _flush("[gpu] persistent loop watchdog")
    plan.set_schedule(0)
    ref = plan.reconstruct(x).cpu().numpy()
    plan.set_schedule(2)
    for bad in (0, 1 << 25):
        with pytest.raises(fwr.FwrError) as e:
            plan.set_wait_limit(bad)
        assert e.value.status == fwr.FWR_E_INVAL
    plan.set_wait_limit(1)
    gave_up = 0
    for _ in range(3):
        got = plan.reconstruct(x).cpu().numpy()
        if np.isnan(got).all():
            gave_up += 1
        else:
            assert np.array_equal(got, ref)
    assert gave_up > 0  # (128 frames: some item always finds its dependency unfinished)
    plan.set_wait_limit(1 << 20)
    assert np.array_equal(plan.reconstruct(x).cpu().numpy(), ref)
    plan.close()
    onchip = fwr.Plan(40, 80, I.pupil_mask(40), max_batch=2)
    with pytest.raises(fwr.FwrError) as e:
        onchip.set_wait_limit(100)
    assert e.value.status == fwr.FWR_E_UNSUPPORTED
    onchip.close()


def test_persistent_loops_on_two_streams(fwr):
    """Two plans on the persistent loop, enqueued on two streams at once (two launches that may share
    the CUs; each waits only on its own items): the bits of each plan run alone."""
    mask = I.pupil_mask(128)
    p = O.Params(n_iter=10, periodic=True, **ELT)
    _flush("[gpu] two persistent loops on two streams")
    plans, xs, refs = [], [], []
    for k in range(2):
        plan = fwr.Plan(128, 256, mask, n_iter=10, periodic=True, gamma=p.gamma, noise_var=p.noise_var, r0=p.r0,
                        L0=p.L0, d=p.d, max_batch=64)
        plan.set_schedule(2)
        x = torch.from_numpy(I.make_batch(I.ELT_128, 64, start=100 * k, dtype=np.float32)).cuda()
        refs.append(plan.reconstruct(x).clone())
        plans.append(plan)
        xs.append(x)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    outs = [torch.empty_like(r) for r in refs]
    for _ in range(3):
        for plan, x, o, st in zip(plans, xs, outs, streams):
            plan.set_stream(st.cuda_stream)
            plan.reconstruct(x, o)
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o, r)
    for plan in plans:
        plan.close()


def test_persistent_loop_in_a_graph(fwr):
    """The persistent loop captured in a HIP graph and replayed several times, with eager work of
    the same plan between the replays: every replay gives the eager bits (the start pass clears the
    loop's counters as a kernel, so a replay starts from zero counts)."""
    mask = I.pupil_mask(128)
    p = O.Params(n_iter=6, periodic=True, **ELT)
    _flush("[gpu] persistent loop in a graph")
    plan = fwr.Plan(128, 256, mask, n_iter=6, periodic=True, gamma=p.gamma, noise_var=p.noise_var, r0=p.r0,
                    L0=p.L0, d=p.d, max_batch=32)
    plan.set_schedule(2)
    x = torch.from_numpy(I.make_batch(I.ELT_128, 32, start=7, dtype=np.float32)).cuda()
    x2 = torch.from_numpy(I.make_batch(I.ELT_128, 32, start=70, dtype=np.float32)).cuda()
    ref = plan.reconstruct(x).clone()
    ref2 = plan.reconstruct(x2).clone()
    out = torch.empty_like(ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.set_stream()
        plan.reconstruct(x, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.set_stream()
        plan.reconstruct(x, out)
    plan.set_stream()
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        assert torch.equal(plan.reconstruct(x2), ref2)  # (eager work of the same plan between replays)
    plan.close()


@pytest.mark.parametrize("B,n_iter,periodic", [(5, 20, True), (7, 2, True), (4, 3, False), (6, 1, True),
                                               (3, 5, False), (64, 10, True)])
def test_persistent_loop_same_bits_as_launch_per_pass(fwr, B, n_iter, periodic):
    """The persistent loop runs the same column-tile and row-block arithmetic as the launch-per-pass
    loop (16 threads per line): bit-identical phases and extended slopes, odd and even batches."""
    mask = I.pupil_mask(128)
    slopes = I.make_batch(I.ELT_128, B, start=3, dtype=np.float32)
    p = O.Params(n_iter=n_iter, periodic=periodic, **ELT)
    _flush(f"[gpu] persistent loop vs launch per pass B={B} n_iter={n_iter} periodic={periodic}")
    for what in ("reconstruct", "extend"):
        a = run_case(fwr, slopes, mask, p, what=what, schedule=0)
        b = run_case(fwr, slopes, mask, p, what=what, schedule=2)
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), what


def test_multipass_autotune_keeps_a_column_shape(fwr):
    """The autotuner times the three launch shapes of a multi-pass plan, keeps the fastest and
    starts later plans of the same shape from it; results stay within the oracle's tolerance."""
    mask = I.pupil_mask(128)
    p = O.Params(n_iter=4, periodic=True, **ELT)
    plan = fwr.Plan(128, 256, mask, n_iter=4, periodic=True, gamma=p.gamma, noise_var=p.noise_var,
                    r0=p.r0, L0=p.L0, d=p.d, max_batch=8)
    assert plan.autotune(8) == 2
    chosen = plan.schedule
    assert chosen in (0, 1, 2)
    threads, fpg, _ = plan.launch_info()
    assert fpg == 2 and threads == {0: 256, 1: 1024, 2: 288}[chosen]
    plan.close()
    again = fwr.Plan(128, 256, mask, n_iter=4, periodic=True, gamma=p.gamma, noise_var=p.noise_var,
                     r0=p.r0, L0=p.L0, d=p.d, max_batch=8)
    assert again.schedule == chosen
    again.close()
    slopes = I.make_batch(I.ELT_128, 2, start=13, dtype=np.float64)
    check_reconstruct(fwr, slopes, mask, p, "elt-tuned", schedule=chosen)


@pytest.mark.parametrize("periodic,schedule", [(False, 0), (True, 0), (True, 1), (True, 2), (False, 2)])
def test_elt128_extend(fwr, periodic, schedule):
    mask = I.pupil_mask(128)
    slopes = I.make_batch(I.ELT_128, 2, start=5, dtype=np.float32)
    p = O.Params(n_iter=6, periodic=periodic, **ELT)
    _flush(f"[gpu] elt extend periodic={periodic} schedule={schedule}")
    got = run_case(fwr, slopes, mask, p, what="extend", schedule=schedule)
    o = 64
    m = mask.astype(bool)
    for b in range(2):
        ref = O.extend(slopes[b].astype(np.float64), mask, p)
        scale = np.sqrt(np.mean(ref.sx ** 2 + ref.sy ** 2))
        assert np.abs(got[b, 0] - ref.sx).max() <= 10 * REL_TOL * scale
        assert np.abs(got[b, 1] - ref.sy).max() <= 10 * REL_TOL * scale
        assert np.array_equal(got[b, 0, o:o + 128, o:o + 128][m].astype(np.float32), slopes[b, 0][m])


@pytest.mark.parametrize("n", [254, 252])
def test_thin_border_multipass_extend(fwr, n):
    mask = I.random_mask(n, seed=n + 1)
    slopes = I.random_slopes(2, n, seed=n + 2).astype(np.float32)
    p = O.Params(n_sub=n, n_grid=256, n_iter=4, periodic=True, gamma=1.0, noise_var=0.01, r0=0.15, L0=25.0,
                 d=39.0 / n)
    _flush(f"[gpu] thin-border extend n={n}")
    got = run_case(fwr, slopes, mask, p, what="extend")
    o = (256 - n) // 2
    m = mask.astype(bool)
    for b in range(2):
        ref = O.extend(slopes[b].astype(np.float64), mask, p)
        scale = np.sqrt(np.mean(ref.sx ** 2 + ref.sy ** 2))
        assert np.abs(got[b, 0] - ref.sx).max() <= 10 * REL_TOL * scale
        assert np.abs(got[b, 1] - ref.sy).max() <= 10 * REL_TOL * scale
        assert np.array_equal(got[b, 0, o:o + n, o:o + n][m].astype(np.float32), slopes[b, 0][m])


@pytest.mark.parametrize("n,N,model", [(40, 80, "fried"), (20, 40, "fried"), (128, 256, "fried"), (40, 80, "sinc")])
def test_alpha_map_replaces_the_regulariser(fwr, n, N, model):
    """A caller's map of gamma W_eta / W_phi (row = frequency l along y, column = k along x; even,
    not symmetric under l <-> k) in the final filter: against the oracle's extension and Eq. 2/3
    with that map."""
    _flush(f"[gpu] alpha map n={n} N={N} {model}")
    mask = I.pupil_mask(n)
    slopes = I.random_slopes(3, n, seed=N + 5).astype(np.float32)
    rng = np.random.default_rng(N)
    raw = 0.05 + rng.uniform(0.0, 0.5, (N, N)) * (1.0 + np.arange(N)[None, :] / N)
    neg = (-np.arange(N)) % N
    alpha = 0.5 * (raw + raw[neg][:, neg])  # even, as a ratio of spectra of real processes is
    assert not np.allclose(alpha, alpha.T)
    p = O.Params(n_sub=n, n_grid=N, n_iter=4, periodic=True, d=8.0 / n, model=model)
    plan = fwr.Plan(n, N, mask, n_iter=4, periodic=True, d=p.d, alpha_map=alpha, max_batch=3, model=model)
    got = plan.reconstruct(torch.from_numpy(slopes).cuda()).cpu().numpy().astype(np.float64)
    plan.close()
    Gx, Gy, S = O.slope_model(model, N)
    Rx, Ry = O.wiener_reconstructor(Gx, Gy, 1.0, alpha, S)
    o = (N - n) // 2
    for b in range(3):
        ext = O.extend(slopes[b].astype(np.float64), mask, p)
        want = O.fourier_reconstruct(ext.sx, ext.sy, Rx, Ry)[o:o + n + 1, o:o + n + 1]
        assert rel_rms(got[b], want) <= REL_TOL, b
