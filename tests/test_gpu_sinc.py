"""Lenslet-averaging (sinc) slope model on the Fourier-domain kernel vs the FP64 oracle (needs
an MI355X).  Same tolerances as the Fried path: phase <= 1e-5 relative rms per frame, extended
slopes to 1e-4 of the frame's rms slope, measured slopes bit for bit."""
import sys

import numpy as np
import pytest

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_04298_amd import fwr
    fwr.load()
    return fwr


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _plan(F, p: O.Params, mask, B):
    return F.Plan(p.n_sub, p.n_grid, mask, n_iter=p.n_iter, periodic=p.periodic, gamma=p.gamma,
                  noise_var=p.noise_var, r0=p.r0, L0=p.L0, d=p.d, max_batch=B, model="sinc", d_px=p.d_px,
                  periodic_each_iter=p.periodic_each_iter)


def _rel(got, want):
    return np.sqrt(np.mean((got - want) ** 2) / np.mean(want ** 2))


@pytest.mark.parametrize("n_iter,periodic", [(10, True), (0, True), (3, False), (20, True)])
def test_sphere40_sinc_matches_oracle(F, n_iter, periodic):
    _flush(f"[gpu] sinc 40x40 it={n_iter} periodic={periodic}")
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40_SINC, 5, dtype=np.float32)
    p = O.Params(n_sub=40, n_grid=80, n_iter=n_iter, periodic=periodic, model="sinc")
    plan = _plan(F, p, mask, 5)
    got = plan.reconstruct(torch.from_numpy(slopes).cuda()).cpu().numpy().astype(np.float64)
    for b in range(5):
        want = O.reconstruct(slopes[b].astype(np.float64), mask, p)
        assert _rel(got[b], want) <= 1e-5, (b, _rel(got[b], want))
    plan.close()


@pytest.mark.parametrize("n_iter,periodic", [(10, True), (3, False)])
def test_sphere40_sinc_pixel_size_correction(F, n_iter, periodic):
    """The d - d_px correction (Table 1: 6 pixels per lenslet, d_px = d / 6) on frames measured with
    it, against the oracle; the plan without the correction gives a different phase."""
    import dataclasses
    _flush(f"[gpu] sinc 40x40 with d_px = d/6, it={n_iter} periodic={periodic}")
    mask = I.pupil_mask(40)
    w = dataclasses.replace(I.SPHERE_40_SINC, d_px_frac=1.0 / 6.0)
    slopes = I.make_batch(w, 4, dtype=np.float32)
    p = O.Params(n_sub=40, n_grid=80, n_iter=n_iter, periodic=periodic, model="sinc", d=0.2, d_px=0.2 / 6.0)
    plan = _plan(F, p, mask, 4)
    x = torch.from_numpy(slopes).cuda()
    got = plan.reconstruct(x).cpu().numpy().astype(np.float64)
    for b in range(4):
        want = O.reconstruct(slopes[b].astype(np.float64), mask, p)
        assert _rel(got[b], want) <= 1e-5, (b, _rel(got[b], want))
    plain = _plan(F, O.Params(n_sub=40, n_grid=80, n_iter=n_iter, periodic=periodic, model="sinc"), mask, 4)
    assert _rel(plain.reconstruct(x).cpu().numpy().astype(np.float64), got) > 1e-3
    plan.close()
    plain.close()


@pytest.mark.parametrize("N,n", [(8, 4), (16, 8), (24, 12), (32, 16), (40, 20), (48, 24), (64, 32), (80, 78),
                                 (128, 64), (128, 126)])
def test_sinc_grid_sizes_and_groups(F, N, n):
    _flush(f"[gpu] sinc grid N={N} n={n}")
    mask = I.random_mask(n, seed=700 + N + n)
    slopes = I.random_slopes(3, n, seed=N + n).astype(np.float32)
    p = O.Params(n_sub=n, n_grid=N, n_iter=5, periodic=True, d=8.0 / n, model="sinc")
    plan = _plan(F, p, mask, 3)
    x = torch.from_numpy(slopes).cuda()
    plan.set_group(1)
    ref = plan.reconstruct(x).clone()
    try:
        plan.set_group(2)
        assert torch.equal(plan.reconstruct(x), ref)
    except F.FwrError as e:
        assert e.status == F.FWR_E_UNSUPPORTED
    got = ref.cpu().numpy().astype(np.float64)
    for b in range(3):
        want = O.reconstruct(slopes[b].astype(np.float64), mask, p)
        assert _rel(got[b], want) <= 1e-5, (b, _rel(got[b], want))
    plan.close()


@pytest.mark.parametrize("periodic", [False, True])
def test_sinc_extend(F, periodic):
    _flush(f"[gpu] sinc extend periodic={periodic}")
    mask = I.pupil_mask(40)
    slopes = I.make_batch(I.SPHERE_40_SINC, 3, start=10, dtype=np.float32)
    p = O.Params(n_sub=40, n_grid=80, n_iter=7, periodic=periodic, model="sinc")
    plan = _plan(F, p, mask, 3)
    got = plan.extend(torch.from_numpy(slopes).cuda()).cpu().numpy().astype(np.float64)
    m = mask.astype(bool)
    for b in range(3):
        ref = O.extend(slopes[b].astype(np.float64), mask, p)
        scale = np.sqrt(np.mean(ref.sx ** 2 + ref.sy ** 2))
        assert np.abs(got[b, 0] - ref.sx).max() <= 1e-4 * scale
        assert np.abs(got[b, 1] - ref.sy).max() <= 1e-4 * scale
        assert np.array_equal(got[b, 0, 20:60, 20:60][m].astype(np.float32), slopes[b, 0][m])
        assert np.array_equal(got[b, 1, 20:60, 20:60][m].astype(np.float32), slopes[b, 1][m])
    plan.close()


def test_sinc_unsupported_calls(F):
    mask = I.pupil_mask(40)
    plan = F.Plan(40, 80, mask, n_iter=2, max_batch=2, model="sinc")
    x = torch.zeros((2, 2, 40, 40), device="cuda")
    with pytest.raises(F.FwrError):
        plan.generate(2, 1)
    big = F.Plan(128, 256, I.pupil_mask(128), n_iter=2, max_batch=2, model="sinc")   # multi-pass grid
    xb = torch.zeros((2, 2, 128, 128), device="cuda")
    with pytest.raises(F.FwrError) as e:
        big.reconstruct(xb, start=torch.zeros((2, 2, 256, 256), device="cuda"))
    assert e.value.status == F.FWR_E_UNSUPPORTED
    with pytest.raises(F.FwrError) as e:
        big.hudgin_extend(xb)
    assert e.value.status == F.FWR_E_UNSUPPORTED
    big.close()
    plan.close()


@pytest.mark.parametrize("N,n,periodic", [(80, 40, True), (80, 40, False), (48, 24, True), (80, 78, True)])
def test_sinc_start_values_and_residual(F, N, n, periodic):
    """Start values outside the pupil and the last iteration's in-pupil residual under the sinc
    model, against the oracle (phase, extended slopes, residual)."""
    _flush(f"[gpu] sinc start N={N} n={n} periodic={periodic}")
    mask = I.random_mask(n, seed=N + 3 * n)
    slopes = I.random_slopes(3, n, seed=N * 7 + n).astype(np.float32)
    start = np.random.default_rng(N + n).standard_normal((3, 2, N, N)).astype(np.float32)
    p = O.Params(n_sub=n, n_grid=N, n_iter=3, periodic=periodic, d=8.0 / n, model="sinc")
    plan = _plan(F, p, mask, 3)
    x = torch.from_numpy(slopes).cuda()
    st = torch.from_numpy(start).cuda()
    resid = torch.empty(3, device="cuda")
    ext = plan.extend(x, start=st, resid=resid).cpu().numpy().astype(np.float64)
    r = resid.cpu().numpy()
    phase = plan.reconstruct(x, start=st).cpu().numpy().astype(np.float64)
    for b in range(3):
        s64 = slopes[b].astype(np.float64)
        st64 = (start[b, 0].astype(np.float64), start[b, 1].astype(np.float64))
        ref = O.extend(s64, mask, p, start=st64)
        scale = np.sqrt(np.mean(ref.sx ** 2 + ref.sy ** 2))
        assert np.abs(ext[b, 0] - ref.sx).max() <= 1e-4 * scale
        assert np.abs(ext[b, 1] - ref.sy).max() <= 1e-4 * scale
        assert abs(r[b] - ref.residuals[-1]) <= 1e-4 * ref.residuals[-1]
        assert _rel(phase[b], O.reconstruct(s64, mask, p, start=st64)) <= 1e-5
    # the residual without start values, and zero with no iteration
    r0 = torch.empty(3, device="cuda")
    plan.reconstruct(x, resid=r0)
    ref0 = O.extend(slopes[0].astype(np.float64), mask, p)
    assert abs(float(r0[0]) - ref0.residuals[-1]) <= 1e-4 * ref0.residuals[-1]
    plan.close()
    p0 = O.Params(n_sub=n, n_grid=N, n_iter=0, periodic=False, d=8.0 / n, model="sinc")
    plan0 = _plan(F, p0, mask, 3)
    rz = torch.full((3,), 7.0, device="cuda")
    plan0.reconstruct(x, resid=rz)
    assert bool((rz == 0).all())
    plan0.close()


@pytest.mark.parametrize("n,N", [(40, 80), (24, 48)])
def test_sinc_hudgin_extension(F, n, N):
    """The Hudgin extension on a lenslet-averaging plan, then Eq. 2/3 of the sinc model from it."""
    _flush(f"[gpu] sinc hudgin n={n} N={N}")
    mask = I.pupil_mask(n)
    slopes = I.random_slopes(3, n, seed=N + n + 11).astype(np.float32)
    p = O.Params(n_sub=n, n_grid=N, n_iter=0, periodic=False, d=8.0 / n, model="sinc")
    plan0 = _plan(F, p, mask, 3)
    x = torch.from_numpy(slopes).cuda()
    ext = plan0.hudgin_extend(x)
    phase = plan0.reconstruct(x, start=ext).cpu().numpy().astype(np.float64)
    ext = ext.cpu().numpy().astype(np.float64)
    for b in range(3):
        s0x, s0y, P = O.padded_measurement(slopes[b].astype(np.float64), mask, N)
        rx, ry = O.hudgin_extend(s0x, s0y, P)
        assert np.array_equal(ext[b, 0, :, :N - 1], rx[:, :N - 1])
        assert np.array_equal(ext[b, 1, :N - 1, :], ry[:N - 1, :])
        assert _rel(phase[b], O.reconstruct_hudgin(slopes[b].astype(np.float64), mask, p)) <= 1e-5
    plan0.close()


@pytest.mark.parametrize("N,n,periodic", [(80, 40, False), (80, 40, True), (48, 46, True), (128, 64, True)])
def test_sinc_eq5_after_every_iteration(F, N, n, periodic):
    """Eq. 5 after every step 4 (plan flag periodic_each_iter) under the lenslet-averaging model:
    phase, extended slopes (measured slopes bit for bit) and residual against the oracle."""
    _flush(f"[gpu] sinc per-iteration Eq. 5 N={N} n={n} periodic={periodic}")
    mask = I.pupil_mask(n)
    slopes = I.random_slopes(3, n, seed=900 + N + n).astype(np.float32)
    p = O.Params(n_sub=n, n_grid=N, n_iter=4, periodic=periodic, periodic_each_iter=True, d=8.0 / n,
                 model="sinc")
    plan = _plan(F, p, mask, 3)
    x = torch.from_numpy(slopes).cuda()
    resid = torch.empty(3, device="cuda")
    ext = plan.extend(x, resid=resid).cpu().numpy().astype(np.float64)
    got = plan.reconstruct(x).cpu().numpy().astype(np.float64)
    r = resid.cpu().numpy()
    o = (N - n) // 2
    for b in range(3):
        s64 = slopes[b].astype(np.float64)
        ref = O.extend(s64, mask, p)
        scale = np.sqrt(np.mean(ref.sx ** 2 + ref.sy ** 2))
        assert np.abs(ext[b, 0] - ref.sx).max() <= 1e-4 * scale
        assert np.abs(ext[b, 1] - ref.sy).max() <= 1e-4 * scale
        inside = mask.astype(bool)
        assert np.array_equal(ext[b, 0, o:o + n, o:o + n][inside], slopes[b, 0][inside].astype(np.float64))
        assert abs(r[b] - ref.residuals[-1]) <= 1e-4 * ref.residuals[-1]
        assert _rel(got[b], O.reconstruct(s64, mask, p)) <= 1e-5
    plan.close()


def test_sinc_128_start_values_and_residual(F):
    """N = 128 (measured slopes read from global memory at step 4): start values and residual."""
    _flush("[gpu] sinc N=128 start values")
    N, n = 128, 64
    mask = I.pupil_mask(n)
    slopes = I.random_slopes(2, n, seed=77).astype(np.float32)
    start = np.random.default_rng(78).standard_normal((2, 2, N, N)).astype(np.float32)
    p = O.Params(n_sub=n, n_grid=N, n_iter=3, periodic=True, d=39.0 / 128, model="sinc")
    plan = _plan(F, p, mask, 2)
    x = torch.from_numpy(slopes).cuda()
    resid = torch.empty(2, device="cuda")
    got = plan.reconstruct(x, start=torch.from_numpy(start).cuda(), resid=resid).cpu().numpy().astype(np.float64)
    r = resid.cpu().numpy()
    for b in range(2):
        st = (start[b, 0].astype(np.float64), start[b, 1].astype(np.float64))
        s64 = slopes[b].astype(np.float64)
        assert _rel(got[b], O.reconstruct(s64, mask, p, start=st)) <= 1e-5
        assert abs(r[b] - O.extend(s64, mask, p, start=st).residuals[-1]) <= 1e-4 * r[b]
    plan.close()


@pytest.mark.parametrize("schedule", [0, 2])
@pytest.mark.parametrize("n,n_iter,periodic,each,dpx", [(128, 20, True, False, 0.0), (128, 5, False, False, 0.0),
                                                       (128, 3, True, True, 0.0), (128, 0, True, False, 0.0),
                                                       (128, 6, True, False, 1.0 / 6.0), (254, 4, True, False, 0.0)])
def test_sinc_256_multipass_matches_oracle(F, n, n_iter, periodic, each, dpx, schedule):
    """The lenslet-averaging model on the 256 x 256 grid (multi-pass through HBM): phase and
    extended slopes against the oracle (measured slopes bit for bit), ELT frames measured with the
    model (D = 39 m), with and without Eq. 5, per-iteration Eq. 5, zero iterations, the d - d_px
    correction, and a one-cell border (n = 254); the loop as one launch per pass (schedule 0) and
    as one persistent launch (schedule 2)."""
    import dataclasses
    _flush(f"[gpu] sinc 256 n={n} it={n_iter} periodic={periodic} each={each} dpx={dpx:.3f} sched={schedule}")
    N, B = 256, 3
    if n == 128:
        w = dataclasses.replace(I.ELT_128, model="sinc", d_px_frac=dpx, config_id=7)
        slopes = I.make_batch(w, B, dtype=np.float32)
        mask = I.pupil_mask(n)
    else:
        mask = I.random_mask(n, seed=5)
        slopes = I.random_slopes(B, n, seed=6).astype(np.float32)
    d = 39.0 / n
    p = O.Params(n_sub=n, n_grid=N, n_iter=n_iter, periodic=periodic, periodic_each_iter=each, d=d,
                 d_px=dpx * d, model="sinc")
    plan = _plan(F, p, mask, B)
    plan.set_schedule(schedule)
    x = torch.from_numpy(slopes).cuda()
    got = plan.reconstruct(x).cpu().numpy().astype(np.float64)
    ext = plan.extend(x).cpu().numpy().astype(np.float64) if n_iter > 0 else None
    o = (N - n) // 2
    m = mask.astype(bool)
    for b in range(B):
        s64 = slopes[b].astype(np.float64)
        assert _rel(got[b], O.reconstruct(s64, mask, p)) <= 1e-5, (b, _rel(got[b], O.reconstruct(s64, mask, p)))
        if ext is not None:
            ref = O.extend(s64, mask, p)
            scale = np.sqrt(np.mean(ref.sx ** 2 + ref.sy ** 2))
            assert np.abs(ext[b, 0] - ref.sx).max() <= 1e-4 * scale
            assert np.abs(ext[b, 1] - ref.sy).max() <= 1e-4 * scale
            assert np.array_equal(ext[b, 0, o:o + n, o:o + n][m], slopes[b, 0][m].astype(np.float64))
            assert np.array_equal(ext[b, 1, o:o + n, o:o + n][m], slopes[b, 1][m].astype(np.float64))
    plan.close()


@pytest.mark.parametrize("B,n_iter,periodic", [(5, 20, True), (7, 2, True), (4, 3, False), (64, 10, True)])
def test_sinc_256_persistent_loop_same_bits(F, B, n_iter, periodic):
    """The persistent loop (schedule 2) runs the column-block and row-step arithmetic of the
    launch-per-pass loop: bit-identical phases and extended slopes."""
    import dataclasses
    _flush(f"[gpu] sinc 256 persistent vs per pass B={B} n_iter={n_iter} periodic={periodic}")
    w = dataclasses.replace(I.ELT_128, model="sinc", config_id=8)
    x = torch.from_numpy(I.make_batch(w, B, dtype=np.float32)).cuda()
    p = O.Params(n_sub=128, n_grid=256, n_iter=n_iter, periodic=periodic, d=39.0 / 128, model="sinc")
    plan = _plan(F, p, I.pupil_mask(128), B)
    res = {}
    for sc in (0, 2):
        plan.set_schedule(sc)
        res[sc] = (plan.reconstruct(x), plan.extend(x))
    assert torch.isfinite(res[2][0]).all()
    assert torch.equal(res[0][0], res[2][0]) and torch.equal(res[0][1], res[2][1])
    plan.close()


@pytest.mark.parametrize("n,periodic", [(100, True), (200, False)])
def test_sinc_256_persistent_loop_other_windows(F, n, periodic):
    """The lenslet-averaging persistent loop on other lenslet counts of the 256 x 256 grid, random
    masks: against the oracle, and bit for bit against one launch per pass."""
    _flush(f"[gpu] sinc 256 persistent n={n} periodic={periodic}")
    mask = I.random_mask(n, seed=n + 3)
    slopes = I.random_slopes(3, n, seed=n + 4).astype(np.float32)
    p = O.Params(n_sub=n, n_grid=256, n_iter=5, periodic=periodic, d=39.0 / n, model="sinc")
    plan = _plan(F, p, mask, 3)
    x = torch.from_numpy(slopes).cuda()
    plan.set_schedule(0)
    ref = plan.reconstruct(x)
    plan.set_schedule(2)
    got = plan.reconstruct(x)
    assert torch.equal(got, ref)
    g = got.cpu().numpy().astype(np.float64)
    for b in range(3):
        assert _rel(g[b], O.reconstruct(slopes[b].astype(np.float64), mask, p)) <= 1e-5
    plan.close()


def test_sinc_256_persistent_loop_watchdog(F):
    """A one-poll wait limit makes the persistent loop give up (forced from the host): every frame
    NaN or every frame exact, and the next call with the default limit exact."""
    import dataclasses
    _flush("[gpu] sinc 256 persistent loop watchdog")
    B = 128
    w = dataclasses.replace(I.ELT_128, model="sinc", config_id=9)
    base = I.make_batch(w, 8, dtype=np.float32)
    x = torch.from_numpy(np.ascontiguousarray(np.concatenate([base] * (B // 8)))).cuda()
    p = O.Params(n_sub=128, n_grid=256, n_iter=10, periodic=True, d=39.0 / 128, model="sinc")
    plan = _plan(F, p, I.pupil_mask(128), B)
    ref = plan.reconstruct(x).cpu().numpy()
    plan.set_schedule(2)
    plan.set_wait_limit(1)
    gave_up = 0
    for _ in range(3):
        got = plan.reconstruct(x).cpu().numpy()
        if np.isnan(got).all():
            gave_up += 1
        else:
            assert np.array_equal(got, ref)
    assert gave_up > 0
    plan.set_wait_limit(1 << 20)
    assert np.array_equal(plan.reconstruct(x).cpu().numpy(), ref)
    plan.close()


def test_sinc_256_autotune_picks_a_loop_shape(F):
    """The autotuner times the two loop shapes of the lenslet-averaging multi-pass plan (one launch
    per pass, persistent), keeps the faster, and later plans of the shape start from it; the chosen
    shape stays within the oracle's tolerance."""
    _flush("[gpu] sinc 256 autotune")
    p = O.Params(n_sub=128, n_grid=256, n_iter=4, periodic=True, d=39.0 / 128, model="sinc")
    mask = I.pupil_mask(128)
    plan = _plan(F, p, mask, 32)
    assert plan.autotune(32) == 1
    chosen = plan.schedule
    assert chosen in (0, 2)
    with pytest.raises(F.FwrError) as e:
        plan.set_schedule(1)
    assert e.value.status == F.FWR_E_UNSUPPORTED
    plan.close()
    again = _plan(F, p, mask, 4)
    assert again.schedule == chosen
    slopes = I.random_slopes(4, 128, seed=31).astype(np.float32)
    got = again.reconstruct(torch.from_numpy(slopes).cuda()).cpu().numpy().astype(np.float64)
    for b in range(4):
        assert _rel(got[b], O.reconstruct(slopes[b].astype(np.float64), mask, p)) <= 1e-5
    again.close()


@pytest.mark.parametrize("mp_schedule", [0, 2])
def test_sinc_256_in_a_grouped_call(F, mp_schedule):
    """A multi-pass sinc plan beside an on-chip sinc plan and a Fried plan in one grouped call gives
    the bits of the individual calls, with the multi-pass plans on either loop shape (beside other
    items they run one launch per pass: the same bits)."""
    _flush(f"[gpu] grouped call with the sinc multi-pass path, schedule {mp_schedule}")
    items = []
    for n, N, model in ((128, 256, "sinc"), (40, 80, "sinc"), (128, 256, "fried")):
        plan = F.Plan(n, N, I.pupil_mask(n), n_iter=3, periodic=True, max_batch=2, d=8.0 / n, model=model)
        if N == 256:
            plan.set_schedule(mp_schedule)
        x = torch.from_numpy(I.random_slopes(2, n, seed=n + N).astype(np.float32)).cuda()
        items.append((plan, x, torch.empty((2, n + 1, n + 1), device="cuda"), None, None))
    F.reconstruct_group(items)
    torch.cuda.synchronize()
    for plan, x, o, _, _ in items:
        assert torch.equal(o, plan.reconstruct(x)), (plan.n_sub, plan.model)
        plan.close()


@pytest.mark.parametrize("n,N", [(40, 80), (128, 256)])
def test_sinc_non_finite_frame_is_isolated(F, n, N):
    """Frames are not paired under the lenslet-averaging model: a frame with a non-finite
    in-pupil slope gets NaN phases and every other frame is unchanged, bit for bit."""
    _flush(f"[gpu] sinc isolation n={n} N={N}")
    mask = I.pupil_mask(n)
    slopes = (I.make_batch(I.SPHERE_40_SINC, 3, start=40, dtype=np.float32) if n == 40
              else np.random.default_rng(5).standard_normal((3, 2, n, n)).astype(np.float32))
    p = O.Params(n_sub=n, n_grid=N, n_iter=3, periodic=True, d=8.0 / n, model="sinc")
    cell = (n // 2, 3)
    assert mask[cell] == 1
    bad, ref = slopes.copy(), slopes.copy()
    bad[1, 1][cell] = np.inf
    ref[1, 1][cell] = 0.0
    plan = _plan(F, p, mask, 3)
    gb = plan.reconstruct(torch.from_numpy(bad).cuda()).cpu().numpy()
    gr = plan.reconstruct(torch.from_numpy(ref).cuda()).cpu().numpy()
    plan.close()
    assert np.isnan(gb[1]).all()
    assert np.array_equal(gb[[0, 2]], gr[[0, 2]])
