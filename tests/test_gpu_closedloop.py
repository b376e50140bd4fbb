"""The closed-loop harness against the same loop run with the FP64 oracle as the reconstructor
(needs an MI355X): same turbulence, same noise, residual phase compared at every step."""
import sys

import numpy as np
import pytest

from oracle import fwr_oracle as O
from paper_1705_04298_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("method,n_iter,periodic", [("gerchberg", 2, False), ("gerchberg", 1, True),
                                                     ("hudgin", 0, True)])
def test_loop_follows_the_oracle(method, n_iter, periodic):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_04298_amd import closedloop as CL
    print(f"[gpu] closed loop {method} it={n_iter} periodic={periodic}", flush=True)
    sys.stdout.flush()
    n, N, B, M, steps, gain, sigma = 24, 48, 3, 64, 5, 0.5, 0.05
    scr = np.stack([I.vk_screen(np.random.default_rng([I.SEED_BASE, 70, b]), M, 8.0 / n, 0.15, 25.0)
                    for b in range(B)]).astype(np.float32)
    noise = np.random.default_rng(71).standard_normal((steps, B, 2, n, n)).astype(np.float32) * sigma
    loop = CL.Loop(scr, n_iter=n_iter, periodic=periodic, gain=gain, sigma=sigma, shift=0.3, method=method, n=n, N=N)
    mask = I.pupil_mask(n)
    p = O.Params(n_sub=n, n_grid=N, n_iter=n_iter, periodic=periodic, d=0.2)
    dm = np.zeros((B, n + 1, n + 1))
    for t in range(steps):
        turb = loop.turbulence(t).cpu().numpy().astype(np.float64)
        if t == 0:
            np.testing.assert_allclose(turb, scr[:, : n + 1, : n + 1], atol=1e-5 * np.abs(scr).max())
        if t == 3:  # 0.9 samples of frozen flow: between the unshifted screen and its one-sample roll
            a = scr[:, : n + 1, : n + 1].astype(np.float64)
            b1 = np.roll(scr, -1, axis=2)[:, : n + 1, : n + 1].astype(np.float64)
            assert np.sqrt(np.mean((turb - b1) ** 2)) < np.sqrt(np.mean((turb - a) ** 2))
        res_gpu = loop.step(noise=torch.from_numpy(noise[t]).cuda()).cpu().numpy().astype(np.float64)
        res = turb - dm
        for b in range(B):
            s = np.stack(I.fried_slopes_from_nodes(res[b])) + noise[t, b]
            s = s * mask
            rec = O.reconstruct_hudgin(s, mask, p) if method == "hudgin" else O.reconstruct(s, mask, p)
            dm[b] += gain * rec
        err = np.sqrt(np.mean((res_gpu - res) ** 2) / np.mean(res ** 2))
        assert err <= 1e-5, (t, err)
    loop.close()


def test_fried_slope_model_call():
    """fwr_fried_slopes (the harness's sensor) against the oracle's Fried transfer function applied
    to the node phase embedded in a periodic grid (the stencil touches only window nodes), plus the
    noise, zero on invalid subapertures; FWR_E_UNSUPPORTED on a lenslet-averaging plan."""
    from oracle import fwr_oracle as O
    from paper_1705_04298_amd import fwr
    fwr.load()
    n, N, B = 40, 80, 3
    mask = I.pupil_mask(n)
    rng = np.random.default_rng(8)
    phase = rng.standard_normal((B, n + 1, n + 1)).astype(np.float32)
    noise = (0.1 * rng.standard_normal((B, 2, n, n))).astype(np.float32)
    plan = fwr.Plan(n, N, mask, max_batch=B)
    ph = torch.from_numpy(phase).cuda()
    clean = plan.fried_slopes(ph).cpu().numpy().astype(np.float64)
    noisy = plan.fried_slopes(ph, torch.from_numpy(noise).cuda()).cpu().numpy().astype(np.float64)
    plan.close()
    Gx, Gy = O.fried_model(N)
    m = mask.astype(bool)
    for b in range(B):
        grid = np.zeros((N, N))
        grid[: n + 1, : n + 1] = phase[b]
        F = O.dft2(grid)
        want = [np.real(O.idft2(G * F))[:n, :n] for G in (Gx, Gy)]
        for c in range(2):
            assert np.abs(clean[b, c][m] - want[c][m]).max() < 2e-6
            assert np.all(clean[b, c][~m] == 0) and np.all(noisy[b, c][~m] == 0)
            assert np.abs(noisy[b, c][m] - (want[c][m] + noise[b, c][m])).max() < 2e-6
    sinc = fwr.Plan(n, N, mask, max_batch=B, model="sinc")
    with pytest.raises(fwr.FwrError) as e:
        sinc.fried_slopes(ph)
    assert e.value.status == fwr.FWR_E_UNSUPPORTED
    sinc.close()
