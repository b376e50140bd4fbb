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
