"""The comparison (Hudgin) extension on the GPU vs the oracle (needs an MI355X): copied cells
bit for bit, the Eq. 5 column / row to float rounding, and the phase reconstructed from it."""
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


@pytest.mark.parametrize("n,N", [(40, 80), (24, 48), (12, 24), (64, 128), (78, 80)])
def test_hudgin_extension_and_phase(F, n, N):
    print(f"[gpu] hudgin n={n} N={N}", flush=True)
    sys.stdout.flush()
    mask = I.pupil_mask(n)
    w = I.Workload(n_sub=n, diameter=8.0, screen_size=256)
    slopes = I.make_batch(w, 3, start=50, dtype=np.float32)
    plan0 = F.Plan(n, N, mask, n_iter=0, periodic=False, d=8.0 / n, max_batch=3)
    x = torch.from_numpy(slopes).cuda()
    ext = plan0.hudgin_extend(x)
    phase = plan0.reconstruct(x, start=ext).cpu().numpy().astype(np.float64)
    ext = ext.cpu().numpy().astype(np.float64)
    p = O.Params(n_sub=n, n_grid=N, d=8.0 / n)
    for b in range(3):
        s0x, s0y, P = O.padded_measurement(slopes[b].astype(np.float64), mask, N)
        rx, ry = O.hudgin_extend(s0x, s0y, P)
        scale = np.sqrt(np.mean(rx ** 2 + ry ** 2))
        assert np.array_equal(ext[b, 0, :, :N - 1], rx[:, :N - 1])  # copies are exact
        assert np.array_equal(ext[b, 1, :N - 1, :], ry[:N - 1, :])
        assert np.abs(ext[b, 0, :, N - 1] - rx[:, N - 1]).max() <= 1e-5 * scale * N
        assert np.abs(ext[b, 1, N - 1, :] - ry[N - 1, :]).max() <= 1e-5 * scale * N
        want = O.reconstruct_hudgin(slopes[b].astype(np.float64), mask, p)
        err = np.sqrt(np.mean((phase[b] - want) ** 2) / np.mean(want ** 2))
        assert err <= 1e-5, (b, err)
    with pytest.raises(F.FwrError):  # the start path with 0 iterations takes no Eq. 5
        F.Plan(n, N, mask, n_iter=0, periodic=True, max_batch=1).reconstruct(x[:1], start=torch.zeros((1, 2, N, N), device="cuda"))
    plan0.close()
