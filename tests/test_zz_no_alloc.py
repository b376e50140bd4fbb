"""The allocation-free learned call (fwr_reconstruct_learned_noalloc) against the allocating one,
through the C ABI (needs an MI355X)."""
import ctypes
import os
import sys

import numpy as np
import pytest

from paper_1705_04298_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_noalloc_learned_call_matches_the_allocating_one():
    """Two calls in a row, the second smaller: 2048 frames that all fall back (three chunks of the
    fixed workspace at 40x40), then 100 frames with the median residual as threshold.  Phases,
    residuals, start values and the count of recomputed frames equal those of
    fwr_reconstruct_learned bit for bit; an empty batch writes the count 0."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_04298_amd import fwr as F
    from paper_1705_04298_amd import learned as L
    F.load()
    params = np.load(os.path.join(os.path.dirname(L.__file__), "weights", "cnn_40x40_fried.npz"))["params"]
    mask = I.pupil_mask(40)
    Bmax = 2048
    net = F.CNN(40, 80, mask, max_batch=Bmax, input_scale=L.INPUT_SCALE)
    net.set_params(params)
    plan = F.Plan(40, 80, mask, n_iter=2, periodic=True, max_batch=Bmax)
    plain = F.Plan(40, 80, mask, n_iter=10, periodic=True, max_batch=Bmax)
    slopes, _ = L.make_frames(Bmax, seed0=93_000)
    x_all = torch.from_numpy(slopes).cuda()
    d_count = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    for B, quantile in ((2048, None), (100, 0.5)):
        _flush(f"[gpu] no-alloc learned call B={B}")
        x = x_all[:B].contiguous()
        outs = {}
        for which in ("alloc", "noalloc"):
            start = torch.full((B, 2, 80, 80), 3.0, device="cuda")
            phase = torch.full((B, 41, 41), 3.0, device="cuda")
            resid = torch.full((B,), 3.0, device="cuda")
            if which == "alloc":
                if quantile is None:
                    thr = -1.0
                else:
                    r0 = torch.empty(B, device="cuda")
                    plan.reconstruct(x, start=net.forward(x), resid=r0)
                    thr = float(np.quantile(r0.cpu().numpy(), quantile))
                count = ctypes.c_int32(-1)
                st = F.fwr_reconstruct_learned(plan.handle, plain.handle, net._h, x.data_ptr(), start.data_ptr(),
                                               phase.data_ptr(), resid.data_ptr(), thr, B, ctypes.byref(count))
                n_fall = count.value
            else:
                st = F.fwr_reconstruct_learned_noalloc(plan.handle, plain.handle, net._h, x.data_ptr(),
                                                       start.data_ptr(), phase.data_ptr(), resid.data_ptr(), thr,
                                                       B, d_count.data_ptr())
                torch.cuda.synchronize()
                n_fall = int(d_count.item())
            assert st == F.FWR_OK, (which, st)
            torch.cuda.synchronize()
            outs[which] = (start, phase, resid, n_fall)
        a, b = outs["alloc"], outs["noalloc"]
        assert a[3] == b[3], (a[3], b[3])
        assert a[3] == (B if quantile is None else int((a[2] > thr).sum()))
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    st = F.fwr_reconstruct_learned_noalloc(plan.handle, plain.handle, net._h, 0, 0, 0, 0, 0.1, 0, d_count.data_ptr())
    torch.cuda.synchronize()
    assert st == F.FWR_OK and int(d_count.item()) == 0
    for h in (net, plan, plain):
        h.close()
