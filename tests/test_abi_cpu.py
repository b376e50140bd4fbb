"""The C-ABI library loads and exports every symbol the header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fwr.h")
LIB = os.path.join(ROOT, "paper_1705_04298_amd", "libfwr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fwr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("fwr_plan", "fwr_extend", "fwr_reconstruct", "fwr_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwr.so not built")
def test_host_side_validation_without_gpu():
    """Status strings and NULL checks run on the host only."""
    from paper_1705_04298_amd import fwr as F
    lib = F.load()
    assert lib.fwr_status_string(F.FWR_E_INVAL).decode() == "invalid argument"
    h = ctypes.c_void_p()
    assert lib.fwr_plan(None, ctypes.byref(h)) == F.FWR_E_INVAL
    assert lib.fwr_destroy(None) == F.FWR_E_STATE
    assert F.fwr_reconstruct_learned(None, None, None, 0, 0, 0, 0, 0.0, 1) == F.FWR_E_STATE
    # launch-shape calls on a NULL plan
    assert lib.fwr_plan_set_schedule(None, 2) == F.FWR_E_STATE
    assert lib.fwr_plan_set_wait_limit(None, 100) == F.FWR_E_STATE
    assert lib.fwr_reconstruct_group(None, 0, None) == F.FWR_OK  # (no items: nothing to do)
    assert lib.fwr_reconstruct_group(None, 1, None) == F.FWR_E_INVAL
    assert sorted(F.EXPORTED) == sorted(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwr.so not built")
def test_alpha_map_must_be_even_and_non_negative():
    """The plan rejects a map of W_eta/W_phi that is not even (or negative) before any device work."""
    import numpy as np
    from paper_1705_04298_amd import fwr as F
    lib = F.load()
    n, N = 4, 8
    mask = np.ones((n, n), dtype=np.uint8)
    for bad in ("odd", "negative"):
        alpha = np.ones((N, N))
        if bad == "odd":
            alpha[1, 2] = 2.0             # alpha[7, 6] stays 1
        else:
            alpha[0, 0] = -1.0
        p = F.FwrParams()
        p.n_sub, p.n_grid, p.n_iter, p.periodic, p.max_batch, p.gamma = n, N, 2, 1, 1, 1.0
        p.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        p.alpha_map = alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        assert lib.fwr_plan(ctypes.byref(p), ctypes.byref(h)) == F.FWR_E_INVAL, bad


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwr.so not built")
def test_cnn_create_validates_on_the_host():
    import numpy as np
    from paper_1705_04298_amd import fwr as F
    lib = F.load()
    mask = np.ones((6, 6), dtype=np.uint8)
    mp = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    h = ctypes.c_void_p()
    assert lib.fwr_cnn_create(6, 12, mp, 1, 0.5, 0, None, ctypes.byref(h)) == F.FWR_E_UNSUPPORTED  # N < 16
    assert lib.fwr_cnn_create(6, 20, mp, 1, 0.5, 0, None, ctypes.byref(h)) == F.FWR_E_UNSUPPORTED  # N^2 % 64
    assert lib.fwr_cnn_create(6, 16, None, 1, 0.5, 0, None, ctypes.byref(h)) == F.FWR_E_INVAL
    assert lib.fwr_cnn_create(6, 16, mp, 0, 0.5, 0, None, ctypes.byref(h)) == F.FWR_E_INVAL
    assert lib.fwr_cnn_create(6, 16, mp, 1, 0.0, 0, None, ctypes.byref(h)) == F.FWR_E_INVAL
    assert lib.fwr_cnn_create(6, 15, mp, 1, 0.5, 0, None, ctypes.byref(h)) == F.FWR_E_INVAL       # N - n odd
    assert lib.fwr_cnn_forward(None, None, None, 1) == F.FWR_E_STATE
    assert lib.fwr_cnn_destroy(None) == F.FWR_E_STATE


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwr.so not built")
@pytest.mark.parametrize("model", [0, 1])
def test_plan_rejects_bad_physical_parameters_for_both_models(model):
    """Eq. 3's W_eta / W_phi needs d > 0, r0 > 0, L0 > 0, sigma^2 >= 0 and gamma >= 0: both slope
    models (Fried 0, lenslet averaging 1) reject other values before any device work."""
    import numpy as np
    from paper_1705_04298_amd import fwr as F
    lib = F.load()
    n, N = 40, 80
    mask = np.ones((n, n), dtype=np.uint8)
    good = dict(gamma=1.0, noise_var=0.0025, r0=0.15, L0=25.0, d=0.2)
    for field, value in (("d", 0.0), ("r0", -1.0), ("L0", 0.0), ("noise_var", -1e-3), ("gamma", -1.0),
                         ("d", float("nan"))):
        p = F.FwrParams()
        p.n_sub, p.n_grid, p.n_iter, p.periodic, p.max_batch, p.model = n, N, 2, 1, 1, model
        for k, v in good.items():
            setattr(p, k, v)
        setattr(p, field, value)
        p.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        h = ctypes.c_void_p()
        assert lib.fwr_plan(ctypes.byref(p), ctypes.byref(h)) == F.FWR_E_INVAL, (model, field, value)
        assert not h.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwr.so not built")
def test_pixel_size_correction_is_checked():
    """d_px (the d - d_px remark after Eq. 4) belongs to the lenslet-averaging model: 0 <= d_px < d
    there; any non-zero value on a Fried plan is unsupported.  No device work on these paths."""
    import numpy as np
    from paper_1705_04298_amd import fwr as F
    lib = F.load()
    n, N = 40, 80
    mask = np.ones((n, n), dtype=np.uint8)
    for model, d_px, want in ((1, -0.01, F.FWR_E_INVAL), (1, 0.2, F.FWR_E_INVAL), (1, 0.3, F.FWR_E_INVAL),
                              (1, float("nan"), F.FWR_E_INVAL), (0, 0.02, F.FWR_E_UNSUPPORTED)):
        p = F.FwrParams()
        p.n_sub, p.n_grid, p.n_iter, p.periodic, p.max_batch, p.model = n, N, 2, 1, 1, model
        p.gamma, p.noise_var, p.r0, p.L0, p.d, p.d_px = 1.0, 0.0025, 0.15, 25.0, 0.2, d_px
        p.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        h = ctypes.c_void_p()
        assert lib.fwr_plan(ctypes.byref(p), ctypes.byref(h)) == want, (model, d_px)
