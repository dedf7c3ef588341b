"""The built HIP library loads on the CPU host and exports every entry point its header declares."""
import ctypes
import os
import re

import pytest

from paper_2006_06823_amd import lddmm_bl as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lddmm_bl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lddmm_\w+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert set(L.EXPORTS) <= set(declared_functions())


def test_library_exports_every_declared_symbol():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, f"missing exports: {missing}"


def test_binding_loads_without_gpu():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built")
    lib = L.load_library()
    assert lib.lddmm_bl_destroy(None) == -1
    # a context-free call records its error text per thread (argument checks run before any HIP call)
    p = L.Params()
    p.dim = 5
    h = ctypes.c_void_p()
    assert lib.lddmm_bl_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert b"dim" in lib.lddmm_bl_last_error(None)
    opts = L.GNOpts(1, 1, 1e-3, 0.0, 0, 0.0)
    assert lib.lddmm_bl_gn_solve_batched(None, 0, None, None, None, ctypes.byref(opts), None, None) == -1
    assert b"count" in lib.lddmm_bl_last_error(None)


def test_report_layout_matches_the_header():
    """The decision log and Jacobian extrema sit where the header puts them (ctypes mirror)."""
    text = open(HEADER).read()
    assert "#define LDDMM_BL_LOG_MAX 64" in text and L.LOG_MAX == 64
    names = [n for n, _ in L.GNReport._fields_]
    assert names[:11] == ["gn_iters", "pcg_iters_total", "backtracks", "hess_matvecs", "E0", "E", "mse_rel",
                          "grad_inf_rel", "det_min", "det_max", "seconds"]
    assert names[11:] == ["log_count", "log_pcg", "log_negcurv", "log_backtracks"]
    r = L.GNReport()
    r.log_count = 2
    r.log_pcg[0], r.log_negcurv[0], r.log_backtracks[0] = 5, 0, 1
    r.log_pcg[1], r.log_negcurv[1], r.log_backtracks[1] = 3, 1, -1
    assert r.as_dict()["decisions"] == [(5, 0, 1), (3, 1, -1)]


def test_committed_warm_start_weights_match_the_architecture():
    import os
    import numpy as np
    from paper_2006_06823_amd import learned as LW
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2006_06823_amd", "weights", "warmstart_v1_128.npz")
    z = np.load(path, allow_pickle=False)
    ch = [int(c) for c in z["channels"]]
    assert tuple(ch) == LW.CHANNELS and int(z["in_size"]) == LW.IN_SIZE
    n, cin = 0, 2
    for c in ch:
        n += c * cin * 27 + c
        cin = c
    n += 3 * cin + 3
    assert z["params"].shape == (n,) and z["params"].dtype == np.float32
    assert np.isfinite(z["params"]).all()


def test_autotuner_cache_round_trip_and_rejections():
    """The tuner cache is host state: no GPU is needed to set, read and reject keys."""
    n = L.tune_candidates("brick")
    assert n == 8
    assert L.tune_candidates("nope") == 0
    key = "brick:7x9x11:gs2"
    assert L.tune_get(key) == -1
    L.tune_set(key, n - 1)
    assert L.tune_get(key) == n - 1
    L.tune_set(key, -1)
    assert L.tune_get(key) == -1
    nd = L.tune_candidates("dft")
    assert nd == 6
    dkey = "dft:expand_bf16:M96:L32:C1024"
    assert L.tune_get(dkey) == -1
    L.tune_set(dkey, nd - 1)
    assert L.tune_get(dkey) == nd - 1
    assert L.tune_table()[dkey] == nd - 1
    L.tune_set(dkey, -1)
    assert L.tune_get(dkey) == -1
    for bad_key, bad_choice in [("brick:7x9x11:gs2", n), ("brick:7x9x11:gs2", -2), (dkey, nd), ("fft:7x9x11", 0)]:
        with pytest.raises(L.LddmmError):
            L.tune_set(bad_key, bad_choice)
    assert L.brick_tune_keys((40, 36, 44)) == ["brick:40x36x44:gs1", "brick:40x36x44:gs2", "brick:40x36x44:gs3"]
    assert L.brick_tune_keys((48, 40))[0] == "brick:1x48x40:gs1"
