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
    assert lib.lddmm_bl_last_error(None) == b"null context"
    assert lib.lddmm_bl_destroy(None) == -1


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
    for bad_key, bad_choice in [("brick:7x9x11:gs2", n), ("brick:7x9x11:gs2", -2), ("dft:7x9x11", 0)]:
        with pytest.raises(L.LddmmError):
            L.tune_set(bad_key, bad_choice)
    assert L.brick_tune_keys((40, 36, 44)) == ["brick:40x36x44:gs1", "brick:40x36x44:gs2", "brick:40x36x44:gs3"]
    assert L.brick_tune_keys((48, 40))[0] == "brick:1x48x40:gs1"
