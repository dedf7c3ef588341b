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
