"""The C-ABI library loads on a machine without a GPU and exports every
function that include/scalevmc.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scalevmc.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(svmc_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_list():
    from paper_2604_25775_amd import _lib
    assert set(declared()) == set(_lib.EXPORTS)


def test_library_exports_all_symbols():
    from paper_2604_25775_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [s for s in declared() if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings_without_device():
    from paper_2604_25775_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    assert lib.svmc_status_string(0) == b"ok"
    assert lib.svmc_status_string(5) == b"unsupported shape"
