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


def test_model_descriptor_checks_without_device():
    """svmc_create rejects network shapes before it touches a device: a kernel
    width other than 3 and more than 8 site-wise MLP layers are not built
    (SVMC_ERR_UNSUPPORTED), a negative layer count and a per-site flag
    outside {0, 1} are invalid."""
    from paper_2604_25775_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    lat = (_lib.Lattice * 1)(_lib.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5))
    h = ctypes.c_void_p()

    def create(**kw):
        f = dict(n_conv=2, channels=8, act=0, conv_prec=0, refresh_every=32, ksize=3, n_mlp=0, per_site_embed=0)
        f.update(kw)
        m = _lib.Model(*[f[k] for k, _ in _lib.Model._fields_])
        return lib.svmc_create(lat, 1, ctypes.byref(m), ctypes.byref(h))

    assert create(ksize=5) == 5
    assert create(ksize=1) == 5
    assert create(n_mlp=9) == 5
    assert create(n_mlp=-1) == 1
    assert create(per_site_embed=2) == 1
    assert create(channels=12) == 5
    assert create(refresh_every=0) == 1
    assert not h.value
