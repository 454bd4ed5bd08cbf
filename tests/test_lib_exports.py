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


def test_tj_lattice_descriptor_checks_without_device():
    """svmc_create rejects t-J descriptor errors before it touches a device:
    J or h_pin on a Hubbard lattice, a model flag outside {0, 1}, a nonzero
    reserved field, more electrons than sites and a non-finite J are invalid;
    a t-J lattice above 2048 sites (the exchange codes' range) is not
    supported."""
    from paper_2604_25775_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    h = ctypes.c_void_p()
    m = _lib.Model(2, 8, 0, 0, 32, 3, 0, 0)

    def create(**kw):
        f = dict(Lx=8, Ly=4, pbc_x=0, pbc_y=1, t=1.0, tp=0.2, U=0.0, n_up=14, n_dn=14, J=1.0 / 3.0, h_pin=0.5,
                 tj=1, reserved=0)
        f.update(kw)
        lat = (_lib.Lattice * 1)(_lib.Lattice(*[f[k] for k, _ in _lib.Lattice._fields_]))
        return lib.svmc_create(lat, 1, ctypes.byref(m), ctypes.byref(h))

    assert create(tj=0) == 1
    assert create(tj=0, J=0.0) == 1                  # h_pin without the t-J model
    assert create(tj=2) == 1
    assert create(reserved=1) == 1
    assert create(n_up=17, n_dn=16) == 1
    assert create(J=float("inf")) == 1
    assert create(Lx=64, Ly=40, n_up=100, n_dn=100) == 5
    assert not h.value
