"""ctypes loader for libscalevmc.so (the C ABI declared in include/scalevmc.h).

There is no fallback: if the library is missing this raises, so nothing can
silently run on another path.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscalevmc.so")

SVMC_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "HIP runtime error",
          4: "call out of order", 5: "unsupported shape"}

EXPORTS = [
    "svmc_create", "svmc_destroy", "svmc_num_params", "svmc_set_params", "svmc_load_walkers",
    "svmc_num_walkers", "svmc_max_hops", "svmc_max_electrons", "svmc_log_psi", "svmc_prepare",
    "svmc_local_energy",
    "svmc_sweep", "svmc_refresh", "svmc_get_state", "svmc_grad_logpsi", "svmc_walker_flags",
    "svmc_status_string", "svmc_last_error", "svmc_tune", "svmc_sweep_async",
    "svmc_local_energy_noalloc", "svmc_set_launch", "svmc_get_launch",
    "svmc_set_symmetry", "svmc_sym_expand", "svmc_local_energy_sym", "svmc_sweep_sym",
]


class Lattice(ct.Structure):
    _fields_ = [("Lx", ct.c_int32), ("Ly", ct.c_int32), ("pbc_x", ct.c_int32), ("pbc_y", ct.c_int32),
                ("t", ct.c_double), ("tp", ct.c_double), ("U", ct.c_double),
                ("n_up", ct.c_int32), ("n_dn", ct.c_int32),
                ("J", ct.c_double), ("h_pin", ct.c_double), ("tj", ct.c_int32), ("reserved", ct.c_int32)]


class Model(ct.Structure):
    _fields_ = [("n_conv", ct.c_int32), ("channels", ct.c_int32), ("act", ct.c_int32),
                ("conv_prec", ct.c_int32), ("refresh_every", ct.c_int32),
                ("ksize", ct.c_int32), ("n_mlp", ct.c_int32), ("per_site_embed", ct.c_int32)]


class Launch(ct.Structure):
    _fields_ = [("slices", ct.c_int32), ("row_form_max", ct.c_int32)]


class SvmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"scalevmc: {STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str | None = None):
    """Load (once) and return the library handle with typed prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with `python -m paper_2604_25775_amd.build`")
    lib = ct.CDLL(p)
    vp, i32, i64, u64, dp = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint64, ct.POINTER(ct.c_double)
    proto = {
        "svmc_create": (i32, [ct.POINTER(Lattice), i32, ct.POINTER(Model), ct.POINTER(vp)]),
        "svmc_destroy": (i32, [vp]),
        "svmc_num_params": (i64, [vp]),
        "svmc_set_params": (i32, [vp, vp, ct.POINTER(vp), vp]),
        "svmc_load_walkers": (i32, [vp, ct.POINTER(i64), vp, vp]),
        "svmc_num_walkers": (i64, [vp]),
        "svmc_max_hops": (i32, [vp]),
        "svmc_max_electrons": (i32, [vp]),
        "svmc_log_psi": (i32, [vp, vp, vp, vp]),
        "svmc_prepare": (i32, [vp, vp]),
        "svmc_local_energy": (i32, [vp, i32, vp, vp, vp, vp, vp]),
        "svmc_sweep": (i32, [vp, i32, u64, u64, vp, vp]),
        "svmc_refresh": (i32, [vp, vp]),
        "svmc_get_state": (i32, [vp, vp, vp, vp]),
        "svmc_grad_logpsi": (i32, [vp, vp, vp, i32, vp]),
        "svmc_walker_flags": (i32, [vp, vp, vp]),
        "svmc_status_string": (ct.c_char_p, [i32]),
        "svmc_last_error": (ct.c_char_p, [vp]),
        "svmc_tune": (i32, [vp, ct.c_char_p, ct.POINTER(i32), vp]),
        "svmc_sweep_async": (i32, [vp, i32, u64, vp, vp, vp]),
        "svmc_local_energy_noalloc": (i32, [vp, vp, vp]),
        "svmc_set_launch": (i32, [vp, ct.POINTER(Launch)]),
        "svmc_get_launch": (i32, [vp, ct.POINTER(Launch)]),
        "svmc_set_symmetry": (i32, [vp, i32, vp, vp, vp]),
        "svmc_sym_expand": (i32, [vp, i64, vp, vp, vp]),
        "svmc_local_energy_sym": (i32, [vp, vp, vp, vp, vp, vp]),
        "svmc_sweep_sym": (i32, [vp, i32, u64, u64, vp, vp]),
    }
    for name, (res, args) in proto.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
