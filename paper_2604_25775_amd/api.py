"""Python binding of the scalevmc C ABI.  Argument marshalling only: every
step of the computation runs in the HIP library; torch supplies device memory
and the current stream.
"""
from __future__ import annotations

import ctypes as ct
from typing import Sequence

import numpy as np
import torch

from . import _lib

PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3, "f16x2": 4}
ACT = {"tanh": 0, "silu": 1}
PATH = {"lowrank": 0, "full": 1}


def _ptr(t: torch.Tensor | None):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def pack_params(params, lattices) -> np.ndarray:
    """Flat FP64 parameter vector in the library's layout:
    embed | conv_w | conv_b | mlp_w | mlp_b | per lattice: W_up | W_dn | b_up
    | b_dn, where embed is the shared [4, C] table or, when params.embed_site
    is set, the per-site tables [N_l, 4, C] of every lattice in order, and
    mlp_w / mlp_b the site-wise layers ([M][C][C], [M][C]; empty when M = 0)."""
    site = getattr(params, "embed_site", None)
    emb = ([np.asarray(e, np.float64).ravel() for e in site] if site is not None
           else [np.asarray(params.embed, np.float64).ravel()])
    parts = emb + [
             np.asarray(params.conv_w, np.float64).ravel(),
             np.asarray(params.conv_b, np.float64).ravel()]
    parts += [np.asarray(w, np.float64).ravel() for w in (getattr(params, "mlp_w", None) or [])]
    parts += [np.asarray(b, np.float64).ravel() for b in (getattr(params, "mlp_b", None) or [])]
    for li, _ in enumerate(lattices):
        parts += [np.asarray(params.proj_w[li][0], np.float64).ravel(),
                  np.asarray(params.proj_w[li][1], np.float64).ravel(),
                  np.asarray(params.proj_b[li][0], np.float64).ravel(),
                  np.asarray(params.proj_b[li][1], np.float64).ravel()]
    return np.concatenate(parts)


class ScaleVMC:
    """One library context: lattices, network shape, parameters and walkers."""

    def __init__(self, lattices: Sequence, n_conv: int, channels: int, act: str = "tanh",
                 conv_prec: str = "f64", refresh_every: int = 32, device: str = "cuda:0",
                 per_site_embed: bool = False, ksize: int = 3, n_mlp: int = 0):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.lattices = list(lattices)
        arr = (_lib.Lattice * len(self.lattices))()
        for k, l in enumerate(self.lattices):
            arr[k] = _lib.Lattice(l.Lx, l.Ly, int(l.pbc_x), int(l.pbc_y), float(l.t), float(l.tp),
                                  float(l.U), l.n_up, l.n_dn, float(getattr(l, "J", 0.0)),
                                  float(getattr(l, "h_pin", 0.0)), int(getattr(l, "tj", 0)), 0)
        m = _lib.Model(n_conv, channels, ACT[act], PREC[conv_prec], refresh_every, ksize, n_mlp,
                       int(bool(per_site_embed)))
        h = ct.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.svmc_create(arr, len(self.lattices), ct.byref(m), ct.byref(h))
        if st != 0:
            raise _lib.SvmcError(st, "svmc_create")
        self.h = h
        self.n_conv, self.channels, self.conv_prec = n_conv, channels, conv_prec
        # bumped by every call that changes parameters or configurations
        # (LogPsi.backward checks that its forward's state is still held)
        self.state_version = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.svmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != 0:
            msg = self.lib.svmc_last_error(self.h)
            raise _lib.SvmcError(st, f"{what}: {msg.decode() if msg else ''}")

    # ---- sizes -----------------------------------------------------------
    @property
    def num_params(self) -> int:
        return int(self.lib.svmc_num_params(self.h))

    @property
    def num_walkers(self) -> int:
        return int(self.lib.svmc_num_walkers(self.h))

    @property
    def max_hops(self) -> int:
        return int(self.lib.svmc_max_hops(self.h))

    @property
    def max_electrons(self) -> int:
        return int(self.lib.svmc_max_electrons(self.h))

    # ---- calls -------------------------------------------------------------
    def set_params(self, theta: torch.Tensor, base: Sequence[torch.Tensor]):
        assert theta.dtype == torch.float64 and theta.is_cuda and theta.numel() == self.num_params
        self._theta = theta.contiguous()
        self._base = [b.to(self.device, torch.float64).contiguous() for b in base]
        arr = (ct.c_void_p * len(self._base))(*[b.data_ptr() for b in self._base])
        self.state_version += 1
        self._check(self.lib.svmc_set_params(self.h, _ptr(self._theta), arr, _stream()), "set_params")

    def set_params_from(self, params):
        """Upload a workloads.Params (FP64 numpy) object."""
        theta = torch.from_numpy(pack_params(params, self.lattices)).to(self.device)
        base = []
        for li, _ in enumerate(self.lattices):
            base.append(torch.from_numpy(np.concatenate([params.base[li][0].ravel(),
                                                         params.base[li][1].ravel()])).to(self.device))
        self.set_params(theta, base)

    def load_walkers(self, counts: Sequence[int], occ: torch.Tensor):
        occ = occ.to(self.device, torch.int8).contiguous()
        self._occ_in = occ
        c = (ct.c_int64 * len(counts))(*[int(x) for x in counts])
        self.state_version += 1
        self._check(self.lib.svmc_load_walkers(self.h, c, _ptr(occ), _stream()), "load_walkers")

    def log_psi(self):
        W = self.num_walkers
        sign = torch.empty(W, dtype=torch.float64, device=self.device)
        la = torch.empty(W, dtype=torch.float64, device=self.device)
        self._check(self.lib.svmc_log_psi(self.h, _ptr(sign), _ptr(la), _stream()), "log_psi")
        return sign, la

    def prepare(self):
        self._check(self.lib.svmc_prepare(self.h, _stream()), "prepare")

    def local_energy(self, path: str = "lowrank", ratios: bool = False, out=None):
        W = self.num_walkers
        eloc = torch.empty(W, dtype=torch.float64, device=self.device) if out is None else out
        nh = code = rat = None
        if ratios:
            H = self.max_hops
            nh = torch.zeros(W, dtype=torch.int32, device=self.device)
            code = torch.full((W, H), -1, dtype=torch.int32, device=self.device)
            rat = torch.full((W, H), float("nan"), dtype=torch.float64, device=self.device)
        self._check(self.lib.svmc_local_energy(self.h, PATH[path], _ptr(eloc), _ptr(nh), _ptr(code),
                                               _ptr(rat), _stream()), "local_energy")
        return (eloc, nh, code, rat) if ratios else eloc

    def local_energy_noalloc(self, out: torch.Tensor):
        """Low-rank local energies into `out` (float64 [W]) through the
        allocation-free entry point (svmc_local_energy_noalloc)."""
        assert out.dtype == torch.float64 and out.is_cuda and out.numel() >= self.num_walkers
        self._check(self.lib.svmc_local_energy_noalloc(self.h, _ptr(out), _stream()), "local_energy_noalloc")
        return out

    def sweep(self, n_sweeps: int, seed: int, step0: int, n_accept: torch.Tensor | None = None):
        if n_accept is None:
            n_accept = torch.zeros(self.num_walkers, dtype=torch.int64, device=self.device)
        self.state_version += 1
        self._check(self.lib.svmc_sweep(self.h, int(n_sweeps), ct.c_uint64(seed), ct.c_uint64(step0),
                                        _ptr(n_accept), _stream()), "sweep")
        return n_accept

    def sweep_async(self, n_sweeps: int, seed: int, step0: torch.Tensor, n_accept: torch.Tensor):
        """Graph-capturable sweep (svmc_sweep_async): step0 is a device uint64
        scalar read at run time (torch.int64 tensor of one element)."""
        self.state_version += 1
        self._check(self.lib.svmc_sweep_async(self.h, int(n_sweeps), ct.c_uint64(seed), _ptr(step0),
                                              _ptr(n_accept), _stream()), "sweep_async")
        return n_accept

    def refresh(self):
        self._check(self.lib.svmc_refresh(self.h, _stream()), "refresh")

    def state(self):
        tot = sum(int(c) * l.Lx * l.Ly for c, l in zip(self._counts, self.lattices))
        occ = torch.empty(tot, dtype=torch.int8, device=self.device)
        pos = torch.empty((self.num_walkers, 2, self.max_electrons), dtype=torch.int16, device=self.device)
        self._check(self.lib.svmc_get_state(self.h, _ptr(occ), _ptr(pos), _stream()), "get_state")
        return occ, pos

    def grad_logpsi(self, vjp: torch.Tensor | None = None, out_prec: str = "f64"):
        """Per-walker Jacobian [W, n_params] (vjp None) or the VJP [n_params],
        as float64 or float32 (out_prec "f64" | "f32")."""
        dt = {"f64": torch.float64, "f32": torch.float32}[out_prec]
        if vjp is None:
            out = torch.empty((self.num_walkers, self.num_params), dtype=dt, device=self.device)
        else:
            vjp = vjp.to(self.device, torch.float64).contiguous()
            out = torch.empty(self.num_params, dtype=dt, device=self.device)
        self._check(self.lib.svmc_grad_logpsi(self.h, _ptr(vjp), _ptr(out), PREC[out_prec], _stream()),
                    "grad_logpsi")
        return out

    def flags(self):
        f = torch.empty(self.num_walkers, dtype=torch.int32, device=self.device)
        self._check(self.lib.svmc_walker_flags(self.h, _ptr(f), _stream()), "walker_flags")
        return f

    def tune(self, cache_path: str | None = None) -> int:
        """Pick the fastest local-energy launch shape for the loaded walkers
        (svmc_tune); returns the chosen slices per walker."""
        out = ct.c_int32(0)
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.svmc_tune(self.h, path, ct.byref(out), _stream()), "tune")
        return int(out.value)

    def set_launch(self, slices: int, row_form_max: int = 16):
        """Low-rank E_loc launch shape (svmc_set_launch)."""
        ln = _lib.Launch(int(slices), int(row_form_max))
        self._check(self.lib.svmc_set_launch(self.h, ct.byref(ln)), "set_launch")

    def get_launch(self) -> dict:
        ln = _lib.Launch(0, 0)
        self._check(self.lib.svmc_get_launch(self.h, ct.byref(ln)), "get_launch")
        return {"slices": int(ln.slices), "row_form_max": int(ln.row_form_max)}

    def set_symmetry(self, group, chi):
        """Symmetry group for the projected amplitude (svmc_set_symmetry):
        group = [(perm, flip)] with the identity first, chi the characters."""
        N = self.lattices[0].N
        n = len(group)
        perm = np.ascontiguousarray(np.array([list(p) for p, _ in group], dtype=np.int32).reshape(n, N))
        flip = np.ascontiguousarray(np.array([int(bool(f)) for _, f in group], dtype=np.int32))
        ch = np.ascontiguousarray(np.array(chi, dtype=np.float64))
        self._check(self.lib.svmc_set_symmetry(self.h, n, perm.ctypes.data, flip.ctypes.data, ch.ctypes.data),
                    "set_symmetry")
        self._sym_n = n

    def sym_expand(self, occ: torch.Tensor) -> torch.Tensor:
        """[W, N] int8 device occupations -> their copies [W n_g, N] (svmc_sym_expand)."""
        N = self.lattices[0].N
        occ = occ.to(self.device, torch.int8).contiguous().reshape(-1, N)
        out = torch.empty(occ.shape[0] * self._sym_n, N, dtype=torch.int8, device=self.device)
        self._check(self.lib.svmc_sym_expand(self.h, occ.shape[0], _ptr(occ), _ptr(out), _stream()), "sym_expand")
        return out

    def local_energy_sym(self, weights: bool = False):
        """(E_sym, sign, log|psi_sym|) [W / n_g] of the loaded symmetric batch
        (svmc_local_energy_sym), and the copies' weights [W] if asked."""
        K = self.num_walkers // self._sym_n
        e = torch.empty(K, dtype=torch.float64, device=self.device)
        sg = torch.empty(K, dtype=torch.float64, device=self.device)
        la = torch.empty(K, dtype=torch.float64, device=self.device)
        wt = torch.empty(self.num_walkers, dtype=torch.float64, device=self.device) if weights else None
        self._check(self.lib.svmc_local_energy_sym(self.h, _ptr(e), _ptr(sg), _ptr(la), _ptr(wt), _stream()),
                    "local_energy_sym")
        return (e, sg, la, wt) if weights else (e, sg, la)

    def sweep_sym(self, n_sweeps: int, seed: int, step0: int):
        """Metropolis sweeps of |psi_sym|^2 (svmc_sweep_sym); accepted moves per copy."""
        n_accept = torch.zeros(self.num_walkers, dtype=torch.int64, device=self.device)
        self.state_version += 1
        self._check(self.lib.svmc_sweep_sym(self.h, int(n_sweeps), ct.c_uint64(seed), ct.c_uint64(step0),
                                            _ptr(n_accept), _stream()), "sweep_sym")
        return n_accept

    def update_params(self, theta: torch.Tensor):
        """Upload a new flat parameter vector (same base orbitals) and rebuild
        the walkers' caches at their current configurations."""
        occ = None
        if getattr(self, "_counts", None):
            occ, _ = self.state()
        self.set_params(theta.detach().to(self.device, torch.float64), self._base)
        if occ is not None:
            self.load_walkers(self._counts, occ)

    # convenience: remember counts for state()
    def load(self, counts: Sequence[int], occ):
        self._counts = list(counts)
        if isinstance(occ, np.ndarray):
            occ = torch.from_numpy(np.ascontiguousarray(occ).reshape(-1))
        self.load_walkers(counts, occ)


class LogPsi(torch.autograd.Function):
    """log|psi| [W] of the walkers held by a ScaleVMC as a differentiable
    function of the flat parameter vector theta (layout of pack_params).
    Forward uploads theta and rebuilds the caches at the walkers' current
    configurations; backward asks the library for sum_w g[w] d log|psi_w| /
    d theta (svmc_grad_logpsi with VJP weights g).  The gradient is taken at
    the parameters and configurations the ScaleVMC holds, so backward raises
    if they changed after this forward (set_params, load, sweep, or another
    forward).

        la = LogPsi.apply(theta, vmc)
    """

    @staticmethod
    def forward(ctx, theta, vmc):
        vmc.update_params(theta)
        _, la = vmc.log_psi()
        ctx.vmc = vmc
        ctx.version = vmc.state_version
        return la

    @staticmethod
    def backward(ctx, g):
        if ctx.vmc.state_version != ctx.version:
            raise RuntimeError("LogPsi.backward: the ScaleVMC's parameters or walkers changed after this "
                               "forward (sweep, set_params, load or another LogPsi forward); the gradient "
                               "would belong to another state")
        return ctx.vmc.grad_logpsi(g.contiguous()).to(g.dtype), None
