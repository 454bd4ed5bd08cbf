"""Seeded synthetic inputs for the SCALE local-energy hot path.

This module only *generates inputs*: lattice descriptions, random network
parameters, the plane-wave base orbitals and walker occupations.  It holds none
of the method's arithmetic (no features, no determinants, no energies), so the
FP64 oracle and the GPU library can both draw their inputs from it without
sharing any computation.

Workloads follow the paper's Hubbard settings (Sec. III: square lattices at
1/8 hole doping, t = 1, U = 8) with the sizes of the five benchmark
configurations listed in ``CONFIGS``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Sequence

import numpy as np


# --------------------------------------------------------------------------
# descriptions
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Lattice:
    """A Lx x Ly lattice; site index s = x + Lx*y (x fastest).  The Hubbard
    model by default; ``tj`` = 1 selects the t-J model (no doubly occupied
    site, exchange coupling ``J`` on nearest-neighbour bonds, staggered
    pinning field ``h_pin`` on the column x = 0); U is then unused."""
    Lx: int
    Ly: int
    pbc_x: int = 1
    pbc_y: int = 1
    t: float = 1.0
    tp: float = 0.0
    U: float = 8.0
    n_up: int = 1
    n_dn: int = 1
    tj: int = 0
    J: float = 0.0
    h_pin: float = 0.0

    @property
    def N(self) -> int:
        return self.Lx * self.Ly

    @property
    def n_dirs(self) -> int:
        return 8 if self.tp != 0.0 else 4


@dataclass(frozen=True)
class Model:
    """Conv-backflow model shape: ``n_conv`` residual 3x3 conv layers of
    ``channels`` channels, activation ``act`` (tanh | silu)."""
    n_conv: int = 2
    channels: int = 8
    act: str = "tanh"
    conv_prec: str = "f64"          # f64 | f32 | bf16 | bf16x3 | f16x2
    refresh_every: int = 32
    per_site_embed: bool = False    # one embedding table per site (else shared)
    n_mlp: int = 0                  # site-wise C x C layers after the conv stack


@dataclass(frozen=True)
class Workload:
    name: str
    lattices: Sequence[Lattice]
    walkers: Sequence[int]
    model: Model
    sweeps: int = 0
    seed_params: int = 0
    seed_occ: int = 1
    seed_mc: int = 2
    stripe: bool = False
    description: str = ""


CONFIGS = {
    "c1": Workload(
        "c1", [Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)], [256],
        Model(2, 8, "tanh", "f64"), sweeps=20,
        description="Hubbard 4x4 PBC, U=4, 5+5 electrons (closed shell), "
                    "2 conv layers x 8 channels, all FP64"),
    "c2": Workload(
        "c2", [Lattice(8, 8, 1, 1, 1.0, -0.2, 8.0, 28, 28)], [4096],
        Model(4, 16, "tanh", "f32"), sweeps=8,
        description="Hubbard 8x8 PBC, t'=-0.2, U=8, 28+28 (1/8 doping), "
                    "4 conv layers x 16 channels, conv FP32"),
    "c3": Workload(
        "c3", [Lattice(16, 16, 1, 0, 1.0, 0.0, 8.0, 112, 112)], [8192],
        Model(4, 32, "tanh", "bf16"), sweeps=8,
        description="Hubbard 16x16 periodic-x/open-y, U=8, 112+112 "
                    "(1/8 doping), 4 conv layers x 32 channels, BF16 MFMA conv"),
    "c4": Workload(
        "c4", [Lattice(8, 8, 1, 1, 1.0, 0.0, 8.0, 28, 28),
               Lattice(12, 12, 1, 1, 1.0, 0.0, 8.0, 63, 63),
               Lattice(16, 8, 1, 1, 1.0, 0.0, 8.0, 56, 56)],
        [2048, 2048, 2048], Model(4, 24, "tanh", "f32"), sweeps=8,
        description="mixed batch 8x8 / 12x12 / 16x8 PBC, U=8, "
                    "4 conv layers x 24 channels, conv FP32"),
    "c5": Workload(
        "c5", [Lattice(32, 32, 1, 0, 1.0, 0.0, 8.0, 448, 448)], [1024],
        Model(4, 32, "tanh", "bf16"), sweeps=0, stripe=True,
        description="Hubbard 32x32 periodic-x/open-y, U=8, 448+448, "
                    "stripe-seeded, 4 conv layers x 32 channels, BF16 conv"),
    "tj": Workload(
        "tj", [Lattice(16, 8, 0, 1, 1.0, 0.2, 0.0, 56, 56, tj=1, J=1.0 / 3.0, h_pin=0.5)], [8192],
        Model(1, 32, "silu", "f16x2", n_mlp=4), sweeps=8,
        description="t-J 16x8 cylinder (open x, periodic y), J=1/3, t'=0.2, staggered pinning "
                    "field 0.5 on the x=0 column, 56+56 (1/8 doping); one conv layer + four "
                    "site-wise layers x 32 channels, SiLU, f16x2 conv"),
}


def get(name: str, **overrides) -> Workload:
    w = CONFIGS[name]
    return replace(w, **overrides) if overrides else w


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
@dataclass
class Params:
    """Network parameters in FP64.

    embed  [4, C]            state -> feature (state = n_up + 2 n_dn)
    embed_site  None, or per lattice [N, 4, C]: one table per site (used
                             instead of embed)
    conv_w [L, 3, 3, C, C]   (ky, kx, c_in, c_out); tap (ky, kx) reads the
                             neighbour at offset (kx-1, ky-1)
    conv_b [L, C]
    proj_w per lattice: [2][C, N_sigma]   (spin up, spin down)
    proj_b per lattice: [2][N_sigma]
    base   per lattice: [2][N, N_sigma]   (fixed input, not trained)
    mlp_w  None, or [M] of [C, C]  site-wise layers after the conv stack
    mlp_b  None, or [M] of [C]
    """
    embed: np.ndarray
    conv_w: np.ndarray
    conv_b: np.ndarray
    proj_w: List[List[np.ndarray]]
    proj_b: List[List[np.ndarray]]
    base: List[List[np.ndarray]] = field(default_factory=list)
    embed_site: List[np.ndarray] | None = None
    mlp_w: List[np.ndarray] | None = None
    mlp_b: List[np.ndarray] | None = None

    def copy(self) -> "Params":
        return Params(self.embed.copy(), self.conv_w.copy(), self.conv_b.copy(),
                      [[a.copy() for a in p] for p in self.proj_w],
                      [[a.copy() for a in p] for p in self.proj_b],
                      [[a.copy() for a in p] for p in self.base],
                      None if self.embed_site is None else [e.copy() for e in self.embed_site],
                      None if self.mlp_w is None else [w.copy() for w in self.mlp_w],
                      None if self.mlp_b is None else [b.copy() for b in self.mlp_b])


def _axis_modes(L: int, periodic: bool):
    """Real one-dimensional hopping eigenmodes of a chain of length L.

    Returns a list of (c, key, f) with c = cos(k) (single-particle energy of
    the mode is -2 t c), key a deterministic tie-break tuple, and f the
    normalised real mode function on x = 0..L-1.
    """
    x = np.arange(L, dtype=np.float64)
    out = []
    if periodic:
        for m in range(L // 2 + 1):
            k = 2.0 * math.pi * m / L
            c = math.cos(k)
            if m == 0 or (L % 2 == 0 and m == L // 2):
                f = np.cos(k * x)
                out.append((c, (m, 0), f / np.linalg.norm(f)))
            else:
                f = np.cos(k * x)
                g = np.sin(k * x)
                out.append((c, (m, 0), f / np.linalg.norm(f)))
                out.append((c, (m, 1), g / np.linalg.norm(g)))
    else:
        for n in range(1, L + 1):
            c = math.cos(math.pi * n / (L + 1))
            f = np.sin(math.pi * n * (x + 1) / (L + 1))
            out.append((c, (n, 0), f / np.linalg.norm(f)))
    return out


def plane_wave_orbitals(lat: Lattice, n: int) -> np.ndarray:
    """The n lowest real plane-wave (standing-wave on open axes) orbitals of
    the one-body hopping term, as an [N, n] FP64 matrix with orthonormal
    columns.  Degenerate levels are ordered by a fixed key so that open shells
    get a deterministic choice; the result is passed to both implementations
    as data."""
    mx = _axis_modes(lat.Lx, bool(lat.pbc_x))
    my = _axis_modes(lat.Ly, bool(lat.pbc_y))
    cand = []
    for cx, kx, fx in mx:
        for cy, ky, fy in my:
            e = -2.0 * lat.t * (cx + cy) - 4.0 * lat.tp * cx * cy
            cand.append((round(e, 9), kx, ky, fx, fy))
    cand.sort(key=lambda z: (z[0], z[1], z[2]))
    if n > len(cand):
        raise ValueError("more electrons than orbitals")
    cols = []
    for e, kx, ky, fx, fy in cand[:n]:
        # site s = x + Lx*y  ->  outer(fy, fx).ravel()
        cols.append(np.outer(fy, fx).reshape(-1))
    if not cols:                               # a spin without electrons
        return np.zeros((lat.N, 0))
    return np.stack(cols, axis=1)


def random_params(lats: Sequence[Lattice], model: Model, seed: int = 0,
                  backflow: float = 0.1) -> Params:
    """Seeded parameters.  Conv kernels and biases ~ N(0, 0.05^2), embedding
    ~ N(0, 1); the projection is scaled so that the backflow term is about
    ``backflow`` times the magnitude of a base-orbital entry.  With
    model.per_site_embed, per-site embedding tables ~ N(0, 1) are drawn after
    everything else (the other parameters are the same as without); with
    model.n_mlp > 0 the site-wise layers are drawn after that, weights
    ~ N(0, 1/C) (unit-variance outputs) and biases ~ N(0, 0.05^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C, L = model.channels, model.n_conv
    embed = rng.standard_normal((4, C))
    conv_w = 0.05 * rng.standard_normal((L, 3, 3, C, C))
    conv_b = 0.05 * rng.standard_normal((L, C))
    proj_w, proj_b, base = [], [], []
    for lat in lats:
        N = lat.N
        scale = backflow / math.sqrt(C * N)
        pw, pb, bs = [], [], []
        for ns in (lat.n_up, lat.n_dn):
            pw.append(scale * rng.standard_normal((C, ns)))
            pb.append((backflow / math.sqrt(N)) * rng.standard_normal(ns))
            bs.append(plane_wave_orbitals(lat, ns))
        proj_w.append(pw)
        proj_b.append(pb)
        base.append(bs)
    site = None
    if model.per_site_embed:
        site = [rng.standard_normal((lat.N, 4, C)) for lat in lats]
    mw = mb = None
    if model.n_mlp:
        mw = [rng.standard_normal((C, C)) / math.sqrt(C) for _ in range(model.n_mlp)]
        mb = [0.05 * rng.standard_normal(C) for _ in range(model.n_mlp)]
    return Params(embed, conv_w, conv_b, proj_w, proj_b, base, site, mw, mb)


def quantise_params(p: Params, prec: str) -> Params:
    """Round the conv-stack parameters (embedding, kernels, biases) to the
    compute precision with round-to-nearest-even, returned widened to FP64.
    The projection and base orbitals stay FP64."""
    import torch
    q = p.copy()
    if prec == "f64":
        return q
    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "bf16x3": torch.bfloat16, "f16x2": torch.float32}[prec]
    for name in ("embed", "conv_w", "conv_b"):
        a = torch.from_numpy(getattr(q, name)).to(dt).to(torch.float64).numpy()
        setattr(q, name, a)
    if q.embed_site is not None:
        q.embed_site = [torch.from_numpy(e).to(dt).to(torch.float64).numpy() for e in q.embed_site]
    if q.mlp_w is not None:
        # site-wise layers: weights as the conv kernels, biases as the conv biases
        q.mlp_w = [torch.from_numpy(w).to(dt).to(torch.float64).numpy() for w in q.mlp_w]
        q.mlp_b = [torch.from_numpy(b).to(dt).to(torch.float64).numpy() for b in q.mlp_b]
        if prec == "f16x2":
            q.mlp_w = [torch.from_numpy(w).to(torch.bfloat16).to(torch.float16).to(torch.float64).numpy()
                       for w in p.mlp_w]
    if prec == "f16x2":
        # the BF16 conv weights carried in FP16 (exact in FP16's normal range),
        # the embedding as an FP16 pair, FP32 bias
        w16 = torch.from_numpy(p.conv_w).to(torch.bfloat16).to(torch.float16)
        q.conv_w = w16.to(torch.float64).numpy()
        q.embed = f16_pair(q.embed)
        if q.embed_site is not None:
            q.embed_site = [f16_pair(e) for e in q.embed_site]
    return q


def f16_rtz(x: np.ndarray) -> np.ndarray:
    """FP32 values rounded toward zero to FP16 (11 significant bits in FP16's
    normal range, multiples of 2^-24 below it, at most 65504), as FP32."""
    x = np.asarray(x, dtype=np.float32)
    a = np.abs(x)
    bits = a.view(np.uint32) & np.uint32(0xFFFFE000)
    r = np.minimum(bits.view(np.float32), np.float32(65504.0))
    sub = np.trunc(a.astype(np.float64) * 2.0 ** 24) * 2.0 ** -24
    r = np.where(a >= np.float32(2.0 ** -14), r, sub.astype(np.float32))
    return np.copysign(r, x).astype(np.float32)


def f16_pair(x: np.ndarray) -> np.ndarray:
    """FP16 pair value hi + lo of FP32(x) (hi = f16_rtz(x), lo = f16_rtz(x -
    hi)), widened to FP64: the features of the f16x2 mode."""
    x = np.asarray(x, dtype=np.float64).astype(np.float32)
    h = f16_rtz(x)
    lo = f16_rtz((x - h).astype(np.float32))
    return (h.astype(np.float64) + lo.astype(np.float64))


# --------------------------------------------------------------------------
# occupations
# --------------------------------------------------------------------------
def random_occupations(lat: Lattice, n_walkers: int, seed: int = 1) -> np.ndarray:
    """[n_walkers, N] int8, value n_up + 2 n_dn, exact electron counts (for
    the t-J model no site doubly occupied)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = lat.N
    occ = np.zeros((n_walkers, N), dtype=np.int8)
    for w in range(n_walkers):
        if lat.tj:
            perm = rng.permutation(N)
            up, dn = perm[: lat.n_up], perm[lat.n_up: lat.n_up + lat.n_dn]
        else:
            up = rng.permutation(N)[: lat.n_up]
            dn = rng.permutation(N)[: lat.n_dn]
        occ[w, up] += 1
        occ[w, dn] += 2
    return occ


def stripe_occupations(lat: Lattice, n_walkers: int, seed: int = 1,
                       n_shuffle: int | None = None) -> np.ndarray:
    """Filled vertical stripes: empty columns at x = 0 (mod 8), the other
    sites singly occupied with spin sign (-1)^(x + y + floor(x/8)).  Each
    walker then gets ``n_shuffle`` random nearest-neighbour moves of single
    electrons (seeded) so walkers differ."""
    N = lat.N
    base = np.zeros(N, dtype=np.int8)
    for y in range(lat.Ly):
        for x in range(lat.Lx):
            if x % 8 == 0:
                continue
            s = x + lat.Lx * y
            base[s] = 1 if (x + y + x // 8) % 2 == 0 else 2
    n_up = int(np.sum((base & 1) != 0))
    n_dn = int(np.sum((base & 2) != 0))
    if (n_up, n_dn) != (lat.n_up, lat.n_dn):
        raise ValueError(f"stripe pattern has {n_up}+{n_dn} electrons, "
                         f"lattice wants {lat.n_up}+{lat.n_dn}")
    rng = np.random.Generator(np.random.PCG64(seed))
    if n_shuffle is None:
        n_shuffle = N // 4
    occ = np.tile(base, (n_walkers, 1))
    dirs = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    for w in range(n_walkers):
        o = occ[w]
        for _ in range(n_shuffle):
            s = int(rng.integers(N))
            spin = int(rng.integers(2))
            bit = 1 << spin
            if not (o[s] & bit):
                continue
            dx, dy = dirs[int(rng.integers(4))]
            x, y = s % lat.Lx + dx, s // lat.Lx + dy
            if lat.pbc_x:
                x %= lat.Lx
            if lat.pbc_y:
                y %= lat.Ly
            if not (0 <= x < lat.Lx and 0 <= y < lat.Ly):
                continue
            t = x + lat.Lx * y
            if o[t] & bit:
                continue
            o[s] -= bit
            o[t] += bit
    return occ


def symmetry_group(lat: Lattice, gens) -> tuple:
    """A lattice symmetry group and a one-dimensional representation of it,
    generated by ``gens``: a list of (kind, chi) with kind "tx" / "ty"
    (translation by one site along a periodic axis; ("tx", k) form: a tuple
    ("tx", step)), "mx" / "my" (mirror x -> Lx-1-x, y -> Ly-1-y) or "flip"
    (exchange of the two spins), chi its character (+1 or -1).  Returns
    (elements, chis): elements [(perm, flip)] with the identity first, perm
    a tuple mapping site s to perm[s]; chis the characters (products along
    the generating words).  Input preparation only: the group and its
    characters are data for the symmetric amplitude, nothing of the method."""
    N, Lx, Ly = lat.N, lat.Lx, lat.Ly

    def site(x, y):
        return (x % Lx) + Lx * (y % Ly)

    def gen_perm(kind):
        name, step = (kind if isinstance(kind, tuple) else (kind, 1))
        out = []
        for s in range(N):
            x, y = s % Lx, s // Lx
            if name == "tx":
                out.append(site(x + step, y))
            elif name == "ty":
                out.append(site(x, y + step))
            elif name == "mx":
                out.append(site(Lx - 1 - x, y))
            elif name == "my":
                out.append(site(x, Ly - 1 - y))
            elif name == "flip":
                out.append(s)
            else:
                raise ValueError(kind)
        return tuple(out), name == "flip"

    gl = [(gen_perm(k), float(c)) for k, c in gens]
    ident = (tuple(range(N)), False)
    elems = {ident: 1.0}
    order = [ident]
    frontier = [ident]
    while frontier:
        nxt = []
        for (perm, flip) in frontier:
            for (gp, gf), c in gl:
                q = (tuple(gp[perm[s]] for s in range(N)), flip != gf)
                chi = elems[(perm, flip)] * c
                if q in elems:
                    if elems[q] != chi:
                        raise ValueError("characters are not a representation of the group")
                    continue
                elems[q] = chi
                order.append(q)
                nxt.append(q)
        frontier = nxt
    return order, [elems[g] for g in order]


def occupations(wl: Workload, lat_index: int = 0, n_walkers: int | None = None,
                seed: int | None = None) -> np.ndarray:
    lat = wl.lattices[lat_index]
    nw = wl.walkers[lat_index] if n_walkers is None else n_walkers
    sd = (wl.seed_occ + 1000 * lat_index) if seed is None else seed
    if wl.stripe:
        return stripe_occupations(lat, nw, sd)
    return random_occupations(lat, nw, sd)
