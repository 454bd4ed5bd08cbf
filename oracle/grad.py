"""d log|psi(n)| / d theta (the quantity the optimiser of Sec. II.F consumes),
two independent routes:

* fd_grad: central finite differences of the full FP64 amplitude;
* autograd_grad: the amplitude of Sec. II.B written with torch CPU FP64
  primitives (conv2d with boundary-following padding, slogdet), differentiated
  by torch autograd.

Flat parameter order (theta):
  embed [4, C] (or, with per-site tables, [N_l, 4, C] of every lattice l) |
  conv_w [L, 3, 3, C, C] | conv_b [L, C] |
  mlp_w [M, C, C] | mlp_b [M, C]   (site-wise layers; absent when M = 0) |
  for each lattice: proj_w up [C, N_up] | proj_w down [C, N_dn] |
                    proj_b up [N_up] | proj_b down [N_dn]
Each block is row-major.  Base orbitals are inputs, not parameters.
"""
from __future__ import annotations

import numpy as np

from .ansatz import log_psi, occupied_sites


def pack(params) -> np.ndarray:
    emb = [params.embed.ravel()] if params.embed_site is None else [e.ravel() for e in params.embed_site]
    parts = emb + [params.conv_w.ravel(), params.conv_b.ravel()]
    parts += [w.ravel() for w in (params.mlp_w or [])] + [b.ravel() for b in (params.mlp_b or [])]
    for pw, pb in zip(params.proj_w, params.proj_b):
        parts += [pw[0].ravel(), pw[1].ravel(), pb[0].ravel(), pb[1].ravel()]
    return np.concatenate(parts).astype(np.float64)


def unpack(theta: np.ndarray, like):
    p = like.copy()
    off = 0

    def take(shape):
        nonlocal off
        n = int(np.prod(shape))
        a = np.array(theta[off:off + n], dtype=np.float64).reshape(shape)
        off += n
        return a

    if like.embed_site is None:
        p.embed = take(like.embed.shape)
    else:
        p.embed_site = [take(e.shape) for e in like.embed_site]
    p.conv_w = take(like.conv_w.shape)
    p.conv_b = take(like.conv_b.shape)
    if like.mlp_w:
        p.mlp_w = [take(w.shape) for w in like.mlp_w]
        p.mlp_b = [take(b.shape) for b in like.mlp_b]
    for li in range(len(like.proj_w)):
        p.proj_w[li] = [take(like.proj_w[li][0].shape), take(like.proj_w[li][1].shape)]
        p.proj_b[li] = [take(like.proj_b[li][0].shape), take(like.proj_b[li][1].shape)]
    assert off == theta.size
    return p


def fd_grad(lat, params, occ, lat_index: int = 0, act: str = "tanh",
            h: float = 1e-5, indices=None) -> np.ndarray:
    """Central differences (f(x+h) - f(x-h)) / 2h of log|psi| for the
    parameters in ``indices`` (all if None)."""
    theta = pack(params)
    idx = np.arange(theta.size) if indices is None else np.asarray(indices)
    g = np.zeros(len(idx))
    for n, k in enumerate(idx):
        tp = theta.copy()
        tp[k] += h
        tm = theta.copy()
        tm[k] -= h
        lp = log_psi(lat, unpack(tp, params), occ, lat_index, act)[1]
        lm = log_psi(lat, unpack(tm, params), occ, lat_index, act)[1]
        g[n] = (lp - lm) / (2.0 * h)
    return g


def _torch_log_psi(lat, theta, like, occ, lat_index: int, act: str):
    """log|psi| as a torch graph of the flat parameter vector theta."""
    import torch
    import torch.nn.functional as F
    C, L = like.embed.shape[1], like.conv_w.shape[0]
    off = 0

    def take(shape):
        nonlocal off
        n = int(np.prod(shape))
        a = theta[off:off + n].reshape(shape)
        off += n
        return a
    if like.embed_site is None:
        E = take((4, C))
    else:
        Es = [take(e.shape) for e in like.embed_site]
    K = take((L, 3, 3, C, C))
    b = take((L, C))
    M = len(like.mlp_w or [])
    MW = [take((C, C)) for _ in range(M)]
    MB = [take((C,)) for _ in range(M)]
    proj = []
    for li in range(len(like.proj_w)):
        nu, nd = like.proj_w[li][0].shape[1], like.proj_w[li][1].shape[1]
        proj.append((take((C, nu)), take((C, nd)), take((nu,)), take((nd,))))
    assert off == theta.numel()
    o = torch.from_numpy(np.asarray(occ, dtype=np.int64))
    if like.embed_site is None:
        H0 = E[o]
    else:
        H0 = Es[lat_index][torch.arange(lat.N), o]            # [N, C]: site s, its occupation
    x = H0.T.reshape(1, C, lat.Ly, lat.Lx)
    for l in range(L):
        # circular padding on periodic axes, zeros on open ones
        xp = F.pad(x, (1, 1, 0, 0), mode="circular") if lat.pbc_x else F.pad(x, (1, 1, 0, 0))
        xp = F.pad(xp, (0, 0, 1, 1), mode="circular") if lat.pbc_y else F.pad(xp, (0, 0, 1, 1))
        y = F.conv2d(xp, K[l].permute(3, 2, 0, 1), b[l])       # weights [cout, cin, ky, kx]
        x = x + (torch.tanh(y) if act == "tanh" else F.silu(y))
    HL = x.reshape(C, lat.N).T
    for W, bb in zip(MW, MB):
        y = F.linear(HL, W.T, bb)                            # H W + b, site by site
        HL = torch.tanh(y) if act == "tanh" else F.silu(y)
    Wu, Wd, bu, bd = proj[lat_index]
    tot = theta.new_zeros(())
    for s, (W, bb) in enumerate(((Wu, bu), (Wd, bd))):
        idx = occupied_sites(occ, s)
        if len(idx) == 0:
            continue
        rows = torch.from_numpy(like.base[lat_index][s]) + HL @ W + bb[None, :]
        tot = tot + torch.linalg.slogdet(rows[torch.from_numpy(idx)])[1]
    return tot


def autograd_grad(lat, params, occ, lat_index: int = 0, act: str = "tanh"):
    """(log|psi|, d log|psi| / d theta) in the flat layout of pack(), by torch
    autograd in FP64 on the CPU; other lattices' projection entries are 0."""
    import torch
    theta = torch.from_numpy(pack(params)).requires_grad_(True)
    lp = _torch_log_psi(lat, theta, params, occ, lat_index, act)
    lp.backward()
    return float(lp.item()), theta.grad.numpy().copy()
