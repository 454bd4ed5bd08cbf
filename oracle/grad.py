"""d log|psi(n)| / d theta by central finite differences of the full FP64
amplitude (the quantity the optimiser of Sec. II.F consumes).

Flat parameter order (theta):
  embed [4, C] | conv_w [L, 3, 3, C, C] | conv_b [L, C] |
  for each lattice: proj_w up [C, N_up] | proj_w down [C, N_dn] |
                    proj_b up [N_up] | proj_b down [N_dn]
Each block is row-major.  Base orbitals are inputs, not parameters.
"""
from __future__ import annotations

import numpy as np

from .ansatz import log_psi


def pack(params) -> np.ndarray:
    parts = [params.embed.ravel(), params.conv_w.ravel(), params.conv_b.ravel()]
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

    p.embed = take(like.embed.shape)
    p.conv_w = take(like.conv_w.shape)
    p.conv_b = take(like.conv_b.shape)
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
