"""The SCALE amplitude psi(n) = det Phi(n), evaluated from scratch in FP64
(Sec. II.B).

  embedding   H0[s]   = E[n_s]                 (Sec. II.B, embedding layer;
                                                one table shared by all sites,
              or      = E_s[n_s]                one table per site, as the
                                                embedding layer is written there)
  conv layer  H_l[s]  = H_{l-1}[s] + act(b_l + sum_{taps} K_l[tap] H_{l-1}[s+tap])
                                               (Sec. II.B, residual conv
                                                equation; stacked n_conv times,
                                                padding follows the lattice
                                                boundary: wrap on periodic axes,
                                                zeros on open axes)
  site-wise   H_{L+m+1}[s] = act(H_{L+m}[s] W_m + b_m),  m = 0 .. M-1
  MLP                                          (Sec. II.B, site-wise MLP
                                                equation, no residual, weights
                                                C x C as that equation writes
                                                them; absent when M = 0)
  projection  row_s(s) = base_s[s] + H_F[s] W_s + b_s   (H_F the last of these)
                                               (Sec. II.B, orbital projection,
                                                one block per spin)
  amplitude   psi(n) = det Phi_up * det Phi_dn, Phi_s = rows of the sites
              occupied by spin s, in ascending site order.

Kernel layout K_l[ky, kx, c_in, c_out]: tap (ky, kx) reads the neighbour at
offset (kx - 1, ky - 1), i.e. a cross-correlation as in common conv layers.
"""
from __future__ import annotations

import numpy as np

from .lattice import neighbour


def activation(name: str, x: np.ndarray) -> np.ndarray:
    if name == "tanh":
        return np.tanh(x)
    if name == "silu":
        return x / (1.0 + np.exp(-x))
    raise ValueError(name)


def tap_tables(lat) -> list:
    """For each of the 9 taps (ky, kx) in row-major order, an int array
    nb[s] of the neighbour site at offset (kx-1, ky-1), -1 off an open edge."""
    tabs = []
    for ky in range(3):
        for kx in range(3):
            tabs.append(np.array([neighbour(lat, s, kx - 1, ky - 1)
                                  for s in range(lat.N)], dtype=np.int64))
    return tabs


def embedding(params, occ, lat_index: int = 0) -> np.ndarray:
    """H_0 [N, C]: the row of each site's occupation in the shared table, or
    in that site's own table when params.embed_site is set."""
    o = np.asarray(occ, dtype=np.int64)
    site = getattr(params, "embed_site", None)
    if site is None:
        return params.embed[o].astype(np.float64)
    E = site[lat_index]                                   # [N, 4, C]
    return np.stack([E[s, o[s]] for s in range(len(o))]).astype(np.float64)


def features(lat, params, occ, act: str = "tanh", conv_input_round=None, lat_index: int = 0) -> list:
    """[H_0, H_1, ..., H_L, H_{L+1}, ..., H_{L+M}], each [N, C] FP64: the
    conv layers, then the site-wise MLP layers (params.mlp_w, when present).

    conv_input_round: optional function applied to the layer input before it
    enters the convolution (not to the residual branch); used to model a conv
    whose multiplier inputs are rounded to a narrower format."""
    H = embedding(params, occ, lat_index)
    out = [H]
    tabs = tap_tables(lat)
    L = params.conv_w.shape[0]
    for l in range(L):
        acc = np.tile(params.conv_b[l], (lat.N, 1))
        Hin = H if conv_input_round is None else conv_input_round(H)
        for t, nb in enumerate(tabs):
            ky, kx = divmod(t, 3)
            valid = nb >= 0
            x = np.zeros_like(H)
            x[valid] = Hin[nb[valid]]
            acc = acc + x @ params.conv_w[l, ky, kx]
        H = H + activation(act, acc)
        out.append(H)
    for W, b in zip(getattr(params, "mlp_w", None) or [], getattr(params, "mlp_b", None) or []):
        H = activation(act, H @ W + b[None, :])
        out.append(H)
    return out


def orbital_rows(params, lat_index: int, HL: np.ndarray, spin: int) -> np.ndarray:
    """All N backflow orbital rows of one spin: [N, N_spin]."""
    return (params.base[lat_index][spin] + HL @ params.proj_w[lat_index][spin]
            + params.proj_b[lat_index][spin][None, :])


def occupied_sites(occ, spin: int) -> np.ndarray:
    bit = 1 << spin
    return np.nonzero(np.asarray(occ) & bit)[0]


def slater_matrices(lat, params, occ, lat_index: int = 0, act: str = "tanh", conv_input_round=None):
    HL = features(lat, params, occ, act, conv_input_round, lat_index)[-1]
    return [orbital_rows(params, lat_index, HL, s)[occupied_sites(occ, s)]
            for s in (0, 1)]


def log_psi(lat, params, occ, lat_index: int = 0, act: str = "tanh", conv_input_round=None):
    """(sign, log|psi|) with canonical (site-ascending) row order."""
    sign, logabs = 1.0, 0.0
    for Phi in slater_matrices(lat, params, occ, lat_index, act, conv_input_round):
        if Phi.shape[0] == 0:
            continue
        s, la = np.linalg.slogdet(Phi)
        sign *= s
        logabs += la
    return sign, logabs


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest BF16 (ties to even), via FP32."""
    import torch
    return torch.from_numpy(np.asarray(x, np.float64)).to(torch.float32).to(torch.bfloat16) \
        .to(torch.float64).numpy()
