"""Local energy and amplitude ratios by full recomputation (Sec. II.A
definition of the local energy; Sec. III Hubbard Hamiltonian).

  E_loc(n) = U * #{doubly occupied sites}
           + sum over hops h = (spin, i -> j) of  -t_h * <n|c^+_i c_j|n_h> * psi(n_h) / psi(n)

With fermion operators ordered spin-up block first and by ascending site
within a spin, <n|c^+_i c_j|n_h> = (-1)^(number of same-spin electrons
strictly between sites i and j).  psi(n_h) is recomputed from scratch
(network forward and determinants) for every hop.

The "in-place" ratio R_h = (-1)^(between) psi(n_h)/psi(n) is the ratio of
determinants when the moving electron keeps its row (row i replaced by row
j); it is what a low-rank update computes and the E_loc term is -t_h R_h.
"""
from __future__ import annotations

import numpy as np

from .ansatz import log_psi
from .lattice import apply_hop, hops


def jw_sign(occ, spin: int, i: int, j: int) -> float:
    bit = 1 << spin
    lo, hi = (i, j) if i < j else (j, i)
    between = sum(1 for s in range(lo + 1, hi) if occ[s] & bit)
    return -1.0 if between % 2 else 1.0


def ratios(lat, params, occ, lat_index: int = 0, act: str = "tanh", conv_input_round=None):
    """(list of Hop, array of in-place ratios R_h, (sign, log|psi|) of n)."""
    s0, l0 = log_psi(lat, params, occ, lat_index, act, conv_input_round)
    hs = hops(lat, occ)
    R = np.empty(len(hs))
    for k, h in enumerate(hs):
        s1, l1 = log_psi(lat, params, apply_hop(occ, h), lat_index, act, conv_input_round)
        R[k] = jw_sign(occ, h.spin, h.i, h.j) * s1 * s0 * np.exp(l1 - l0)
    return hs, R, (s0, l0)


def local_energy(lat, params, occ, lat_index: int = 0, act: str = "tanh",
                 return_ratios: bool = False, conv_input_round=None):
    hs, R, _ = ratios(lat, params, occ, lat_index, act, conv_input_round)
    occ = np.asarray(occ)
    e = lat.U * float(np.sum(occ == 3))
    for h, r in zip(hs, R):
        e += -h.t * r
    if return_ratios:
        return e, hs, R
    return e
