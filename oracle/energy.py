"""Local energy and amplitude ratios by full recomputation (Sec. II.A
definition of the local energy; Sec. III Hubbard and t-J Hamiltonians).

  E_loc(n) = E_diag(n)
           + sum over hops h = (spin, i -> j) of  -t_h * <n|c^+_i c_j|n_h> * psi(n_h) / psi(n)
           + sum over spin exchanges x of  (J/2) * <n|S^+_i S^-_j + S^-_i S^+_j|n_x> * psi(n_x) / psi(n)

With fermion operators ordered spin-up block first and by ascending site
within a spin, <n|c^+_i c_j|n_h> = (-1)^(number of same-spin electrons
strictly between sites i and j).  psi(n_h) is recomputed from scratch
(network forward and determinants) for every hop.

E_diag is U times the doubly occupied sites (Hubbard); in the t-J model it
is J sum over nearest-neighbour bonds of S^z_i S^z_j (S^z = (n_up - n_dn)/2,
each bond once) plus the staggered pinning field h_pin sum_y (-1)^y S^z on
the column x = 0, and there is no U term (no site is doubly occupied).

Spin exchange: S^+_i S^-_j = c^+_{i up} c_{i dn} c^+_{j dn} c_{j up}
= -(c^+_{i up} c_{j up})(c^+_{j dn} c_{i dn}), two hops of opposite spins, so
its matrix element is minus the product of the two hops' signs.

The "in-place" ratio R_h = (-1)^(between) psi(n_h)/psi(n) is the ratio of
determinants when the moving electron keeps its row (row i replaced by row
j); it is what a low-rank update computes and the E_loc term is -t_h R_h.
For a spin exchange both spins move in place, R_x = (product of both spins'
signs) psi(n_x)/psi(n), and the term is -(J/2) R_x.
"""
from __future__ import annotations

import numpy as np

from .ansatz import log_psi
from .lattice import DIRS, Exchange, apply_hop, connections, neighbour


def jw_sign(occ, spin: int, i: int, j: int) -> float:
    bit = 1 << spin
    lo, hi = (i, j) if i < j else (j, i)
    between = sum(1 for s in range(lo + 1, hi) if occ[s] & bit)
    return -1.0 if between % 2 else 1.0


def connection_sign(occ, h) -> float:
    """Sign relating the in-place ratio of a hop or exchange to psi(n')/psi(n)."""
    if isinstance(h, Exchange):
        return jw_sign(occ, 0, h.i, h.j) * jw_sign(occ, 1, h.i, h.j)
    return jw_sign(occ, h.spin, h.i, h.j)


def diagonal_energy(lat, occ) -> float:
    occ = np.asarray(occ)
    if not lat.tj:
        return lat.U * float(np.sum(occ == 3))
    sz = 0.5 * ((occ & 1) != 0) - 0.5 * ((occ & 2) != 0)
    e = 0.0
    for s in range(lat.N):
        for d in (0, 2):                      # +x and +y: every bond once
            j = neighbour(lat, s, *DIRS[d])
            if j >= 0:
                e += lat.J * sz[s] * sz[j]
    for y in range(lat.Ly):
        e += lat.h_pin * (-1.0) ** y * sz[lat.Lx * y]
    return e


def ratios(lat, params, occ, lat_index: int = 0, act: str = "tanh", conv_input_round=None):
    """(list of Hop / Exchange, array of in-place ratios R_h, (sign, log|psi|) of n)."""
    s0, l0 = log_psi(lat, params, occ, lat_index, act, conv_input_round)
    hs = connections(lat, occ)
    R = np.empty(len(hs))
    for k, h in enumerate(hs):
        s1, l1 = log_psi(lat, params, apply_hop(occ, h), lat_index, act, conv_input_round)
        R[k] = connection_sign(occ, h) * s1 * s0 * np.exp(l1 - l0)
    return hs, R, (s0, l0)


def local_energy(lat, params, occ, lat_index: int = 0, act: str = "tanh",
                 return_ratios: bool = False, conv_input_round=None):
    hs, R, _ = ratios(lat, params, occ, lat_index, act, conv_input_round)
    e = diagonal_energy(lat, occ)
    for h, r in zip(hs, R):
        e += -h.t * r
    if return_ratios:
        return e, hs, R
    return e
