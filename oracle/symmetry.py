"""Symmetry-projected amplitudes (App. B, symmetrized wavefunction):

  psi_sym(n) = sum over g in G of Pi(n, g) chi_g psi(g n)

A group element g maps site s to perm[s] and, with flip, exchanges the two
spins.  On Fock states it acts as U_g c^+_{s, sigma} U_g^-1 = c^+_{perm[s],
sigma'} (sigma' = sigma, or the other spin under flip), and U_g |n> =
Pi(n, g) |g n>: Pi is the sign of reordering the mapped creation operators
into the canonical order of g n (spin-up block first, ascending site within
a spin).

The local energy of psi_sym is taken from its plain definition,
  E_loc_sym(n) = E_diag(n) + sum over connected n' of H_{n n'} psi_sym(n') / psi_sym(n),
every psi_sym(n') recomputed in full (|G| network evaluations each).  The
oracle does not assume that G is a symmetry of the Hamiltonian.

Sampling |psi_sym|^2 uses the proposals of oracle.sampler (the same Philox
block, counter (walker, step)); the ratio psi_sym(n') / psi_sym(n) is
recomputed in full.

Test infrastructure: used by the tests, never by the library.
"""
from __future__ import annotations

import numpy as np

from .ansatz import log_psi
from .energy import connection_sign, diagonal_energy
from .lattice import DIRS, apply_hop, connections, neighbour
from .philox import proposal_draw


def apply_symmetry(occ, perm, flip: bool):
    """Occupation g n: site s of n goes to perm[s]; flip swaps the spins."""
    occ = np.asarray(occ)
    out = np.zeros_like(occ)
    for s, o in enumerate(occ):
        if flip:
            o = ((o & 1) << 1) | ((o >> 1) & 1)
        out[perm[s]] = o
    return out


def _perm_sign(seq) -> int:
    """Sign of the permutation that sorts ``seq`` (distinct values), by
    counting inversions."""
    inv = 0
    for a in range(len(seq)):
        for b in range(a + 1, len(seq)):
            inv += seq[a] > seq[b]
    return -1 if inv % 2 else 1


def fermion_sign(occ, perm, flip: bool) -> int:
    """Pi(n, g): U_g |n> = Pi(n, g) |g n>.  The creation operators of n in
    canonical order, mapped by g, are [c^+_{perm[s], up'} for up sites s
    ascending] then [c^+_{perm[s], dn'} for down sites s ascending]; the sign
    is that of sorting this list into g n's canonical order."""
    occ = np.asarray(occ)
    ups = [s for s in range(len(occ)) if occ[s] & 1]
    dns = [s for s in range(len(occ)) if occ[s] & 2]
    # canonical position key of an operator on (site, spin): spin major
    n_sites = len(occ)
    keys = [perm[s] + n_sites * (1 if flip else 0) for s in ups] + \
           [perm[s] + n_sites * (0 if flip else 1) for s in dns]
    return _perm_sign(keys)


def psi_sym(lat, params, occ, group, chi, lat_index: int = 0, act: str = "tanh") -> float:
    """psi_sym(n) as a plain float (small lattices: no overflow handling
    beyond a common scale)."""
    terms = []
    for (perm, flip), c in zip(group, chi):
        gn = apply_symmetry(occ, perm, flip)
        s, la = log_psi(lat, params, gn, lat_index, act)
        terms.append((fermion_sign(occ, perm, flip) * c * s, la))
    top = max(la for _, la in terms)
    if top == -np.inf:
        return 0.0, 0.0
    return sum(a * np.exp(la - top) for a, la in terms), top


def log_psi_sym(lat, params, occ, group, chi, lat_index: int = 0, act: str = "tanh"):
    """(sign, log|psi_sym|) of n."""
    v, top = psi_sym(lat, params, occ, group, chi, lat_index, act)
    if v == 0.0:
        return 0.0, -np.inf
    return float(np.sign(v)), float(np.log(abs(v)) + top)


def local_energy_sym(lat, params, occ, group, chi, lat_index: int = 0, act: str = "tanh") -> float:
    occ = np.asarray(occ)
    s0, l0 = log_psi_sym(lat, params, occ, group, chi, lat_index, act)
    if s0 == 0.0:
        return float("nan")          # psi_sym(n) = 0: no local energy
    e = diagonal_energy(lat, occ)
    for h in connections(lat, occ):
        s1, l1 = log_psi_sym(lat, params, apply_hop(occ, h), group, chi, lat_index, act)
        if s1 == 0.0:
            continue
        e += -h.t * connection_sign(occ, h) * s1 * s0 * np.exp(l1 - l0)
    return e


def metropolis_sym(lat, params, occ, pos, walker: int, seed: int, step0: int, n_sweeps: int,
                   group, chi, lat_index: int = 0, act: str = "tanh"):
    """n_sweeps Metropolis sweeps of |psi_sym|^2 on one walker: proposals as
    in oracle.sampler.metropolis, accepted iff u < (psi_sym(n') / psi_sym(n))^2
    (rejected while psi_sym(n) = 0).  Returns (occ, pos, n_accept)."""
    occ = np.array(occ, dtype=np.int8)
    pos = [p.copy() for p in pos]
    n_up, n_dn = lat.n_up, lat.n_dn
    ne = n_up + n_dn
    if ne == 0:
        return occ, pos, 0
    s0, l0 = log_psi_sym(lat, params, occ, group, chi, lat_index, act)
    n_acc = 0
    for sweep in range(n_sweeps):
        for p in range(lat.N):
            step = step0 + sweep * lat.N + p
            e, d, u = proposal_draw(seed, walker, step, ne)
            spin, k = (0, e) if e < n_up else (1, e - n_up)
            bit = 1 << spin
            i = int(pos[spin][k])
            j = neighbour(lat, i, *DIRS[d])
            if j < 0 or (occ[j] != 0 if lat.tj else occ[j] & bit):
                continue
            new = occ.copy()
            new[i] -= bit
            new[j] += bit
            s1, l1 = log_psi_sym(lat, params, new, group, chi, lat_index, act)
            if s0 == 0.0 or s1 == 0.0:
                continue
            if u < float(np.exp(2.0 * (l1 - l0))):
                occ = new
                pos[spin][k] = j
                s0, l0 = s1, l1
                n_acc += 1
    return occ, pos, n_acc
