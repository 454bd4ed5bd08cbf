"""Metropolis sampling of |psi|^2 with single-electron nearest-neighbour
moves (Sec. II.A: configurations are drawn from P(n) ~ |psi(n)|^2 by Markov
chain Monte Carlo).  The paper does not fix the proposal; this one is
symmetric, so the acceptance probability is min(1, |psi(n')/psi(n)|^2).

Proposal p of walker w draws one Philox block (counter (w, step, 0, 0)):
an electron index e over all N_up + N_dn electrons (labels of spin up first),
a direction d in {+x, -x, +y, -y} and a uniform u.  The move is rejected
without evaluation when the target site is off the lattice or already holds
an electron of the same spin (in the t-J model: any electron, since the
Gutzwiller projector gives a doubly occupied site amplitude zero); otherwise it is accepted iff u < R^2 with R the
amplitude ratio, here recomputed in full.  Electron labels keep their
identity: an accepted move changes the site of label e only.  One sweep is N
proposals.
"""
from __future__ import annotations

import numpy as np

from .ansatz import log_psi
from .lattice import DIRS, neighbour
from .philox import proposal_draw


def initial_labels(lat, occ):
    """pos[spin][k] = site of electron label k, labels in ascending site order."""
    occ = np.asarray(occ)
    return [np.nonzero(occ & 1)[0].astype(np.int64),
            np.nonzero(occ & 2)[0].astype(np.int64)]


def metropolis(lat, params, occ, pos, walker: int, seed: int, step0: int,
               n_sweeps: int, lat_index: int = 0, act: str = "tanh"):
    """Run n_sweeps sweeps on one walker; returns (occ, pos, n_accept)."""
    occ = np.array(occ, dtype=np.int8)
    pos = [p.copy() for p in pos]
    n_up, n_dn = lat.n_up, lat.n_dn
    ne = n_up + n_dn
    if ne == 0:
        return occ, pos, 0
    _, l0 = log_psi(lat, params, occ, lat_index, act)
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
            s1, l1 = log_psi(lat, params, new, lat_index, act)
            if s1 == 0.0:
                continue
            r2 = float(np.exp(2.0 * (l1 - l0)))
            if u < r2:
                occ = new
                pos[spin][k] = j
                l0 = l1
                n_acc += 1
    return occ, pos, n_acc
