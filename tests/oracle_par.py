"""The oracle spread over host processes, for parity checks at full workload
sizes.  Only the oracle's own functions run here (one hop ratio, one
Metropolis chain per task); this module adds the process pool and puts the
pieces back together exactly as oracle.energy.local_energy does."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_P = {}


def _init(lat, params, li, act):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    _P.update(lat=lat, params=params, li=li, act=act)


def _ratio(task):
    from oracle.ansatz import log_psi
    from oracle.energy import connection_sign
    from oracle.lattice import apply_hop
    occ, h, s0, l0 = task
    s1, l1 = log_psi(_P["lat"], _P["params"], apply_hop(occ, h), _P["li"], _P["act"])
    return connection_sign(occ, h) * s1 * s0 * np.exp(l1 - l0)


def _logpsi(occ):
    from oracle.ansatz import log_psi
    return log_psi(_P["lat"], _P["params"], occ, _P["li"], _P["act"])


def _chain(task):
    from oracle.sampler import initial_labels, metropolis
    occ, w, seed, step0, ns = task
    return metropolis(_P["lat"], _P["params"], occ, initial_labels(_P["lat"], occ), w, seed, step0, ns,
                      lat_index=_P["li"], act=_P["act"])


def procs(n_tasks: int) -> int:
    return max(1, min(16, os.cpu_count() or 1, n_tasks))


def _pool(n, lat, params, li, act):
    return mp.get_context("fork").Pool(procs(n), initializer=_init, initargs=(lat, params, li, act))


def local_energies(lat, params, occs, li: int = 0, act: str = "tanh"):
    """[(E_loc, hops, ratios, (sign, log|psi|))] of each occupation, every hop
    ratio recomputed in full by the oracle, the hops of all walkers spread
    over the pool."""
    from oracle.energy import diagonal_energy
    from oracle.lattice import connections
    occs = [np.asarray(o) for o in occs]
    with _pool(len(occs), lat, params, li, act) as pool:
        ref = pool.map(_logpsi, occs)
        hs = [connections(lat, o) for o in occs]
        tasks = [(o, h, s0, l0) for o, hh, (s0, l0) in zip(occs, hs, ref) for h in hh]
        R = pool.map(_ratio, tasks, chunksize=max(1, len(tasks) // (8 * procs(len(tasks)))))
    out, k = [], 0
    for o, hh, r0 in zip(occs, hs, ref):
        r = np.array(R[k:k + len(hh)])
        k += len(hh)
        e = diagonal_energy(lat, o)
        for h, x in zip(hh, r):
            e += -h.t * x
        out.append((e, hh, r, r0))
    return out


def chains(lat, params, occs, w0: int, seed: int, step0: int, n_sweeps: int, li: int = 0, act: str = "tanh"):
    """oracle.sampler.metropolis of walkers w0, w0 + 1, ... in parallel:
    [(occ, pos, n_accept)]."""
    tasks = [(np.asarray(o), w0 + k, seed, step0, n_sweeps) for k, o in enumerate(occs)]
    with _pool(len(tasks), lat, params, li, act) as pool:
        return pool.map(_chain, tasks, chunksize=1)
