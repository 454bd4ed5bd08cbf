"""The process-parallel oracle helper used by the full-size GPU parity tests
gives exactly what the oracle's sequential functions give."""
import numpy as np

import workloads as wl
from oracle.energy import local_energy
from oracle.sampler import initial_labels, metropolis
from oracle_par import chains, local_energies


def test_parallel_local_energy_equals_oracle():
    lat = wl.Lattice(5, 4, 1, 0, 1.0, -0.3, 6.0, 6, 5)
    p = wl.random_params([lat], wl.Model(2, 4), seed=2, backflow=0.5)
    occs = wl.random_occupations(lat, 3, seed=7)
    par = local_energies(lat, p, occs, 0, "tanh")
    for o, (e, hs, R, _) in zip(occs, par):
        e_ref, hs_ref, R_ref = local_energy(lat, p, o, 0, "tanh", return_ratios=True)
        assert hs == hs_ref
        assert np.array_equal(R, R_ref)
        assert e == e_ref


def test_parallel_chains_equal_oracle():
    lat = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)
    p = wl.random_params([lat], wl.Model(2, 4), seed=1, backflow=0.5)
    occs = wl.random_occupations(lat, 3, seed=5)
    par = chains(lat, p, occs, 10, 99, 3, 2)
    for k, o in enumerate(occs):
        o2, p2, na = metropolis(lat, p, o, initial_labels(lat, o), 10 + k, 99, 3, 2)
        assert np.array_equal(par[k][0], o2) and par[k][2] == na
        assert all(np.array_equal(a, b) for a, b in zip(par[k][1], p2))
