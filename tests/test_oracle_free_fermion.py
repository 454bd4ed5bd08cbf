"""Closed-form pin of the oracle's local energy, sign convention and hop
enumeration.

With U = 0 and no backflow (projection weights and bias zero), the amplitude
is a Slater determinant of the lowest one-body orbitals.  For a closed shell
that determinant is an exact eigenstate of the hopping Hamiltonian, so the
local energy (Sec. II.A definition) is the same number on every configuration:
twice the sum of the N_sigma lowest single-particle energies
  e(k) = -2 t (cos kx + cos ky) - 4 t' cos kx cos ky,
with k = 2 pi m / L on periodic axes and k = pi n / (L + 1) on open axes.
A wrong fermion sign, a missing or doubled bond, or a wrong ratio breaks the
zero variance.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.ansatz import log_psi
from oracle.energy import local_energy


def nonzero_configs(lat, p, occ):
    """Configurations on which psi does not vanish (a plane-wave Slater
    determinant has exact nodes on symmetric configurations)."""
    vals = [log_psi(lat, p, o) for o in occ]
    top = max(la for s, la in vals if s != 0.0)
    return [o for o, (s, la) in zip(occ, vals) if s != 0.0 and la > top - 12.0]


def closed_form_e0(lat):
    def ks(L, periodic):
        if periodic:
            return [math.cos(2 * math.pi * m / L) for m in range(L)]
        return [math.cos(math.pi * n / (L + 1)) for n in range(1, L + 1)]
    es = sorted(-2 * lat.t * (cx + cy) - 4 * lat.tp * cx * cy
                for cx in ks(lat.Lx, lat.pbc_x) for cy in ks(lat.Ly, lat.pbc_y))
    return sum(es[:lat.n_up]) + sum(es[:lat.n_dn])


def no_backflow(lat, C=4, L=2, seed=3):
    p = wl.random_params([lat], wl.Model(L, C), seed=seed)
    for s in (0, 1):
        p.proj_w[0][s][:] = 0.0
        p.proj_b[0][s][:] = 0.0
    return p


def golden_cases():
    """Closed-form values of tests/golden/free_fermion_e0.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "free_fermion_e0.txt")
    out = []
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        Lx, Ly, px, py = (int(v) for v in line[:4])
        t, tp = float(line[4]), float(line[5])
        nu, nd = int(line[6]), int(line[7])
        out.append((wl.Lattice(Lx, Ly, px, py, t, tp, 0.0, nu, nd), float(line[8])))
    return out


GOLDEN = golden_cases()
CASES = [c for c in GOLDEN if c[0].N <= 64]


@pytest.mark.parametrize("lat,e0", CASES)
def test_zero_variance_small(lat, e0):
    assert closed_form_e0(lat) == pytest.approx(e0, abs=1e-12)
    p = no_backflow(lat)
    occ = nonzero_configs(lat, p, wl.random_occupations(lat, 64, seed=7))
    assert len(occ) >= 4
    for o in occ:
        assert local_energy(lat, p, o) == pytest.approx(e0, abs=1e-9)


@pytest.mark.slow
def test_zero_variance_16x16_open_y():
    """The headline lattice: 16x16 periodic-x / open-y, 112 per spin; the
    shell is closed (gap 9.1e-3), E0 = -405.312933627526."""
    lat, e_gold = [c for c in GOLDEN if c[0].N == 256][0]
    e0 = closed_form_e0(lat)
    assert e0 == pytest.approx(e_gold, abs=1e-9)
    p = no_backflow(lat, C=4, L=1)
    occ = nonzero_configs(lat, p, wl.random_occupations(lat, 2, seed=11))
    assert len(occ) == 2
    for o in occ:
        assert local_energy(lat, p, o) == pytest.approx(e0, abs=1e-8)


def test_u_term_counts_double_occupancy():
    """With the hopping switched off, E_loc is U times the number of doubly
    occupied sites."""
    lat = wl.Lattice(4, 4, 1, 1, 0.0, 0.0, 3.5, 5, 5)
    p = wl.random_params([lat], wl.Model(2, 4), seed=1)
    for o in wl.random_occupations(lat, 8, seed=2):
        assert local_energy(lat, p, o) == pytest.approx(3.5 * np.sum(o == 3), abs=1e-12)
