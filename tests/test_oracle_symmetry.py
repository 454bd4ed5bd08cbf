"""Pins of the oracle's symmetry-projected amplitude (App. B):
psi_sym(n) = sum_g Pi(n, g) chi_g psi(g n).

* Pi(n, g) against the operator definition: the canonical creation
  operators of n, mapped by g, applied one by one to the vacuum with
  Jordan-Wigner signs from bit counting (an independent route to the sign).
* Projection: with a one-dimensional representation chi, the vector psi_sym
  is an eigenvector of every U_g (built from the same operator application)
  with eigenvalue chi_g; a wrong fermion sign, a composition error in the
  group or a wrong character fails it.
* E_loc_sym(n) psi_sym(n) = (H psi_sym)(n) with H built by brute force
  (Hubbard and t-J).
* When G commutes with H: E_loc_sym(n) = sum_g w_g E_loc(g n) with
  w_g = Pi(n, g) chi_g psi(g n) / psi_sym(n), the identity the library uses.
"""
import numpy as np
import pytest

import workloads as wl
from oracle.ansatz import log_psi
from oracle.energy import local_energy
from oracle.symmetry import apply_symmetry, fermion_sign, log_psi_sym, local_energy_sym

from test_oracle_bruteforce import hamiltonian, sector, to_occ
from test_oracle_tj import apply_string, projected_sector, tj_hamiltonian


def bits(lat, occ):
    N = lat.N
    return sum(1 << s for s in range(N) if occ[s] & 1) | (sum(1 << s for s in range(N) if occ[s] & 2) << N)


def op_sign(lat, occ, perm, flip):
    """(sign, bitstring) of U_g |n> by operator application."""
    N = lat.N
    modes = [s for s in range(N) if occ[s] & 1] + [N + s for s in range(N) if occ[s] & 2]
    mapped = []
    for m in modes:
        s, sp = m % N, m // N
        mapped.append((perm[s] + N * (sp ^ int(flip)), 1))
    return apply_string(0, mapped)


def sym_vector(lat, p, states, G, chi, act="tanh"):
    v = np.empty(len(states))
    for k, b in enumerate(states):
        s, la = log_psi_sym(lat, p, to_occ(lat, b), G, chi, 0, act)
        v[k] = s * np.exp(la)
    return v


def u_matrix(lat, states, perm, flip):
    index = {b: k for k, b in enumerate(states)}
    U = np.zeros((len(states), len(states)))
    for k, b in enumerate(states):
        sg, nb = op_sign(lat, to_occ(lat, b), perm, flip)
        U[index[nb], k] = sg
    return U


HUB = wl.Lattice(2, 4, 0, 1, 1.0, 0.3, 4.0, 2, 2)            # open x, periodic y
HUB3 = wl.Lattice(2, 4, 0, 1, 1.0, 0.3, 4.0, 3, 3)           # n_up n_dn odd: the spin flip's block sign shows
TJ = wl.Lattice(3, 3, 1, 1, 1.0, -0.2, 0.0, 3, 3, tj=1, J=0.5)
GENS = {
    "ty_mx_my": [("ty", 1.0), ("mx", 1.0), ("my", 1.0)],
    "ty_flip_odd": [("ty", 1.0), ("flip", -1.0)],
    "mx_odd_my": [("mx", -1.0), ("my", 1.0), ("flip", 1.0)],
}


@pytest.mark.parametrize("lat", [HUB, HUB3])
@pytest.mark.parametrize("gname", list(GENS))
def test_fermion_sign_is_the_operator_sign(gname, lat):
    G, _ = wl.symmetry_group(lat, GENS[gname])
    for occ in wl.random_occupations(lat, 6, seed=3):
        for perm, flip in G:
            sg, nb = op_sign(lat, occ, perm, flip)
            assert nb == bits(lat, apply_symmetry(occ, perm, flip))
            assert sg == fermion_sign(occ, perm, flip)


@pytest.mark.parametrize("lat,gname", [(HUB, g) for g in GENS] + [(HUB3, "ty_flip_odd")])
def test_projected_vector_transforms_by_the_character(lat, gname):
    G, chi = wl.symmetry_group(lat, GENS[gname])
    p = wl.random_params([lat], wl.Model(1, 4), seed=8, backflow=0.6)
    states = sector(lat)
    v = sym_vector(lat, p, states, G, chi)
    assert np.max(np.abs(v)) > 1e-6
    for (perm, flip), c in zip(G, chi):
        U = u_matrix(lat, states, perm, flip)
        assert np.allclose(U @ v, c * v, atol=1e-12 * np.max(np.abs(v)))


@pytest.mark.parametrize("lat,gens", [
    (HUB, GENS["ty_mx_my"]),
    (HUB, GENS["ty_flip_odd"]),
    (TJ, [("tx", 1.0), ("ty", 1.0), ("mx", 1.0), ("flip", 1.0)]),
])
def test_symmetric_local_energy_equals_h_psi_and_weighted_copies(lat, gens):
    G, chi = wl.symmetry_group(lat, gens)
    p = wl.random_params([lat], wl.Model(1, 4, "silu"), seed=4, backflow=0.5)
    states = projected_sector(lat) if lat.tj else sector(lat)
    H = tj_hamiltonian(lat, states) if lat.tj else hamiltonian(lat, states)
    v = sym_vector(lat, p, states, G, chi, "silu")
    Hv = H @ v
    scale = np.max(np.abs(v))
    rng = np.random.default_rng(1)
    nz = [k for k in range(len(states)) if abs(v[k]) > 1e-8 * scale]
    for k in rng.choice(nz, 12, replace=False):
        occ = to_occ(lat, states[k])
        e = local_energy_sym(lat, p, occ, G, chi, 0, "silu")
        assert e * v[k] == pytest.approx(Hv[k], abs=1e-11 * scale * (1 + abs(e)))
        # the weighted copies: G commutes with H on these lattices
        num = den = 0.0
        for (perm, flip), c in zip(G, chi):
            gn = apply_symmetry(occ, perm, flip)
            s, la = log_psi(lat, p, gn, 0, "silu")
            a = fermion_sign(occ, perm, flip) * c * s * np.exp(la)
            num += a * local_energy(lat, p, gn, 0, "silu")
            den += a
        assert num / den == pytest.approx(e, abs=1e-10 * (1 + abs(e)))


@pytest.mark.parametrize("lat,gname", [(HUB, "ty_flip_odd"), (HUB3, "mx_odd_my")])
def test_fermion_sign_update_along_a_hop(lat, gname):
    """Pi(n', g) = Pi(n, g) jw_n(h) jw_gn(g h) for a hop h: the relation the
    symmetric sampler keeps Pi up to date with."""
    from oracle.energy import jw_sign
    from oracle.lattice import apply_hop, hops
    G, _ = wl.symmetry_group(lat, GENS[gname])
    for occ in wl.random_occupations(lat, 4, seed=9):
        for h in hops(lat, occ):
            for perm, flip in G:
                gocc = apply_symmetry(occ, perm, flip)
                sp2 = h.spin ^ int(flip)
                lhs = fermion_sign(apply_hop(occ, h), perm, flip)
                rhs = (fermion_sign(occ, perm, flip) * jw_sign(occ, h.spin, h.i, h.j)
                       * jw_sign(gocc, sp2, perm[h.i], perm[h.j]))
                assert lhs == rhs


def test_symmetric_sampler_histogram_chi2():
    """metropolis_sym samples |psi_sym|^2 (chi^2 against the exact
    distribution on a 36-state lattice)."""
    from oracle.sampler import initial_labels
    from oracle.symmetry import metropolis_sym
    lat = wl.Lattice(2, 3, 0, 1, 1.0, 0.0, 4.0, 1, 1)
    G, chi = wl.symmetry_group(lat, [("mx", -1.0), ("my", 1.0)])      # total variation 0.3 from |psi|^2
    p = wl.random_params([lat], wl.Model(1, 4), seed=8, backflow=1.0)
    states = []
    for a in range(lat.N):
        for b in range(lat.N):
            o = np.zeros(lat.N, dtype=np.int8)
            o[a] += 1
            o[b] += 2
            states.append(o)
    v = np.array([log_psi_sym(lat, p, o, G, chi) for o in states])
    w = np.where(v[:, 0] != 0.0, np.exp(2 * v[:, 1]), 0.0)
    prob = w / w.sum()
    key = {o.tobytes(): k for k, o in enumerate(states)}
    counts = np.zeros(len(states))
    init = wl.random_occupations(lat, 8, seed=3)
    for wk in range(8):
        o, pos = init[wk], initial_labels(lat, init[wk])
        o, pos, _ = metropolis_sym(lat, p, o, pos, wk, 99, 0, 10, G, chi)
        for blk in range(100):
            o, pos, _ = metropolis_sym(lat, p, o, pos, wk, 99, (blk + 1) * 4 * lat.N, 4, G, chi)
            counts[key[o.tobytes()]] += 1
    n = counts.sum()
    exp = n * prob
    mask = exp > 5
    chi2 = np.sum((counts[mask] - exp[mask]) ** 2 / exp[mask])
    dof = mask.sum() - 1
    assert chi2 < dof + 8 * np.sqrt(2 * dof) + 20
    # |psi_sym|^2 differs from |psi|^2 here, so the test tells them apart
    w0 = np.array([np.exp(2 * log_psi(lat, p, o)[1]) for o in states])
    exp0 = n * w0 / w0.sum()
    m0 = exp0 > 5
    assert np.sum((counts[m0] - exp0[m0]) ** 2 / exp0[m0]) > 4 * (m0.sum() + 8 * np.sqrt(2 * m0.sum()) + 20)
