"""Pins of the oracle's t-J local energy (Sec. III, t-J Hamiltonian:
Gutzwiller-projected hopping t, t', exchange J S_i.S_j on nearest-neighbour
bonds, and the staggered pinning field on the first column of the
cylinders' open edge).

The Hamiltonian is built here a second, independent way: every term is a
product of single fermion operators applied one by one to occupation
bitstrings (modes ordered spin-up block first, ascending site; the sign of
c_m or c^+_m is the parity of the occupied modes before m).  S^+_i = c^+_{i up}
c_{i dn}, S^-_i = c^+_{i dn} c_{i up}, S^z_i = (n_{i up} - n_{i dn}) / 2.  The
projected space holds the configurations without a doubly occupied site.

* Closed forms: two sites with one up and one down electron have the
  Heisenberg spectrum {-3J/4, J/4}; the half-filled 2x2 open plaquette (a
  four-site ring) has ground energy -2J.
* E_loc(n) psi(n) = (H psi)(n) for every projected configuration of small
  cylinders, with t', J and the pinning field; a sign error in the exchange
  term, a dropped bond or a hop into a doubly occupied site fails it.
* The sampler never leaves the projected space.
"""
import itertools

import numpy as np
import pytest

import workloads as wl
from oracle.ansatz import log_psi
from oracle.energy import local_energy
from oracle.lattice import Exchange, connections, exchanges, hops
from oracle.sampler import initial_labels, metropolis

from test_oracle_bruteforce import to_occ


def apply_op(b, mode, create):
    """(sign, new bitstring) of c^+_mode (create) or c_mode on b, or (0, None)."""
    occupied = (b >> mode) & 1
    if occupied == create:
        return 0, None
    sign = -1 if bin(b & ((1 << mode) - 1)).count("1") % 2 else 1
    return sign, b ^ (1 << mode)


def apply_string(b, ops):
    """ops = [(mode, create), ...] applied right to left."""
    sign = 1
    for mode, create in reversed(ops):
        s, b = apply_op(b, mode, create)
        if s == 0:
            return 0, None
        sign *= s
    return sign, b


def nn_bonds(lat, diagonal=False):
    offs = [(1, 1), (1, -1)] if diagonal else [(1, 0), (0, 1)]
    out = []
    for s in range(lat.N):
        x, y = s % lat.Lx, s // lat.Lx
        for dx, dy in offs:
            X, Y = x + dx, y + dy
            if lat.pbc_x:
                X %= lat.Lx
            if lat.pbc_y:
                Y %= lat.Ly
            if 0 <= X < lat.Lx and 0 <= Y < lat.Ly:
                out.append((s, X + lat.Lx * Y))
    return out


def projected_sector(lat):
    N = lat.N
    st = []
    for ups in itertools.combinations(range(N), lat.n_up):
        rest = [s for s in range(N) if s not in ups]
        for dns in itertools.combinations(rest, lat.n_dn):
            st.append(sum(1 << s for s in ups) | (sum(1 << s for s in dns) << N))
    return st


def tj_hamiltonian(lat, states):
    N = lat.N
    index = {b: k for k, b in enumerate(states)}
    H = np.zeros((len(states), len(states)))

    def add(col, b, amp, ops):
        sign, nb = apply_string(b, ops)
        if sign and nb in index:             # the projector on the left
            H[index[nb], col] += amp * sign

    def sz(b, s):
        return 0.5 * (((b >> s) & 1) - ((b >> (s + N)) & 1))

    hop_bonds = [(i, j, lat.t) for i, j in nn_bonds(lat)]
    if lat.tp != 0.0:
        hop_bonds += [(i, j, lat.tp) for i, j in nn_bonds(lat, diagonal=True)]
    for col, b in enumerate(states):
        for (i, j, t) in hop_bonds:
            for spin in (0, 1):
                for src, dst in ((j, i), (i, j)):
                    add(col, b, -t, [(dst + N * spin, 1), (src + N * spin, 0)])
        for (i, j) in nn_bonds(lat):
            H[col, col] += lat.J * sz(b, i) * sz(b, j)
            up_i, dn_i, up_j, dn_j = i, i + N, j, j + N
            # S^+_i S^-_j and S^-_i S^+_j
            add(col, b, 0.5 * lat.J, [(up_i, 1), (dn_i, 0), (dn_j, 1), (up_j, 0)])
            add(col, b, 0.5 * lat.J, [(dn_i, 1), (up_i, 0), (up_j, 1), (dn_j, 0)])
        for y in range(lat.Ly):
            H[col, col] += lat.h_pin * (-1.0) ** y * sz(b, lat.Lx * y)
    return H


def tj(Lx, Ly, px, py, tp, J, h, nu, nd):
    return wl.Lattice(Lx, Ly, px, py, 1.0, tp, 0.0, nu, nd, tj=1, J=J, h_pin=h)


def test_two_site_heisenberg_spectrum():
    lat = tj(2, 1, 0, 0, 0.0, 0.7, 0.0, 1, 1)
    H = tj_hamiltonian(lat, projected_sector(lat))
    assert np.allclose(np.linalg.eigvalsh(H), [-0.75 * 0.7, 0.25 * 0.7])


def test_four_site_ring_ground_energy():
    lat = tj(2, 2, 0, 0, 0.0, 1.3, 0.0, 2, 2)
    H = tj_hamiltonian(lat, projected_sector(lat))
    assert len(nn_bonds(lat)) == 4
    assert np.linalg.eigvalsh(H)[0] == pytest.approx(-2.0 * 1.3, abs=1e-12)


@pytest.mark.parametrize("lat", [
    tj(2, 4, 0, 1, 0.3, 0.4, 0.5, 3, 2),        # cylinder: open x, periodic y
    tj(3, 3, 1, 1, -0.2, 1.0 / 3.0, 0.5, 4, 4),  # one hole
    tj(2, 3, 0, 0, 0.0, 0.8, 0.3, 3, 3),         # half filled: exchanges only
])
def test_tj_local_energy_equals_h_psi(lat):
    p = wl.random_params([lat], wl.Model(1, 4, "silu", n_mlp=1), seed=7, backflow=0.5)
    states = projected_sector(lat)
    H = tj_hamiltonian(lat, states)
    assert np.allclose(H, H.T)
    psi = np.empty(len(states))
    for k, b in enumerate(states):
        s, la = log_psi(lat, p, to_occ(lat, b), 0, "silu")
        psi[k] = s * np.exp(la)
    Hpsi = H @ psi
    scale = np.max(np.abs(psi))
    n_ex = 0
    for k, b in enumerate(states):
        occ = to_occ(lat, b)
        e, hs, _ = local_energy(lat, p, occ, 0, "silu", return_ratios=True)
        n_ex += sum(isinstance(h, Exchange) for h in hs)
        assert e * psi[k] == pytest.approx(Hpsi[k], abs=1e-11 * scale * (1 + abs(e)))
    assert n_ex > 0


def test_hops_and_exchanges_stay_projected():
    lat = tj(6, 4, 0, 1, 0.2, 1.0 / 3.0, 0.5, 10, 10)
    for occ in wl.random_occupations(lat, 20, seed=3):
        assert not np.any(occ == 3)
        for h in hops(lat, occ):
            assert occ[h.j] == 0
        for x in exchanges(lat, occ):
            assert occ[x.i] == 1 and occ[x.j] == 2
        # canonical order: hops first, then exchanges by up site
        cs = connections(lat, occ)
        k = next((n for n, c in enumerate(cs) if isinstance(c, Exchange)), len(cs))
        assert all(isinstance(c, Exchange) for c in cs[k:])
        assert [c.i for c in cs[k:]] == sorted(c.i for c in cs[k:])


def test_sampler_stays_projected():
    lat = tj(4, 4, 0, 1, 0.2, 1.0 / 3.0, 0.5, 6, 6)
    p = wl.random_params([lat], wl.Model(1, 4), seed=2)
    acc = 0
    for w, occ in enumerate(wl.random_occupations(lat, 3, seed=4)):
        o, pos, n = metropolis(lat, p, occ, initial_labels(lat, occ), w, 9, 0, 3)
        acc += n
        assert not np.any(o == 3)
        assert np.sum(o & 1) == 6 and np.sum((o >> 1) & 1) == 6
        for sp in (0, 1):
            assert all((o[s] >> sp) & 1 for s in pos[sp])
    assert acc > 0
