"""Brute-force pin of the oracle's local energy on a tiny lattice.

The Hubbard Hamiltonian (Sec. III) is built here independently as a matrix
in the occupation-number basis: modes ordered spin-up block first and by
ascending site, fermion signs from the parity of occupied modes strictly
between the two modes of a hop (bit counting), every bond listed once.  The
amplitude vector psi(n) comes from the oracle.  The local energy definition
(Sec. II.A) then requires, configuration by configuration,
  E_loc(n) psi(n) = (H psi)(n),
and the |psi|^2-weighted mean of E_loc equals psi^T H psi / psi^T psi, which
is bounded below by the exact ground energy (variational principle).
"""
import itertools

import numpy as np
import pytest

import workloads as wl
from oracle.ansatz import log_psi
from oracle.energy import local_energy


def bonds(lat):
    out = []
    offs = [((1, 0), lat.t), ((0, 1), lat.t)]
    if lat.tp != 0.0:
        offs += [((1, 1), lat.tp), ((1, -1), lat.tp)]
    for s in range(lat.N):
        x, y = s % lat.Lx, s // lat.Lx
        for (dx, dy), t in offs:
            X, Y = x + dx, y + dy
            if lat.pbc_x:
                X %= lat.Lx
            if lat.pbc_y:
                Y %= lat.Ly
            if 0 <= X < lat.Lx and 0 <= Y < lat.Ly:
                out.append((s, X + lat.Lx * Y, t))
    return out


def hamiltonian(lat, states):
    N = lat.N
    index = {b: k for k, b in enumerate(states)}
    H = np.zeros((len(states), len(states)))
    bl = bonds(lat)
    for col, b in enumerate(states):
        up, dn = b & ((1 << N) - 1), b >> N
        H[col, col] += lat.U * bin(up & dn).count("1")
        for (i, j, t) in bl:
            for spin in (0, 1):
                for src, dst in ((j, i), (i, j)):     # c^+_dst c_src
                    ms, md = src + N * spin, dst + N * spin
                    if not (b >> ms) & 1 or (b >> md) & 1:
                        continue
                    lo, hi = min(ms, md), max(ms, md)
                    between = bin(b & (((1 << hi) - 1) ^ ((1 << (lo + 1)) - 1))).count("1")
                    nb = b ^ (1 << ms) ^ (1 << md)
                    H[index[nb], col] += -t * (-1) ** between
    return H


def sector(lat):
    N = lat.N
    st = []
    for ups in itertools.combinations(range(N), lat.n_up):
        for dns in itertools.combinations(range(N), lat.n_dn):
            st.append(sum(1 << s for s in ups) | (sum(1 << s for s in dns) << N))
    return st


def to_occ(lat, b):
    N = lat.N
    return np.array([((b >> s) & 1) + 2 * ((b >> (s + N)) & 1) for s in range(N)], dtype=np.int8)


@pytest.mark.parametrize("lat", [
    wl.Lattice(2, 4, 0, 1, 1.0, 0.0, 4.0, 3, 2),
    wl.Lattice(2, 4, 0, 1, 1.0, 0.3, 6.0, 2, 2),
    wl.Lattice(3, 3, 1, 1, 1.0, -0.25, 4.0, 2, 2),
    # spin-polarised sectors: the empty spin's determinant is 1
    wl.Lattice(2, 4, 0, 1, 1.0, 0.3, 6.0, 3, 0),
    wl.Lattice(3, 3, 1, 1, 1.0, -0.25, 4.0, 0, 3),
])
def test_local_energy_equals_h_psi(lat):
    p = wl.random_params([lat], wl.Model(2, 4), seed=5, backflow=0.5)
    states = sector(lat)
    H = hamiltonian(lat, states)
    assert np.allclose(H, H.T)
    psi = np.empty(len(states))
    for k, b in enumerate(states):
        s, la = log_psi(lat, p, to_occ(lat, b))
        psi[k] = s * np.exp(la)
    Hpsi = H @ psi
    scale = np.max(np.abs(psi))
    # every configuration for the smallest sector, a seeded subset otherwise;
    # E_loc is undefined on exact nodes (psi = 0, which the symmetric
    # polarised sectors have), where they carry no weight either
    rng = np.random.default_rng(0)
    nodes = {k for k in range(len(states)) if psi[k] == 0.0}
    assert len(nodes) < len(states) // 2
    pick = range(len(states)) if len(states) <= 800 else rng.choice(len(states), 400, replace=False)
    pick = [k for k in pick if k not in nodes]
    eloc = {}
    for k in pick:
        e = local_energy(lat, p, to_occ(lat, states[k]))
        eloc[k] = e
        assert e * psi[k] == pytest.approx(Hpsi[k], abs=1e-11 * scale * (1 + abs(e)))
    if len(eloc) + len(nodes) == len(states):
        w = psi ** 2
        e_var = sum(w[k] * eloc[k] for k in eloc) / w.sum()
        assert e_var == pytest.approx(psi @ Hpsi / (psi @ psi), rel=1e-12)
        assert np.linalg.eigvalsh(H)[0] <= e_var + 1e-12
