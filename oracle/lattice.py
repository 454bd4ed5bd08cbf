"""Lattice geometry and the connected configurations of the Hubbard and t-J
Hamiltonians (Sec. III: nearest-neighbour hopping t, next-nearest-neighbour
hopping t', on-site U; in the t-J model the hops are Gutzwiller-projected,
so none may create a doubly occupied site, and J S_i.S_j on nearest-neighbour
bonds adds the spin exchanges).

Site index s = x + Lx*y.  Periodic axes wrap; open axes drop neighbours that
fall off the lattice.  A periodic axis must have length >= 3 so that its +
and - neighbours are distinct sites (otherwise a bond would be counted twice).
"""
from __future__ import annotations

from dataclasses import dataclass

# hop directions: nearest neighbours first, then next-nearest neighbours
DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]


def check_lattice(lat) -> None:
    if lat.Lx < 1 or lat.Ly < 1:
        raise ValueError("empty lattice")
    if lat.pbc_x and lat.Lx < 3:
        raise ValueError("periodic x axis needs Lx >= 3")
    if lat.pbc_y and lat.Ly < 3:
        raise ValueError("periodic y axis needs Ly >= 3")
    if lat.n_up > lat.N or lat.n_dn > lat.N or lat.n_up < 0 or lat.n_dn < 0:
        raise ValueError("bad electron count")


def neighbour(lat, s: int, dx: int, dy: int) -> int:
    """Site at offset (dx, dy) from s, or -1 if it falls off an open edge."""
    x, y = s % lat.Lx + dx, s // lat.Lx + dy
    if lat.pbc_x:
        x %= lat.Lx
    elif not 0 <= x < lat.Lx:
        return -1
    if lat.pbc_y:
        y %= lat.Ly
    elif not 0 <= y < lat.Ly:
        return -1
    return x + lat.Lx * y


@dataclass(frozen=True)
class Hop:
    spin: int      # 0 = up, 1 = down
    i: int         # site the electron leaves
    j: int         # site it moves to
    d: int         # direction index into DIRS
    t: float       # hopping amplitude of the bond (t or t')


@dataclass(frozen=True)
class Exchange:
    """Spin exchange across a nearest-neighbour bond (t-J model, the
    transverse part of J S_i.S_j): the up electron at i and the down electron
    at j trade sites."""
    i: int         # site of the up electron (it moves to j)
    j: int         # site of the down electron (it moves to i)
    d: int         # direction of j from i, 0..3
    t: float       # J / 2: the local-energy term is -t * R, as for a hop


def hops(lat, occ) -> list:
    """All configurations connected to ``occ`` by one hopping term, in the
    canonical order: spin up before down, source site ascending, direction
    in DIRS order (the four next-nearest directions only when t' != 0).  In
    the t-J model a hop onto a site that holds the other spin is left out
    (the Gutzwiller projector gives it amplitude zero)."""
    nd = 8 if lat.tp != 0.0 else 4
    out = []
    for spin in (0, 1):
        bit = 1 << spin
        for i in range(lat.N):
            if not occ[i] & bit:
                continue
            for d in range(nd):
                j = neighbour(lat, i, *DIRS[d])
                if j < 0 or (occ[j] != 0 if lat.tj else occ[j] & bit):
                    continue
                out.append(Hop(spin, i, j, d, lat.t if d < 4 else lat.tp))
    return out


def exchanges(lat, occ) -> list:
    """The spin exchanges of the t-J model (none otherwise): every
    nearest-neighbour bond with an up electron alone on one end and a down
    electron alone on the other, listed once from its up end, up site
    ascending, direction in DIRS order."""
    if not lat.tj:
        return []
    out = []
    for i in range(lat.N):
        if occ[i] != 1:
            continue
        for d in range(4):
            j = neighbour(lat, i, *DIRS[d])
            if j >= 0 and occ[j] == 2:
                out.append(Exchange(i, j, d, 0.5 * lat.J))
    return out


def connections(lat, occ) -> list:
    """The canonical order of the connected configurations: the hops, then
    the spin exchanges."""
    return hops(lat, occ) + exchanges(lat, occ)


def apply_hop(occ, h):
    """The configuration reached by a Hop or an Exchange."""
    o = occ.copy()
    if isinstance(h, Exchange):
        o[h.i], o[h.j] = occ[h.j], occ[h.i]
        return o
    bit = 1 << h.spin
    o[h.i] -= bit
    o[h.j] += bit
    return o
