"""bench.lowrank_flops, the algorithmic work behind the roofline figure,
against a brute-force enumeration of every hop: per layer l the union of the
two Chebyshev balls of radius l around the hop's sites (wrapped on periodic
axes, clipped on open ones), and per spin the electrons inside the layer-L
union.  Covers nearest-neighbour and diagonal hops, periodic and open axes,
axes short enough for the balls to wrap onto themselves, and t-J lattices
(the oracle's Gutzwiller-projected hops and spin exchanges).  bench.ctx_hops
counts the oracle's connections."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as wl  # noqa: E402
from oracle.lattice import Exchange, connections  # noqa: E402

DX = [1, -1, 0, 0, 1, 1, -1, -1]
DY = [0, 0, 1, -1, 1, -1, 1, -1]


def brute_flops(lat, occ, L, C, n_mlp=0):
    W, N = occ.shape
    Lx, Ly = lat.Lx, lat.Ly
    nd = 8 if lat.tp != 0.0 else 4

    def wrap(x, y):
        if lat.pbc_x:
            x %= Lx
        elif not 0 <= x < Lx:
            return None
        if lat.pbc_y:
            y %= Ly
        elif not 0 <= y < Ly:
            return None
        return x, y

    def ball(x, y, l):
        out = set()
        for dy in range(-l, l + 1):
            for dx in range(-l, l + 1):
                p = wrap(x + dx, y + dy)
                if p is not None:
                    out.add(p)
        return out

    conv = det = 0.0
    for w in range(W):
        g = occ[w].reshape(Ly, Lx)
        if lat.tj:
            # the oracle's connections: Gutzwiller-projected hops, then the
            # spin exchanges (both spins move)
            moves = [(c.i, c.j, (0, 1) if isinstance(c, Exchange) else (c.spin,))
                     for c in connections(lat, occ[w])]
        else:
            moves = []
            for sp in (0, 1):
                for y in range(Ly):
                    for x in range(Lx):
                        if not (g[y, x] >> sp) & 1:
                            continue
                        for d in range(nd):
                            pj = wrap(x + DX[d], y + DY[d])
                            if pj is None or (g[pj[1], pj[0]] >> sp) & 1:
                                continue
                            moves.append((x + Lx * y, pj[0] + Lx * pj[1], (sp,)))
        for i, j, movers in moves:
            x, y, pj = i % Lx, i // Lx, (j % Lx, j // Lx)
            for l in range(1, L + 1):
                conv += len(ball(x, y, l) | ball(*pj, l)) * 9 * C * C * 2
            box = ball(x, y, L) | ball(*pj, L)
            conv += len(box) * n_mlp * C * C * 2
            for tau in (0, 1):
                k = sum(1 for (bx, by) in box if (g[by, bx] >> tau) & 1)
                r = min(k, C + (1 if tau in movers else 0))
                det += 2.0 * (k * C * r + r ** 3 / 3.0)
    return conv, det


CASES = [
    ("6x5_open_y_nn", wl.Lattice(6, 5, 1, 0, 1.0, 0.0, 4.0, 7, 6), 2, 8),
    ("6x5_open_y_diag", wl.Lattice(6, 5, 1, 0, 1.0, 0.3, 4.0, 7, 6), 2, 8),
    ("9x8_pbc_diag_L3", wl.Lattice(9, 8, 1, 1, 1.0, -0.2, 4.0, 20, 18), 3, 8),
    ("5x7_open_diag_C16", wl.Lattice(5, 7, 0, 0, 1.0, 0.2, 4.0, 8, 9), 2, 16),
    ("4x4_pbc_wrapping_L2", wl.Lattice(4, 4, 1, 1, 1.0, 0.1, 4.0, 5, 5), 2, 8),
    ("8x4_tj_cylinder", wl.Lattice(8, 4, 0, 1, 1.0, 0.2, 0.0, 14, 14, tj=1, J=0.3, h_pin=0.5), 1, 8),
    ("6x6_tj_half_filled_L2", wl.Lattice(6, 6, 1, 1, 1.0, 0.0, 0.0, 18, 18, tj=1, J=1.0), 2, 8),
]


@pytest.mark.parametrize("name,lat,L,C", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("n_mlp", [0, 3])
def test_lowrank_flops_match_brute_force(name, lat, L, C, n_mlp):
    occ = wl.random_occupations(lat, 3, seed=4)
    got = bench.lowrank_flops(lat, occ, L, C, n_mlp)
    ref = brute_flops(lat, occ, L, C, n_mlp)
    assert got[0] == pytest.approx(ref[0], rel=1e-12)
    assert got[1] == pytest.approx(ref[1], rel=1e-12)


@pytest.mark.parametrize("name,lat,L,C", CASES, ids=[c[0] for c in CASES])
def test_ctx_hops_counts_connections(name, lat, L, C):
    occ = wl.random_occupations(lat, 4, seed=6)
    assert list(bench.ctx_hops(lat, occ)) == [len(connections(lat, o)) for o in occ]
