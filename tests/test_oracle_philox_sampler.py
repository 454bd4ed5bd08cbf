"""Pins of the oracle's random numbers and Metropolis sampler.

* philox4x64 (written from the SC'11 definition) must produce the same words
  as numpy.random.Philox, an independent implementation of Philox4x64-10
  (numpy increments its counter before generating, so its state c-1 yields
  our block c).
* Ratio invariants (Sec. II.A/II.C): reciprocity R(n->n') R(n'->n) = 1, and
  with no backflow the in-place ratio equals the textbook single-row
  replacement ratio (row_j Phi^-1)[k] (matrix determinant lemma, rank 1).
* The sampler's visit histogram on a tiny lattice agrees with |psi|^2 / Z
  (chi-square), and moves never change the electron counts.
"""
import itertools

import numpy as np
import pytest

import workloads as wl
from oracle.ansatz import log_psi, occupied_sites, orbital_rows, features
from oracle.energy import ratios
from oracle.lattice import apply_hop
from oracle.philox import philox4x64, proposal_draw
from oracle.sampler import initial_labels, metropolis


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (1, 0, 0, 0)),
    ((5, 0), (8, 3, 0, 0)),
    ((2**63 + 12345, 77), (2**40 + 1, 2**33 + 5, 9, 11)),
    ((123456789, 0), (4095, 65535, 0, 0)),
])
def test_philox_matches_numpy(key, ctr):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([ctr[0] - 1, *ctr[1:]], dtype=np.uint64))
    ref = [int(v) for v in bg.random_raw(4)]
    assert list(philox4x64(ctr, key)) == ref


def test_proposal_draw_ranges():
    for step in range(200):
        e, d, u = proposal_draw(42, 3, step, 17)
        assert 0 <= e < 17 and 0 <= d < 4 and 0.0 <= u < 1.0


def test_reciprocity_and_rank_one():
    lat = wl.Lattice(4, 4, 1, 1, 1.0, -0.3, 4.0, 5, 4)
    p = wl.random_params([lat], wl.Model(2, 4), seed=2, backflow=0.5)
    o = wl.random_occupations(lat, 1, seed=5)[0]
    hs, R, _ = ratios(lat, p, o)
    for h, r in list(zip(hs, R))[::3]:
        o2 = apply_hop(o, h)
        hs2, R2, _ = ratios(lat, p, o2)
        back = [k for k, g in enumerate(hs2) if g.spin == h.spin and g.i == h.j and g.j == h.i]
        assert len(back) == 1
        assert r * R2[back[0]] == pytest.approx(1.0, rel=1e-10)
    # zero backflow: textbook single-row replacement
    q = p.copy()
    for s in (0, 1):
        q.proj_w[0][s][:] = 0.0
        q.proj_b[0][s][:] = 0.0
    cands = wl.random_occupations(lat, 16, seed=6)
    o = max(cands, key=lambda c: log_psi(lat, q, c)[1])   # far from a node
    hs, R, _ = ratios(lat, q, o)
    for h, r in zip(hs, R):
        rows = q.base[0][h.spin]
        sites = occupied_sites(o, h.spin)
        k = int(np.nonzero(sites == h.i)[0][0])
        inv = np.linalg.inv(rows[sites])
        assert r == pytest.approx(float(rows[h.j] @ inv[:, k]), rel=1e-9, abs=1e-12)


@pytest.mark.slow
def test_sampler_histogram_chi2():
    lat = wl.Lattice(2, 3, 0, 1, 1.0, 0.0, 4.0, 1, 1)
    p = wl.random_params([lat], wl.Model(1, 4), seed=8, backflow=1.0)
    states = []
    for a in range(lat.N):
        for b in range(lat.N):
            o = np.zeros(lat.N, dtype=np.int8)
            o[a] += 1
            o[b] += 2
            states.append(o)
    w = np.array([np.exp(2 * log_psi(lat, p, o)[1]) for o in states])
    prob = w / w.sum()
    key = {o.tobytes(): k for k, o in enumerate(states)}
    counts = np.zeros(len(states))
    init = wl.random_occupations(lat, 16, seed=3)
    for wk in range(16):
        o, pos = init[wk], initial_labels(lat, init[wk])
        o, pos, _ = metropolis(lat, p, o, pos, wk, seed=99, step0=0, n_sweeps=10)
        for blk in range(120):
            o, pos, _ = metropolis(lat, p, o, pos, wk, seed=99, step0=(blk + 1) * 4 * lat.N,
                                   n_sweeps=4)
            assert np.sum(o & 1) == 1 and np.sum((o >> 1) & 1) == 1
            counts[key[o.tobytes()]] += 1
    n = counts.sum()
    exp = n * prob
    mask = exp > 5
    chi2 = np.sum((counts[mask] - exp[mask]) ** 2 / exp[mask])
    dof = mask.sum() - 1
    # 4 sweeps between samples decorrelate this 36-state chain well; allow a
    # generous bound (mean dof, sd sqrt(2 dof)) with autocorrelation slack
    assert chi2 < dof + 8 * np.sqrt(2 * dof) + 20
