"""Slater blocks above 128 electrons per spin: the global-memory Gauss-Jordan
inverse, 16-bit hop codes, and the sweep's Woodbury update over more than one
block of label columns.

* 16x16 periodic-x / open-y with 130 + 129 electrons (one column block) and
  24x24 periodic with 300 + 300 (two blocks), FP64 conv: log|psi|, every hop
  ratio and E_loc at 1e-10 against the oracle, and the Metropolis chain
  bit-exact with the oracle's.
* The 32x32 periodic-x / open-y workload at 1/8 doping (448 + 448,
  stripe-seeded, 4 layers x 32 channels, bf16x3 conv) at its full 1024
  walkers: the oracle evaluates log|psi| and a sample of hop ratios of
  sampled walkers (a full E_loc there costs it minutes); E_loc of every
  walker must equal U * doubles - t * sum of its own reported ratios.
* The per-spin limit of the library, 512 + 512 at half filling on a 32x32
  torus, FP64 (2 layers x 8 channels): log|psi| and E_loc at 1e-10 and
  every hop ratio at 1e-9 of one walker against the oracle (its hops spread over host
  processes); after one sweep of two walkers the maintained state (G and P
  by Woodbury over four column blocks, log|psi| by ratio products) equals a
  context loaded fresh from the new configurations; 513 electrons of one
  spin are refused.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, hop_code, say  # noqa: E402
from oracle.ansatz import log_psi  # noqa: E402
from oracle.energy import jw_sign  # noqa: E402
from oracle.lattice import apply_hop, hops  # noqa: E402
from oracle.sampler import initial_labels, metropolis  # noqa: E402
from oracle_par import local_energies  # noqa: E402

SEED = 424242


def chain_check(ctx, lat, params, occs, model, ns):
    n_acc = ctx.sweep(ns, SEED, 3).cpu().numpy()
    occ, pos = ctx.state()
    occ = occ.cpu().numpy().reshape(len(occs), lat.N)
    pos = pos.cpu().numpy()
    for w, o in enumerate(occs):
        o2, p2, na = metropolis(lat, params, o, initial_labels(lat, o), w, SEED, 3, ns, act=model.act)
        assert np.array_equal(occ[w], o2), w
        for sp in range(2):
            n = (lat.n_up, lat.n_dn)[sp]
            assert np.array_equal(pos[w, sp, :n].astype(np.int64), p2[sp]), (w, sp)
        assert int(n_acc[w]) == na, (w, int(n_acc[w]), na)
    say(f"  chain bit-exact, accepted {n_acc.tolist()}")
    return [occ]


@pytest.mark.parametrize("name,lat,nw", [
    ("16x16_130+129_one_block", wl.Lattice(16, 16, 1, 0, 1.0, 0.0, 8.0, 130, 129), 2),
    ("24x24_300+300_two_blocks", wl.Lattice(24, 24, 1, 1, 1.0, 0.0, 8.0, 300, 300), 1),
])
def test_big_blocks_fp64(name, lat, nw):
    model = wl.Model(2, 8, "tanh", "f64", 16)
    say(f"[big f64] {name}")
    ctx, params, occs = build([lat], model, [nw], backflow=0.5)
    worst = check_walkers(ctx, [lat], params, occs, model, 1e-10, 1e-10)
    say(f"  E_loc parity {worst}")
    new = chain_check(ctx, lat, params, occs[0], model, 1)
    worst = check_walkers(ctx, [lat], params, new, model, 1e-9, 1e-9)
    say(f"  after the sweep {worst}")


def test_32x32_448_full_batch_sampled():
    w = wl.get("c5")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "bf16x3", 32)
    W = w.walkers[0]
    say(f"[big c5] 32x32 448+448, {W} walkers, bf16x3")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    eloc, nh, code, rat = ctx.local_energy(ratios=True)
    sign, la = ctx.log_psi()
    eloc, nh, code, rat = eloc.cpu().numpy(), nh.cpu().numpy(), code.cpu().numpy(), rat.cpu().numpy()
    sign, la = sign.cpu().numpy(), la.cpu().numpy()
    f = ctx.flags().cpu().numpy()
    assert not (f & (1 | 2 | 8)).any()
    assert np.isfinite(eloc).all()
    # E_loc = U * doubles - t * sum of the walker's reported ratios (t' = 0)
    for k in range(W):
        e = lat.U * np.sum(occ[k] == 3) - lat.t * np.sum(rat[k, :nh[k]])
        assert abs(eloc[k] - e) <= 1e-9 * max(1.0, abs(e)), k
    rng = np.random.default_rng(5)
    for k in (0, W - 1):
        s_ref, l_ref = log_psi(lat, params, occ[k], 0, model.act)
        assert sign[k] == s_ref
        assert abs(la[k] - l_ref) <= 1e-6 * max(1.0, abs(l_ref)), (k, la[k], l_ref)
        hs = hops(lat, occ[k])
        assert nh[k] == len(hs)
        assert list(code[k, :len(hs)]) == [hop_code(h, lat.N) for h in hs]
        rms = np.sqrt(np.mean(rat[k, :nh[k]] ** 2))
        for hh in rng.choice(len(hs), 6, replace=False):
            h = hs[hh]
            s1, l1 = log_psi(lat, params, apply_hop(occ[k], h), 0, model.act)
            R = jw_sign(occ[k], h.spin, h.i, h.j) * s1 * s_ref * np.exp(l1 - l_ref)
            err = abs(rat[k, hh] - R) / max(abs(R), 1e-3 * rms)
            assert err <= 1e-3, (k, hh, rat[k, hh], R)
        say(f"  walker {k}: log|psi| and 6 sampled ratios agree")
    # one sweep through the two-block Woodbury update (on 32 of the walkers:
    # each accepted move there updates 2 x 1024 x 448 entries of G)
    del ctx
    ctx, _, _ = build([lat], model, [32], occ_list=[occ[:32]])
    n_acc = ctx.sweep(1, SEED, 0).cpu().numpy()
    f = ctx.flags().cpu().numpy()
    say(f"  sweep: accept rate {n_acc.mean() / lat.N:.3f}, flags {int(np.count_nonzero(f))}")
    assert not (f & (1 | 2 | 8)).any()
    assert n_acc.sum() > 0


def test_512_electrons_per_spin_limit():
    from paper_2604_25775_amd._lib import SvmcError
    from paper_2604_25775_amd.api import ScaleVMC
    lat = wl.Lattice(32, 32, 1, 1, 1.0, 0.0, 4.0, 512, 512)
    model = wl.Model(2, 8, "tanh", "f64", 32)
    say("[big] 32x32 512+512 FP64 (the per-spin limit)")
    occ = wl.random_occupations(lat, 2, seed=17)
    ctx, params, _ = build([lat], model, [2], occ_list=[occ], backflow=0.3)
    assert not ctx.flags().cpu().numpy().any()
    eloc, nh, code, rat = (t.cpu().numpy() for t in ctx.local_energy(ratios=True))
    sign, la = (t.cpu().numpy() for t in ctx.log_psi())
    e_ref, hs, R_ref, (s_ref, l_ref) = local_energies(lat, params, [occ[0]], 0, model.act)[0]
    assert sign[0] == s_ref
    assert abs(la[0] - l_ref) <= 1e-10 * max(1.0, abs(l_ref)), (la[0], l_ref)
    assert nh[0] == len(hs)
    assert list(code[0, :len(hs)]) == [hop_code(h, lat.N) for h in hs]
    floor = 1e-3 * np.sqrt(np.mean(R_ref ** 2))
    err = max(abs(r - rr) / max(abs(rr), floor) for r, rr in zip(rat[0, :len(hs)], R_ref))
    # the FP64 bound of the smaller cases, widened for 512-row eliminations
    # on both sides (rounding grows with the order; measured 8.5e-11)
    assert err <= 1e-9, err
    assert abs(eloc[0] - e_ref) <= 1e-10 * max(1.0, abs(e_ref)), (eloc[0], e_ref)
    say(f"  walker 0: {len(hs)} ratios (max err {err:.1e}), E_loc and log|psi| agree")
    n_acc = ctx.sweep(1, SEED, 0).cpu().numpy()
    assert n_acc.sum() > 0
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
    o, _ = ctx.state()
    o = o.cpu().numpy().reshape(2, lat.N)
    e1 = ctx.local_energy().cpu().numpy()
    s1, l1 = (t.cpu().numpy() for t in ctx.log_psi())
    ctx2, _, _ = build([lat], model, [2], occ_list=[o], backflow=0.3)
    e2 = ctx2.local_energy().cpu().numpy()
    s2, l2 = (t.cpu().numpy() for t in ctx2.log_psi())
    assert np.array_equal(s1, s2)
    assert np.max(np.abs(l1 - l2) / np.maximum(1.0, np.abs(l2))) <= 1e-10
    assert np.max(np.abs(e1 - e2) / np.maximum(1.0, np.abs(e2))) <= 1e-9
    say(f"  sweep: accepted {n_acc.tolist()}, maintained state equals a fresh load")
    with pytest.raises(SvmcError) as err:
        ScaleVMC([wl.Lattice(32, 32, 1, 1, 1.0, 0.0, 4.0, 513, 511)], 2, 8)
    assert err.value.status == 5                  # SVMC_ERR_UNSUPPORTED
