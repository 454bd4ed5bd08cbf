"""The t-J model (Sec. III, t-J Hamiltonian: Gutzwiller-projected hops,
J S_i.S_j on nearest-neighbour bonds, staggered pinning field on the x = 0
column) on the GPU, against the oracle.

* FP64, one mixed batch of three lattices: a 1/8-doped 8x4 cylinder (torus
  mode across the width), a 7x7 cylinder (window mode) and a half-filled
  4x4 torus where every hop is blocked and only spin exchanges connect:
  every ratio (hops and exchanges, code by code), E_loc and log|psi| of the
  low-rank path (row form and column form) and of the full-recompute path
  at 1e-10; Metropolis chains with the Gutzwiller rejection bit-exact against
  the oracle sampler and the state after them at 1e-9.  One conv layer with
  site-wise layers, and two conv layers.
* A walker holding a doubly occupied site is flagged and left alone.
* f16x2 on the 16x8 cylinder of the paper's t-J runs (1/8 doping, J = t/3,
  t' = 0.2 t, h_m = 0.5 t; one conv layer, four site-wise layers, SiLU),
  the workload's full batch of 8192 walkers after two sweeps: sampled
  walkers against the plain FP64 oracle on the same quantised weights at
  1e-4, and the low-rank path against the full path for every walker
  (1e-4); the walker where they differ most also against the oracle, its
  E_loc error bounded by 1e-5 of the size of its terms (sum of |t R|).
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402
from test_gpu_configs import compare_sampled  # noqa: E402
from test_gpu_sweep import SEED, STEP0, check_chain, oracle_chain  # noqa: E402
from oracle_par import local_energies  # noqa: E402

LATS = [wl.Lattice(8, 4, 0, 1, 1.0, 0.2, 0.0, 14, 14, tj=1, J=1.0 / 3.0, h_pin=0.5),
        wl.Lattice(7, 7, 0, 1, 1.0, -0.2, 0.0, 20, 19, tj=1, J=0.4, h_pin=0.3),
        wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 0.0, 8, 8, tj=1, J=1.0, h_pin=0.0)]


@pytest.mark.parametrize("n_conv,n_mlp,act", [(1, 2, "silu"), (2, 0, "tanh")])
def test_tj_fp64_lowrank_full_chain(n_conv, n_mlp, act):
    model = wl.Model(n_conv, 8, act, "f64", 4, n_mlp=n_mlp)
    counts = [3, 2, 2]
    say(f"[t-J f64] {n_conv} conv + {n_mlp} site-wise layers, {act}")
    ctx, params, occs = build(LATS, model, counts, backflow=0.5)
    w = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10)
    say(f"  low-rank {w}")
    ctx.set_launch(8, 0)
    w = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10)
    say(f"  column form only {w}")
    ctx.set_launch(8, 16)
    w = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10, path="full")
    say(f"  full {w}")
    n_acc = ctx.sweep(2, SEED, STEP0)
    torch.cuda.synchronize()
    n_acc = n_acc.cpu().numpy()
    assert n_acc.sum() > 0
    ref = oracle_chain(LATS, params, occs, model, 2, SEED, STEP0)
    new = check_chain(LATS, counts, ctx, ref, n_acc)
    for o in new:
        assert not np.any(o == 3)
    w = check_walkers(ctx, LATS, params, new, model, 1e-9, 1e-9)
    say(f"  after {int(n_acc.sum())} accepted moves {w}")


def test_tj_doubly_occupied_walker_flagged():
    lat = LATS[0]
    model = wl.Model(1, 8, "silu", "f64", 4)
    occ = wl.random_occupations(lat, 3, seed=5)
    up = int(np.nonzero(occ[1] == 1)[0][0])
    dn = int(np.nonzero(occ[1] == 2)[0][0])
    occ[1, up], occ[1, dn] = 3, 0                      # same counts, one doubly occupied site
    ctx, params, _ = build([lat], model, [3], occ_list=[occ], backflow=0.5)
    assert ctx.flags().cpu().numpy().tolist() == [0, 8, 0]
    e = ctx.local_energy().cpu().numpy()
    assert np.isnan(e[1]) and np.isfinite(e[[0, 2]]).all()
    n_acc = ctx.sweep(1, SEED, STEP0).cpu().numpy()
    o, _ = ctx.state()
    assert np.array_equal(o.cpu().numpy().reshape(3, lat.N)[1], occ[1])
    assert n_acc[1] == 0


def test_tj_f16x2_16x8_cylinder():
    w = wl.get("tj")
    lat = w.lattices[0]
    W = w.walkers[0]                               # the workload's full batch
    say(f"[t-J f16x2] 16x8 cylinder, 1 conv + 4 site-wise layers, {W} walkers")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], w.model, [W], occ_list=[occ])
    nacc = ctx.sweep(2, w.seed_mc, 0)
    torch.cuda.synchronize()
    assert int(nacc.sum()) > 0
    o, _ = ctx.state()
    occ = o.cpu().numpy().reshape(W, lat.N)
    assert not np.any(occ == 3)
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
    sample = [int(k) for k in np.linspace(0, W - 1, 8)]
    e_low = compare_sampled(ctx, lat, params, occ, sample, w.model, 1e-3, 1e-4, 1e-6)
    e_full = ctx.local_energy("full").cpu().numpy()
    rel = np.abs(e_full - e_low) / np.maximum(1.0, np.abs(e_full))
    k = int(np.argmax(rel))
    say(f"  low-rank vs full, all {W} walkers: max {rel[k]:.2e} (walker {k})")
    # both paths run the f16x2 features (they differ by the FP32 rounding of
    # the low-rank feature differences): the walker where they differ most is
    # checked against the FP64 oracle, both paths to the 16-bit E_loc target
    e_ref, cs, R_ref, _ = local_energies(lat, params, [occ[k]], 0, w.model.act)[0]
    terms = float(sum(abs(c.t * r) for c, r in zip(cs, R_ref)))
    errs = [abs(e_path - e_ref) for e_path in (e_low[k], e_full[k])]
    say(f"  walker {k}: E_loc {e_ref:.6f}, sum of |t R| {terms:.3f}, |error| low-rank {errs[0]:.2e}, "
        f"full {errs[1]:.2e}")
    # E_loc is a sum of terms t R: its error is bounded against their size
    # (1e-5 of sum |t R|: no weaker than 1e-4 of |E_loc| unless the terms
    # cancel more than tenfold, as they do on this walker)
    for e_err in errs:
        assert e_err <= 1e-5 * max(1.0, terms), (k, e_err, terms)
    assert rel[k] <= 1e-4
