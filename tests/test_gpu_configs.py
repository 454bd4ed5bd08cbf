"""Parity on the configurations the benchmark and its configuration list
name, at their full sizes, in the launch configuration the benchmark times.

* 4x4 periodic, U = 4, 5 + 5 (closed shell), 2 layers x 8 channels, all
  FP64, 256 walkers x 20 Metropolis sweeps of 16 proposals: the chains
  (occupations, electron positions, accept counts) bit-exact with the
  oracle's sampler, then every walker's E_loc and hop ratios at 1e-10.
* 8x8 periodic, t' = -0.2, U = 8, 28 + 28, 4 layers x 16 channels, FP32
  conv, 4096 walkers after the workload's 8 thermalising sweeps: the
  low-rank E_loc of every walker equal to the full-recompute path's to 1e-5
  (both use the same FP32 conv; they differ by the FP32 rounding of the
  low-rank path's feature differences, 2^-24 relative per element), and 16
  walkers spread over the batch against the FP64 oracle (E_loc 1e-4, hop
  ratios 1e-3, log|psi| 1e-6). Here the layer-4 box covers the whole
  lattice, so every ratio takes the column form of the determinant lemma.
* 16x16 periodic-x / open-y, 112 + 112, 4 layers x 32 channels, the
  benchmark's f16x2 conv mode and parameters, 8192 walkers after the
  benchmark's 8 thermalising sweeps, at the slice count the autotuner picks:
  16 walkers spread over the batch against the plain FP64 oracle (E_loc
  1e-4, hop ratios 1e-3, log|psi| 1e-6), every hop code checked.
* 32x32 periodic-x / open-y, 448 + 448 stripe-seeded, 4 x 32, f16x2, all
  1024 walkers in one launch: the full E_loc of two walkers against the
  oracle at 1e-4 (every one of their ~1960 hop ratios recomputed in full by
  the oracle, spread over host processes), and a Metropolis sweep whose
  maintained state (features, G and P by Woodbury, log|psi| by ratio
  products) equals a context loaded fresh from the swept configurations.

The oracle's hops run in host processes (tests/oracle_par.py); the GPU runs
through the C ABI.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, hop_code, rel_err, say  # noqa: E402
from oracle_par import chains, local_energies  # noqa: E402


def compare_sampled(ctx, lat, params, occ, sample, model, tol_ratio, tol_eloc, tol_logpsi):
    eloc, nh, code, rat = ctx.local_energy(ratios=True)
    sign, la = ctx.log_psi()
    torch.cuda.synchronize()
    eloc, nh, code, rat = eloc.cpu().numpy(), nh.cpu().numpy(), code.cpu().numpy(), rat.cpu().numpy()
    sign, la = sign.cpu().numpy(), la.cpu().numpy()
    ref = local_energies(lat, params, [occ[k] for k in sample], 0, model.act)
    worst = {"ratio": 0.0, "eloc": 0.0, "logpsi": 0.0}
    for k, (e_ref, hs, R_ref, (s_ref, l_ref)) in zip(sample, ref):
        assert sign[k] == s_ref, k
        worst["logpsi"] = max(worst["logpsi"], abs(la[k] - l_ref) / max(1.0, abs(l_ref)))
        assert nh[k] == len(hs), (k, nh[k], len(hs))
        assert list(code[k, :len(hs)]) == [hop_code(h, lat.N) for h in hs], k
        floor = 1e-3 * np.sqrt(np.mean(R_ref ** 2))
        for r, rr in zip(rat[k, :len(hs)], R_ref):
            worst["ratio"] = max(worst["ratio"], rel_err(r, rr, floor))
        worst["eloc"] = max(worst["eloc"], rel_err(eloc[k], e_ref, 1.0))
    say(f"  {len(sample)} sampled walkers vs oracle: {worst}")
    assert worst["logpsi"] <= tol_logpsi, worst
    assert worst["ratio"] <= tol_ratio, worst
    assert worst["eloc"] <= tol_eloc, worst
    return eloc


def test_c1_256_walkers_20_sweeps_fp64_bit_exact():
    w = wl.get("c1")
    lat = w.lattices[0]
    model = w.model
    W, ns = w.walkers[0], w.sweeps
    say(f"[c1] 4x4, {W} walkers x {ns} sweeps, FP64")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    n_acc = ctx.sweep(ns, w.seed_mc, 0).cpu().numpy()
    o2, pos = ctx.state()
    o2 = o2.cpu().numpy().reshape(W, lat.N)
    pos = pos.cpu().numpy()
    ref = chains(lat, params, occ, 0, w.seed_mc, 0, ns, 0, model.act)
    for k, (ro, rp, ra) in enumerate(ref):
        assert np.array_equal(o2[k], ro), k
        assert np.array_equal(pos[k, 0, :lat.n_up].astype(np.int64), rp[0]), k
        assert np.array_equal(pos[k, 1, :lat.n_dn].astype(np.int64), rp[1]), k
        assert int(n_acc[k]) == ra, (k, int(n_acc[k]), ra)
    say(f"  chains bit-exact; accept rate {n_acc.sum() / (W * ns * lat.N):.3f}")
    assert not ctx.flags().cpu().numpy().any()
    compare_sampled(ctx, lat, params, o2, range(W), model, 1e-10, 1e-10, 1e-10)


def test_c2_fp32_4096_lowrank_vs_full_and_oracle():
    w = wl.get("c2")
    lat = w.lattices[0]
    model = w.model
    W = w.walkers[0]
    say(f"[c2] 8x8 t'=-0.2 FP32 conv, {W} walkers, {w.sweeps} sweeps")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    nacc = ctx.sweep(w.sweeps, w.seed_mc, 0)
    torch.cuda.synchronize()
    say(f"  accept rate {float(nacc.double().mean()) / (w.sweeps * lat.N):.3f}")
    o, _ = ctx.state()
    occ = o.cpu().numpy().reshape(W, lat.N)
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
    e_low = ctx.local_energy("lowrank").cpu().numpy()
    e_full = ctx.local_energy("full").cpu().numpy()
    assert np.isfinite(e_low).all() and np.isfinite(e_full).all()
    d = np.abs(e_full - e_low) / np.maximum(1.0, np.abs(e_low))
    say(f"  low-rank vs full-recompute, all {W} walkers: max {d.max():.2e}")
    assert d.max() <= 1e-5
    sample = [int(k) for k in np.linspace(0, W - 1, 16)]
    compare_sampled(ctx, lat, params, occ, sample, model, 1e-3, 1e-4, 1e-6)


def test_c3_f16x2_bench_mode_8192_after_sweeps_tuned():
    w = wl.get("c3")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    W = w.walkers[0]
    say(f"[c3] 16x16 f16x2, {W} walkers, {w.sweeps} sweeps, tuned launch")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    nacc = ctx.sweep(w.sweeps, w.seed_mc, 0)
    torch.cuda.synchronize()
    say(f"  accept rate {float(nacc.double().mean()) / (w.sweeps * lat.N):.3f}")
    o, _ = ctx.state()
    occ = o.cpu().numpy().reshape(W, lat.N)
    slices = ctx.tune()
    say(f"  autotuner: {slices} slices per walker")
    f = ctx.flags().cpu().numpy()
    assert not (f & (1 | 2 | 8)).any()
    sample = [int(k) for k in np.linspace(0, W - 1, 16)]
    e = compare_sampled(ctx, lat, params, occ, sample, model, 1e-3, 1e-4, 1e-6)
    assert np.isfinite(e).all()


def test_c5_f16x2_full_batch_eloc_and_sweep():
    w = wl.get("c5")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    W = w.walkers[0]
    say(f"[c5] 32x32 448+448 f16x2, {W} walkers")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    f = ctx.flags().cpu().numpy()
    assert not (f & (1 | 2 | 8)).any()
    compare_sampled(ctx, lat, params, occ, [0, W - 1], model, 1e-3, 1e-4, 1e-6)
    del ctx
    # one sweep of 64 walkers (1024 proposals each, Woodbury updates of the
    # 448-column blocks), then the maintained state against a fresh load
    nw = 64
    ctx, _, _ = build([lat], model, [nw], occ_list=[occ[:nw]])
    n_acc = ctx.sweep(1, w.seed_mc, 0).cpu().numpy()
    say(f"  sweep: accept rate {n_acc.mean() / lat.N:.3f}")
    assert n_acc.sum() > 0
    f = ctx.flags().cpu().numpy()
    assert not (f & (1 | 2 | 8)).any()
    o, _ = ctx.state()
    o = o.cpu().numpy().reshape(nw, lat.N)
    e1 = ctx.local_energy().cpu().numpy()
    s1, l1 = (t.cpu().numpy() for t in ctx.log_psi())
    ctx2, _, _ = build([lat], model, [nw], occ_list=[o])
    e2 = ctx2.local_energy().cpu().numpy()
    s2, l2 = (t.cpu().numpy() for t in ctx2.log_psi())
    dl = np.max(np.abs(l1 - l2) / np.maximum(1.0, np.abs(l2)))
    de = np.max(np.abs(e1 - e2) / np.maximum(1.0, np.abs(e2)))
    say(f"  swept vs fresh: log|psi| {dl:.3e}  E_loc {de:.3e}")
    assert np.array_equal(s1, s2)
    assert dl < 1e-8
    assert de < 1e-6
