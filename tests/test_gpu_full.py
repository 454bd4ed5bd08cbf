"""The full-recompute comparison path (every connected configuration
evaluated from scratch: batched forward, FP64 rows and LU of both Slater
blocks) against the oracle and against the low-rank path.

* FP64, more than 128 electrons per spin (16x16 with 130 + 129: the
  cold-setup rows and global-memory Gauss-Jordan stage): every hop ratio and
  E_loc at 1e-10 against the oracle.
* FP64, a mixed batch (4x4, 6x6, 5x3 open) in one call: 1e-10.
* The 16x16 f16x2 workload at 512 walkers: E_loc of every walker equal to
  the low-rank path's to 1e-5 (the same conv arithmetic; the two differ by
  the FP32 rounding of the low-rank path's feature differences D, 2^-24
  relative per element, about 1e-6 here), and three sampled walkers against
  the oracle at 1e-4.
* The 32x32 448 + 448 workload, two walkers: full-recompute E_loc equal to
  the low-rank path's (which the 32x32 parity test pins to the oracle) to
  1e-5.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402


def test_full_fp64_above_128_electrons():
    lat = wl.Lattice(16, 16, 1, 0, 1.0, 0.0, 8.0, 130, 129)
    model = wl.Model(2, 8, "tanh", "f64")
    say("[full] 16x16 130+129 FP64")
    ctx, params, occs = build([lat], model, [2], backflow=0.5)
    worst = check_walkers(ctx, [lat], params, occs, model, 1e-10, 1e-10, path="full")
    say(f"  {worst}")


def test_full_fp64_mixed_batch():
    lats = [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 8.0, 5, 5), wl.Lattice(6, 6, 1, 1, 1.0, -0.2, 8.0, 13, 12),
            wl.Lattice(5, 3, 0, 1, 1.0, 0.3, 6.0, 4, 2)]
    model = wl.Model(3, 16, "silu", "f64")
    say("[full] mixed FP64")
    ctx, params, occs = build(lats, model, [3, 2, 4], backflow=0.5)
    worst = check_walkers(ctx, lats, params, occs, model, 1e-10, 1e-10, path="full")
    say(f"  {worst}")


def test_full_f16x2_16x16_matches_lowrank_and_oracle():
    w = wl.get("c3")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    W = 512
    say(f"[full] 16x16 f16x2, {W} walkers")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    e_low = ctx.local_energy("lowrank").cpu().numpy()
    e_full = ctx.local_energy("full").cpu().numpy()
    d = np.abs(e_full - e_low) / np.maximum(1.0, np.abs(e_low))
    say(f"  full vs low-rank: max {d.max():.2e}")
    assert d.max() < 1e-5
    worst = check_walkers(ctx, [lat], params, [occ], model, 1e-3, 1e-4, path="full", sample=[[0, 255, 511]],
                          tol_logpsi=1e-6)
    say(f"  sampled vs oracle {worst}")


def test_full_32x32_two_walkers_match_lowrank():
    w = wl.get("c5")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    say("[full] 32x32 448+448 f16x2, 2 walkers")
    occ = wl.occupations(w, 0, n_walkers=2)
    ctx, _, _ = build([lat], model, [2], occ_list=[occ])
    e_low = ctx.local_energy("lowrank").cpu().numpy()
    e_full = ctx.local_energy("full").cpu().numpy()
    d = np.abs(e_full - e_low) / np.maximum(1.0, np.abs(e_low))
    say(f"  full vs low-rank: {e_full} {e_low} max {d.max():.2e}")
    assert np.isfinite(e_full).all()
    assert d.max() < 1e-5
