"""Site-wise MLP layers after the conv stack (Sec. II.B, site-wise MLP
equation: H <- act(H W_m + b_m) at every site, no residual) on the GPU,
against the oracle.

* FP64, one batch of a window-mode lattice (8x7 periodic-x / open-y) and a
  torus-mode one (4x4 periodic, t' != 0 so diagonal hops too): every hop
  ratio, E_loc and log|psi| of the low-rank path and of the full-recompute
  path at 1e-10; the Jacobian against the oracle's autograd at 1e-10;
  Metropolis chains bit-exact against the oracle sampler (the accepted moves
  commit the site-wise layers' planes on the box), the maintained state at
  1e-9 and after a refresh at 1e-10.  One conv layer (boxes of 12-16 sites:
  the row form) and two conv layers (also the column form).
* f16x2 at 16x16 (the paper's head shape: one conv layer, four site-wise
  layers, SiLU) after sweeps: sampled walkers against the plain FP64 oracle
  on the same quantised weights (E_loc 1e-4), and the low-rank path against
  the full-recompute path on the same GPU (1e-5: both round the features to
  the same FP16 pairs; the products differ only in summation order).
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402
from test_gpu_configs import compare_sampled  # noqa: E402
from test_gpu_grad import check_rows, jac_ref  # noqa: E402
from test_gpu_sweep import SEED, STEP0, check_chain, oracle_chain  # noqa: E402

LATS = [wl.Lattice(8, 7, 1, 0, 1.0, 0.0, 4.0, 10, 9), wl.Lattice(4, 4, 1, 1, 1.0, 0.2, 4.0, 5, 5)]


@pytest.mark.parametrize("n_conv,n_mlp,act", [(1, 4, "silu"), (2, 2, "tanh")])
def test_mlp_fp64_lowrank_full_grad_chain(n_conv, n_mlp, act):
    model = wl.Model(n_conv, 8, act, "f64", 4, n_mlp=n_mlp)
    counts = [3, 2]
    say(f"[mlp f64] {n_conv} conv + {n_mlp} site-wise layers, {act}")
    ctx, params, occs = build(LATS, model, counts, backflow=0.5)
    w = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10)
    say(f"  low-rank {w}")
    w = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10, path="full")
    say(f"  full {w}")
    # the column form as well as the row form
    ctx.set_launch(8, 0)
    w = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10)
    say(f"  column form only {w}")
    ctx.set_launch(8, 16)
    J = ctx.grad_logpsi().cpu().numpy()
    assert J.shape == (sum(counts), ctx.num_params)
    say(f"  Jacobian worst {check_rows(J, jac_ref(LATS, params, occs, act), 1e-10):.3e}")
    n_acc = ctx.sweep(2, SEED, STEP0)
    torch.cuda.synchronize()
    n_acc = n_acc.cpu().numpy()
    assert n_acc.sum() > 0
    ref = oracle_chain(LATS, params, occs, model, 2, SEED, STEP0)
    new = check_chain(LATS, counts, ctx, ref, n_acc)
    w = check_walkers(ctx, LATS, params, new, model, 1e-9, 1e-9)
    say(f"  after {int(n_acc.sum())} accepted moves {w}")
    ctx.refresh()
    assert not (ctx.flags().cpu().numpy() & 4).any()
    check_walkers(ctx, LATS, params, new, model, 1e-10, 1e-10)


def test_mlp_f16x2_16x16_scale_head():
    w = wl.get("c3")
    lat = w.lattices[0]
    model = wl.Model(1, 32, "silu", "f16x2", 32, n_mlp=4)
    W = 256
    say(f"[mlp f16x2] 16x16, 1 conv + 4 site-wise layers, {W} walkers")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    nacc = ctx.sweep(2, w.seed_mc, 0)
    torch.cuda.synchronize()
    assert int(nacc.sum()) > 0
    o, _ = ctx.state()
    occ = o.cpu().numpy().reshape(W, lat.N)
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
    sample = [int(k) for k in np.linspace(0, W - 1, 8)]
    e_low = compare_sampled(ctx, lat, params, occ, sample, model, 1e-3, 1e-4, 1e-6)
    e_full = ctx.local_energy("full").cpu().numpy()
    d = float(np.max(np.abs(e_full - e_low) / np.maximum(1.0, np.abs(e_full))))
    say(f"  low-rank vs full: {d:.2e}")
    assert d <= 1e-5
