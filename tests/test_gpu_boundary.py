"""Boundary features of the C ABI beyond the default network, through the
library, against the oracle.

* per_site_embed: one embedding table per site (the embedding layer as
  Sec. II.B writes it), mixed lattices: low-rank and full-recompute ratios
  and E_loc at 1e-10 (FP64), the Metropolis chain bit-exact with the
  oracle's, the gradient rows at 1e-10 against the oracle's autograd
  gradient; f16x2 at 1e-4 on the 16x16-style geometry.
* svmc_grad_logpsi's FP32 output: the Jacobian and the VJP in FP32 equal the
  FP64 results rounded to nearest.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402
from oracle.grad import autograd_grad  # noqa: E402
from oracle.sampler import initial_labels, metropolis  # noqa: E402

LATS = [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5), wl.Lattice(5, 3, 0, 1, 1.0, 0.3, 6.0, 4, 3)]


def test_per_site_embed_fp64_lowrank_full_chain_grad():
    model = wl.Model(2, 8, "tanh", "f64", 3, per_site_embed=True)
    counts = [4, 5]
    say("[boundary] per-site embedding, FP64, mixed 4x4 / 5x3 open-x")
    ctx, params, occs = build(LATS, model, counts, backflow=0.5)
    assert params.embed_site is not None
    assert ctx.num_params == (16 + 15) * 4 * 8 + 9 * 2 * 64 + 2 * 8 + 8 * 10 + 10 + 8 * 7 + 7
    worst = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10)
    say(f"  low-rank {worst}")
    worst = check_walkers(ctx, LATS, params, occs, model, 1e-10, 1e-10, path="full")
    say(f"  full {worst}")
    J = ctx.grad_logpsi().cpu().numpy()
    w0 = 0
    for li, (lat, occ) in enumerate(zip(LATS, occs)):
        for k in (0, counts[li] - 1):
            g_ref = autograd_grad(lat, params, occ[k], li, model.act)[1]
            err = float(np.max(np.abs(J[w0 + k] - g_ref))) / max(1.0, float(np.max(np.abs(g_ref))))
            assert err <= 1e-10, (li, k, err)
        w0 += counts[li]
    say("  gradient rows agree")
    seed, step0, ns = 77, 5, 2
    n_acc = ctx.sweep(ns, seed, step0).cpu().numpy()
    o, pos = ctx.state()
    o, pos = o.cpu().numpy(), pos.cpu().numpy()
    off, w = 0, 0
    new = []
    for li, (lat, occ) in enumerate(zip(LATS, occs)):
        cur = o[off:off + counts[li] * lat.N].reshape(counts[li], lat.N)
        off += counts[li] * lat.N
        for k in range(counts[li]):
            ro, rp, ra = metropolis(lat, params, occ[k], initial_labels(lat, occ[k]), w, seed, step0, ns,
                                    lat_index=li, act=model.act)
            assert np.array_equal(cur[k], ro), (li, k)
            assert np.array_equal(pos[w, 0, :lat.n_up].astype(np.int64), rp[0])
            assert np.array_equal(pos[w, 1, :lat.n_dn].astype(np.int64), rp[1])
            assert int(n_acc[w]) == ra
            w += 1
        new.append(cur.copy())
    assert n_acc.sum() > 0
    worst = check_walkers(ctx, LATS, params, new, model, 1e-9, 1e-9)
    say(f"  chain bit-exact, maintained state {worst}")


def test_per_site_embed_f16x2_16x16_geometry():
    lat = wl.Lattice(10, 10, 1, 0, 1.0, 0.0, 8.0, 44, 44)
    model = wl.Model(4, 32, "tanh", "f16x2", 32, per_site_embed=True)
    say("[boundary] per-site embedding, f16x2, 10x10 open-y, 4 x 32")
    ctx, params, occs = build([lat], model, [3], backflow=0.1)
    worst = check_walkers(ctx, [lat], params, occs, model, 1e-3, 1e-4, tol_logpsi=1e-6)
    say(f"  {worst}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_grad_fp32_output_is_rounded_fp64(prec):
    lat = wl.Lattice(6, 5, 1, 0, 1.0, 0.0, 8.0, 8, 7)
    model = wl.Model(3, 16, "tanh", prec)
    say(f"[boundary] FP32 gradient output, conv {prec}")
    ctx, params, occs = build([lat], model, [6], backflow=0.3)
    J64 = ctx.grad_logpsi()
    J32 = ctx.grad_logpsi(out_prec="f32")
    assert J32.dtype == torch.float32 and J32.shape == J64.shape
    assert torch.equal(J32, J64.to(torch.float32))
    v = torch.linspace(-1.0, 2.0, 6, dtype=torch.float64, device="cuda")
    g64 = ctx.grad_logpsi(v)
    g32 = ctx.grad_logpsi(v, out_prec="f32")
    assert torch.equal(g32, g64.to(torch.float32))
    assert torch.allclose(g64, (v[:, None] * J64).sum(0), rtol=1e-12, atol=1e-12)
