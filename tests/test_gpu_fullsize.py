"""Parity at the full workload sizes, in the launch configuration the
benchmark times (all walkers of the batch in one launch), on sampled walkers
the oracle evaluates one by one, plus properties checked on every walker.

* 16x16 periodic-x / open-y, 112 + 112, 4 layers x 32 channels, bf16x3 conv,
  8192 walkers, after one Metropolis sweep: E_loc within 1e-4, every hop
  ratio within 1e-3 and log|psi| within 1e-6 on three sampled walkers; all
  E_loc finite, no walker flagged.
* Mixed batch 8x8 / 12x12 / 16x8 (28 / 63 / 56 per spin), 4 layers x 24
  channels, FP32 conv, 2048 walkers per lattice in one launch, after the
  workload's 8 thermalising sweeps: sampled walkers of every lattice against
  the oracle (every ratio 1e-3, E_loc 1e-4), and the gradient rows of those
  walkers against the oracle's autograd gradient.
* The benchmark workload (16x16, 4 x 32, f16x2, 8192 walkers after a
  sweep): the VJP with random weights, formed launch by launch over the
  walkers, against J^T v from the library's own Jacobian rows (1e-12 of the
  largest |entry|), and two sampled rows against the oracle's autograd
  gradient (2e-5, the FP32-feature bound).
* The same three lattices and network shape in FP64, two walkers each in
  one batch: the library's gradient rows against central differences of
  the library's own log|psi| (parameters moved by +-h, the context reloaded)
  on parameters of every kind, no oracle involved.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402


def test_headline_8192_walkers_after_sweep():
    w = wl.get("c3")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "bf16x3", 32)
    W = w.walkers[0]
    say(f"[fullsize] 16x16 bf16x3, {W} walkers, 1 sweep")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    nacc = ctx.sweep(1, w.seed_mc, 0)
    torch.cuda.synchronize()
    say(f"  accept rate {float(nacc.double().mean()) / lat.N:.3f}")
    o, _ = ctx.state()
    occs = [o.cpu().numpy().reshape(W, lat.N)]
    e = ctx.local_energy().cpu().numpy()
    assert np.isfinite(e).all()
    f = ctx.flags().cpu().numpy()
    say(f"  flags: singular {int((f & 1).astype(bool).sum())} nonfinite {int((f & 2).astype(bool).sum())} "
        f"drift {int((f & 4).astype(bool).sum())} badcount {int((f & 8).astype(bool).sum())}")
    # DRIFT only reports that the Woodbury-maintained G had moved more than
    # 1e-8 from exact unit rows before a refresh (the refresh repairs it)
    assert not (f & (1 | 2 | 8)).any()
    assert (f & 4).astype(bool).sum() <= W // 1000
    sample = [[0, W // 2 + 1, W - 1]]
    worst = check_walkers(ctx, [lat], params, occs, model, 1e-3, 1e-4, sample=sample, tol_logpsi=1e-6)
    say(f"  sampled walkers vs oracle {worst}")


def test_mixed_lattices_2048_each_with_gradient():
    from oracle.grad import autograd_grad
    w = wl.get("c4")
    lats = list(w.lattices)
    model = wl.Model(4, 24, "tanh", "f32", 32)
    counts = list(w.walkers)
    say(f"[fullsize] mixed {[(l.Lx, l.Ly) for l in lats]} f32, {counts} walkers")
    occs = [wl.occupations(w, li, n_walkers=c) for li, c in enumerate(counts)]
    ctx, params, _ = build(lats, model, counts, occ_list=occs)
    # the workload's thermalising sweeps first: E_loc on |psi|^2 samples
    ctx.sweep(w.sweeps, w.seed_mc, 0)
    o, _ = ctx.state()
    o = o.cpu().numpy()
    occs, off = [], 0
    for lat, c in zip(lats, counts):
        occs.append(o[off:off + c * lat.N].reshape(c, lat.N))
        off += c * lat.N
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
    e = ctx.local_energy().cpu().numpy()
    assert np.isfinite(e).all()
    sample = [[0, c // 2, c - 1] for c in counts]
    worst = check_walkers(ctx, lats, params, occs, model, 1e-3, 1e-4, sample=sample, tol_logpsi=1e-6)
    say(f"  sampled walkers vs oracle {worst}")
    J = ctx.grad_logpsi().cpu().numpy()
    assert J.shape == (sum(counts), ctx.num_params)
    w0 = 0
    for li, lat in enumerate(lats):
        g_ref = autograd_grad(lat, params, occs[li][0], li, model.act)[1]
        scale = max(1.0, float(np.max(np.abs(g_ref))))
        err = float(np.max(np.abs(J[w0] - g_ref))) / scale
        say(f"  gradient lattice {li}: max err / scale {err:.2e}")
        assert err <= 2e-5
        w0 += counts[li]


def test_c4_lattices_gradient_by_finite_differences_of_the_library():
    from oracle.grad import pack, unpack
    w = wl.get("c4")
    lats = w.lattices
    model = wl.Model(4, 24, "tanh", "f64")
    counts = [2] * len(lats)
    say("[fullsize] mixed 8x8/12x12/16x8, 4 x 24 FP64: gradient vs central differences")
    occs = [wl.occupations(w, li, n_walkers=c) for li, c in enumerate(counts)]
    ctx, params, _ = build(lats, model, counts, occ_list=occs, backflow=0.5)
    flat = np.concatenate([o.reshape(-1) for o in occs]).astype(np.int8)
    J = ctx.grad_logpsi().cpu().numpy()
    theta = pack(params)
    assert J.shape == (sum(counts), theta.size)
    rng = np.random.default_rng(5)
    # every kind of parameter: embedding, conv kernels and biases, each
    # lattice's projection (the tail of the vector), plus random indices
    n_conv = params.conv_w.size + params.conv_b.size
    idx = np.unique(np.concatenate([[0, params.embed.size, params.embed.size + params.conv_w.size,
                                     params.embed.size + n_conv, theta.size - 1],
                                    rng.choice(theta.size, 40, replace=False)]))
    h = 1e-5
    fd = np.empty((sum(counts), len(idx)))
    for n, j in enumerate(idx):
        la = []
        for dh in (h, -h):
            tp = theta.copy()
            tp[j] += dh
            ctx.set_params_from(unpack(tp, params))
            ctx.load(counts, flat)
            la.append(ctx.log_psi()[1].cpu().numpy())
        fd[:, n] = (la[0] - la[1]) / (2 * h)
    ctx.set_params_from(params)
    for k in range(sum(counts)):
        scale = max(1.0, float(np.max(np.abs(fd[k]))))
        err = float(np.max(np.abs(J[k, idx] - fd[k]))) / scale
        say(f"  walker {k}: max |J - FD| / scale {err:.2e}")
        assert err <= 1e-6


def test_headline_vjp_against_jacobian_rows():
    from oracle.grad import autograd_grad
    w = wl.get("c3")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    W = w.walkers[0]
    say(f"[fullsize] 16x16 f16x2, {W} walkers: VJP against the Jacobian rows")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, params, _ = build([lat], model, [W], occ_list=[occ])
    ctx.sweep(1, w.seed_mc, 0)
    o, _ = ctx.state()
    o = o.cpu().numpy().reshape(W, lat.N)
    v = torch.from_numpy(np.random.default_rng(3).standard_normal(W)).cuda()
    g = ctx.grad_logpsi(v)
    J = ctx.grad_logpsi()
    ref = J.t().matmul(v)
    scale = float(ref.abs().max())
    err = float((g - ref).abs().max()) / scale
    say(f"  VJP vs J^T v: max err / max |entry| {err:.2e}")
    assert err <= 1e-12
    Jh = J[[0, W - 1]].cpu().numpy()
    del J
    for row, k in zip(Jh, (0, W - 1)):
        gr = autograd_grad(lat, params, o[k], 0, model.act)[1]
        e = float(np.max(np.abs(row - gr))) / max(1.0, float(np.max(np.abs(gr))))
        say(f"  walker {k}: row vs oracle autograd {e:.2e}")
        assert e <= 2e-5
