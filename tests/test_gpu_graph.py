"""HIP-graph capture of the hot path through the C ABI.

* The local-energy step (per-walker precompute + low-rank E_loc) recorded
  once and replayed several times, with other GPU work and synchronisation
  between replays: every replay equals the eager result bit for bit.
* Metropolis sweeps by svmc_sweep_async (a fixed launch sequence, step0 read from a
  device scalar): two replays with step0 advanced in between reproduce the
  chain of two eager svmc_sweep calls exactly (configurations, electron
  positions, accept counts), and the state afterwards gives the oracle's
  E_loc.
* Both at the benchmark's size: 16x16, 112 + 112, 4 layers x 32 channels,
  f16x2, 8192 walkers at the tuned launch shape: the captured E_loc step
  replayed three times (other GPU work between the replays) equals the
  eager result bit for bit, and a captured sweep replayed twice reproduces
  two eager sweeps of a second context (configurations, electron positions,
  accept counts).
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402


def test_eloc_step_graph_replays_match_eager():
    lat = wl.Lattice(8, 8, 1, 1, 1.0, -0.2, 8.0, 28, 28)
    model = wl.Model(2, 16, "tanh", "bf16x3")
    ctx, params, occs = build([lat], model, [96], backflow=0.3)
    e = torch.empty(96, dtype=torch.float64, device="cuda")
    ctx.prepare()
    ctx.local_energy(out=e)
    torch.cuda.synchronize()
    e_ref = e.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.prepare()
        ctx.local_energy(out=e)
    for rep in range(3):
        e.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(e, e_ref), rep
    say("[graph] E_loc step: 3 replays equal to eager")


def test_sweep_graph_replays_match_eager_chain():
    lat = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)
    model = wl.Model(2, 8, "tanh", "f64", 3)
    W, seed, ns = 6, 99, 2
    ref, params, occs = build([lat], model, [W], backflow=0.5)
    ctx, _, _ = build([lat], model, [W], backflow=0.5)
    ctx.prepare()
    step0 = torch.tensor([5], dtype=torch.int64, device="cuda")
    nacc = torch.zeros(W, dtype=torch.int64, device="cuda")
    ctx.sweep_async(0, seed, step0, nacc)          # allocates outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.sweep_async(ns, seed, step0, nacc)
    nref = torch.zeros(W, dtype=torch.int64, device="cuda")
    for rep in range(2):
        s0 = 5 + rep * ns * lat.N
        ref.sweep(ns, seed, s0, nref)
        step0.fill_(s0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o1, p1 = ctx.state()
        o2, p2 = ref.state()
        assert torch.equal(o1, o2) and torch.equal(p1, p2), rep
        assert torch.equal(nacc, nref), rep
        say(f"[graph] sweep replay {rep}: chain equal to eager, accepted {nacc.tolist()}")
    occ = o1.cpu().numpy().reshape(W, lat.N)
    check_walkers(ctx, [lat], params, [occ], model, 1e-9, 1e-9)


def test_graphs_at_the_benchmark_size():
    w = wl.get("c3")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    W, seed = w.walkers[0], 7
    say(f"[graph] 16x16 f16x2, {W} walkers: E_loc step and sweep replays")
    occ = wl.occupations(w, 0, n_walkers=W)
    ctx, _, _ = build([lat], model, [W], occ_list=[occ])
    ref, _, _ = build([lat], model, [W], occ_list=[occ])
    ctx.sweep(1, w.seed_mc, 0)
    ref.sweep(1, w.seed_mc, 0)
    ctx.tune()
    e = torch.empty(W, dtype=torch.float64, device="cuda")
    ctx.prepare()
    ctx.local_energy(out=e)
    torch.cuda.synchronize()
    e_ref = e.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.prepare()
        ctx.local_energy(out=e)
    for rep in range(3):
        e.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()     # other work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(e, e_ref), rep
    say("  E_loc step: 3 replays equal to eager")
    step0 = torch.tensor([lat.N], dtype=torch.int64, device="cuda")
    nacc = torch.zeros(W, dtype=torch.int64, device="cuda")
    ctx.sweep_async(0, seed, step0, nacc)
    torch.cuda.synchronize()
    gs = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gs):
        ctx.sweep_async(1, seed, step0, nacc)
    nref = torch.zeros(W, dtype=torch.int64, device="cuda")
    for rep in range(2):
        s0 = (1 + rep) * lat.N
        ref.sweep(1, seed, s0, nref)
        step0.fill_(s0)
        torch.cuda.synchronize()
        gs.replay()
        torch.cuda.synchronize()
        o1, p1 = ctx.state()
        o2, p2 = ref.state()
        assert torch.equal(o1, o2) and torch.equal(p1, p2), rep
        assert torch.equal(nacc, nref), rep
        rate = float(nacc.double().mean()) / ((rep + 1) * lat.N)
        say(f"  sweep replay {rep}: {W} chains equal to eager, accept rate {rate:.3f} so far")
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
