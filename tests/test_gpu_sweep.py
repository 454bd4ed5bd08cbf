"""GPU Metropolis sweeps (Woodbury updates, masked FP64 refresh) against the
oracle chain, through the C ABI.

FP64 conv: the chain (occupations, electron positions, accept counts) is
bit-exact with the oracle's, which recomputes every ratio in full; both
sides take the accept decision u < ratio^2 in FP64.  Afterwards the state
the sweep maintained (features written on the update box, G and P by
Woodbury, log|psi| by ratio products) must give the oracle's log|psi| and
every hop ratio / E_loc of the new configurations, before and after a
refresh, and no walker may carry the drift flag.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402
from oracle.sampler import initial_labels, metropolis  # noqa: E402

SEED, STEP0 = 20260417, 7

CASES = [
    # name, lattices, model, walkers, sweeps
    ("4x4pbc_L2C8_every3", [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)], wl.Model(2, 8, "tanh", "f64", 3), [8], 3),
    ("3x5open_x_L1C8_silu", [wl.Lattice(3, 5, 0, 1, 1.0, 0.3, 4.0, 4, 3)], wl.Model(1, 8, "silu", "f64", 4),
     [8], 3),
    ("6x6pbc_L3C16", [wl.Lattice(6, 6, 1, 1, 1.0, 0.0, 8.0, 15, 14)], wl.Model(3, 16, "tanh", "f64", 5), [4], 2),
    ("8x8pbc_cform_L2C8", [wl.Lattice(8, 8, 1, 1, 1.0, 0.0, 8.0, 28, 28)], wl.Model(2, 8, "tanh", "f64", 16),
     [3], 2),
    ("10x8_open_y_L4C8", [wl.Lattice(10, 8, 1, 0, 1.0, 0.0, 8.0, 35, 35)], wl.Model(4, 8, "tanh", "f64", 8),
     [2], 1),
    ("mixed_4x4_5x3open", [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 8.0, 5, 5), wl.Lattice(5, 3, 0, 1, 1.0, 0.0, 8.0, 4, 2)],
     wl.Model(2, 8, "tanh", "f64", 4), [3, 4], 2),
]


def oracle_chain(lats, params, occs, model, n_sweeps, seed, step0):
    out_occ, out_pos, out_acc = [], [], []
    w = 0
    for li, (lat, occ) in enumerate(zip(lats, occs)):
        for o in occ:
            o2, p2, na = metropolis(lat, params, o, initial_labels(lat, o), w, seed, step0, n_sweeps,
                                    lat_index=li, act=model.act)
            out_occ.append(o2)
            out_pos.append(p2)
            out_acc.append(na)
            w += 1
    return out_occ, out_pos, out_acc


def split_state(ctx, lats, counts):
    occ, pos = ctx.state()
    torch.cuda.synchronize()
    occ, pos = occ.cpu().numpy(), pos.cpu().numpy()
    per_lat, off, w = [], 0, 0
    for lat, c in zip(lats, counts):
        per_lat.append(occ[off:off + c * lat.N].reshape(c, lat.N).copy())
        off += c * lat.N
    return per_lat, pos


def check_chain(lats, counts, ctx, ref, n_acc):
    occ_ref, pos_ref, acc_ref = ref
    per_lat, pos = split_state(ctx, lats, counts)
    w = 0
    for li, lat in enumerate(lats):
        for k in range(counts[li]):
            assert np.array_equal(per_lat[li][k], occ_ref[w]), (li, k)
            for sp in range(2):
                n = (lat.n_up, lat.n_dn)[sp]
                assert np.array_equal(pos[w, sp, :n].astype(np.int64), pos_ref[w][sp]), (li, k, sp)
            assert int(n_acc[w]) == acc_ref[w], (li, k, int(n_acc[w]), acc_ref[w])
            w += 1
    return per_lat


@pytest.mark.parametrize("name,lats,model,counts,ns", CASES, ids=[c[0] for c in CASES])
def test_sweep_chain_matches_oracle(name, lats, model, counts, ns):
    say(f"[sweep f64] {name}")
    ctx, params, occs = build(lats, model, counts, backflow=0.5)
    n_acc = ctx.sweep(ns, SEED, STEP0)
    torch.cuda.synchronize()
    n_acc = n_acc.cpu().numpy()
    ref = oracle_chain(lats, params, occs, model, ns, SEED, STEP0)
    say(f"  accepted {n_acc.tolist()}")
    assert n_acc.sum() > 0
    new_occs = check_chain(lats, counts, ctx, ref, n_acc)
    # maintained state: Woodbury G/P, accumulated log|psi|
    worst = check_walkers(ctx, lats, params, new_occs, model, 1e-9, 1e-9)
    say(f"  maintained {worst}")
    ctx.refresh()
    flags = ctx.flags().cpu().numpy()
    assert not (flags & 4).any(), flags
    worst = check_walkers(ctx, lats, params, new_occs, model, 1e-10, 1e-10)
    say(f"  refreshed {worst}")


def test_sweep_resumes_across_calls():
    """Two calls (2 sweeps, then 1 more at step0 + 2N) give the chain of one
    3-sweep call; n_accept accumulates."""
    lat = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 6, 5)
    model = wl.Model(2, 8, "tanh", "f64", 2)
    say("[sweep f64 resume]")
    ctx, params, occs = build([lat], model, [6], backflow=0.5)
    n_acc = torch.zeros(6, dtype=torch.int64, device="cuda")
    ctx.sweep(2, SEED, STEP0, n_acc)
    ctx.sweep(1, SEED, STEP0 + 2 * lat.N, n_acc)
    torch.cuda.synchronize()
    ref = oracle_chain([lat], params, occs, model, 3, SEED, STEP0)
    new_occs = check_chain([lat], [6], ctx, ref, n_acc.cpu().numpy())
    check_walkers(ctx, [lat], params, new_occs, model, 1e-9, 1e-9)


def test_sweep_zero_and_bad_walkers():
    """Zero sweeps change nothing; a walker with a wrong electron count is
    left in place and keeps its flag."""
    lat = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)
    model = wl.Model(1, 8, "tanh", "f64", 4)
    occ = wl.random_occupations(lat, 3, seed=5)
    occ[1, np.nonzero(occ[1] == 0)[0][0]] = 1          # one extra up electron
    say("[sweep f64 bad walker]")
    ctx, params, occs = build([lat], model, [3], occ_list=[occ], backflow=0.5)
    n0 = ctx.sweep(0, SEED, STEP0)
    per_lat, _ = split_state(ctx, [lat], [3])
    assert np.array_equal(per_lat[0], occ)
    assert int(n0.sum().item()) == 0
    n_acc = ctx.sweep(2, SEED, STEP0).cpu().numpy()
    per_lat, _ = split_state(ctx, [lat], [3])
    assert np.array_equal(per_lat[0][1], occ[1])
    assert n_acc[1] == 0
    assert ctx.flags().cpu().numpy()[1] & 8


def test_sweep_bf16x3_state_consistent():
    """BF16x3 conv (FP32-accurate on BF16 matrix units) on the 16x16-style
    geometry (periodic x, open y, 4 layers, 32 channels) at a smaller size:
    after sweeps the maintained state agrees with the oracle on the new
    configurations, and with a context loaded fresh from them."""
    lat = wl.Lattice(10, 10, 1, 0, 1.0, 0.0, 8.0, 44, 44)
    model = wl.Model(4, 32, "tanh", "bf16x3", 6)
    say("[sweep bf16x3]")
    ctx, params, occs = build([lat], model, [3], backflow=0.1)
    n_acc = ctx.sweep(2, SEED, STEP0).cpu().numpy()
    say(f"  accepted {n_acc.tolist()}")
    assert n_acc.sum() > 0
    per_lat, _ = split_state(ctx, [lat], [3])
    worst = check_walkers(ctx, [lat], params, per_lat, model, 1e-3, 1e-4, tol_logpsi=1e-6)
    say(f"  maintained vs oracle {worst}")
    e1 = ctx.local_energy("lowrank").cpu().numpy()
    s1, l1 = (t.cpu().numpy() for t in ctx.log_psi())
    ctx2, _, _ = build([lat], model, [3], occ_list=per_lat, backflow=0.1)
    e2 = ctx2.local_energy("lowrank").cpu().numpy()
    s2, l2 = (t.cpu().numpy() for t in ctx2.log_psi())
    dl = np.max(np.abs(l1 - l2) / np.maximum(1.0, np.abs(l2)))
    de = np.max(np.abs(e1 - e2) / np.maximum(1.0, np.abs(e2)))
    say(f"  swept vs fresh: log|psi| {dl:.3e}  E_loc {de:.3e}")
    assert np.array_equal(s1, s2)
    # log|psi| adds one log|ratio| per accepted move since the last refresh;
    # with FP32 features each ratio sees D = H'_L - H_L rounded to FP32
    # (relative 2^-24 per element), about 1e-9 per move here
    assert dl < 1e-8
    ctx.refresh()
    s3, l3 = (t.cpu().numpy() for t in ctx.log_psi())
    assert np.array_equal(s3, s2)
    assert np.max(np.abs(l3 - l2) / np.maximum(1.0, np.abs(l2))) < 1e-12
    assert de < 1e-6
