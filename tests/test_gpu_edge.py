"""Edge cases of the batch layout, FP64 through the C ABI against the oracle.

* A spin without electrons: 6 + 0 on a 4x4 torus and 0 + 3 on a 3x4
  cylinder with t' (the empty spin's determinant is 1, its log|det| 0, and
  it has no hops), in one mixed batch with a 5x3 lattice that has zero
  walkers between them: log|psi|, every hop ratio and E_loc at 1e-10 on the
  low-rank and the full-recompute paths; two sweeps of the sampler with
  chains (occupations, electron positions, accept counts) bit-exact with the
  oracle's; the Jacobian rows against the oracle's autograd gradient at
  1e-10.
* An empty batch is refused by the library with an error, before any
  kernel runs.
* The site limits of the 16-bit connection codes: a 64x64 Hubbard torus
  with t' (4096 sites, hop codes up to (4095 << 4) | 15) and a 64x32 t-J
  cylinder (2048 sites, exchange codes up to ((2048 + 2047) << 4) | 3), 40 +
  40 electrons, FP64: every code, ratio, E_loc and log|psi| of a walker at
  1e-10 against the oracle (its connections spread over host processes),
  and after one sweep the maintained state equal to a fresh load.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, check_walkers, say  # noqa: E402
from oracle.ansatz import log_psi  # noqa: E402
from oracle.grad import autograd_grad  # noqa: E402
from oracle.sampler import initial_labels, metropolis  # noqa: E402

SEED, STEP0 = 20261203, 11
LATS = [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 6, 0),
        wl.Lattice(5, 3, 0, 1, 1.0, 0.3, 6.0, 4, 3),
        wl.Lattice(3, 4, 1, 0, 1.0, -0.2, 6.0, 0, 3)]
COUNTS = [3, 0, 2]
MODEL = wl.Model(2, 8, "tanh", "f64", 3)


def nonzero_walkers(lat, li, params, n, seed):
    """n configurations with psi != 0 (random draws on small lattices can
    make the Slater matrix exactly singular)."""
    out = [o for o in wl.random_occupations(lat, 8 * n + 8, seed=seed)
           if log_psi(lat, params, o, li, MODEL.act)[0] != 0.0][:n]
    assert len(out) == n
    return np.array(out, dtype=np.int8).reshape(n, lat.N)


def test_empty_spin_and_zero_walker_lattice():
    params = wl.random_params(LATS, MODEL, seed=0, backflow=0.5)
    occs = [nonzero_walkers(lat, li, params, c, 40 + li) for li, (lat, c) in enumerate(zip(LATS, COUNTS))]
    say("[edge] 4x4 6+0, 5x3 with no walkers, 3x4 0+3: E_loc, chains, gradient")
    ctx, params2, _ = build(LATS, MODEL, COUNTS, occ_list=occs, backflow=0.5)
    assert np.array_equal(params.conv_w, params2.conv_w) and np.array_equal(params.embed, params2.embed)
    assert not ctx.flags().cpu().numpy().any()
    for path in ("lowrank", "full"):
        worst = check_walkers(ctx, LATS, params, occs, MODEL, 1e-10, 1e-10, path=path)
        say(f"  {path}: {worst}")
    # gradient rows
    J = ctx.grad_logpsi().cpu().numpy()
    w = 0
    for li, (lat, occ) in enumerate(zip(LATS, occs)):
        for o in occ:
            g = autograd_grad(lat, params, o, li, MODEL.act)[1]
            err = float(np.max(np.abs(J[w] - g))) / max(1.0, float(np.max(np.abs(g))))
            assert err <= 1e-10, (li, w, err)
            w += 1
    say(f"  gradient rows of {w} walkers at 1e-10")
    # two sweeps against the oracle's chains
    n_acc = ctx.sweep(2, SEED, STEP0).cpu().numpy()
    occ_g, pos_g = ctx.state()
    occ_g, pos_g = occ_g.cpu().numpy(), pos_g.cpu().numpy()
    w, off = 0, 0
    new = []
    for li, (lat, occ) in enumerate(zip(LATS, occs)):
        o_lat = occ_g[off:off + len(occ) * lat.N].reshape(len(occ), lat.N)
        off += len(occ) * lat.N
        new.append(o_lat)
        for k, o in enumerate(occ):
            o2, p2, na = metropolis(lat, params, o, initial_labels(lat, o), w, SEED, STEP0, 2,
                                    lat_index=li, act=MODEL.act)
            assert np.array_equal(o_lat[k], o2), (li, k)
            assert np.array_equal(pos_g[w, 0, :lat.n_up].astype(np.int64), p2[0]), (li, k)
            assert np.array_equal(pos_g[w, 1, :lat.n_dn].astype(np.int64), p2[1]), (li, k)
            assert int(n_acc[w]) == na, (li, k, int(n_acc[w]), na)
            w += 1
    say(f"  chains bit-exact, accepted {n_acc.tolist()}")
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
    worst = check_walkers(ctx, LATS, params, new, MODEL, 1e-10, 1e-10)
    say(f"  after the sweeps: {worst}")


def test_empty_batch_refused():
    from paper_2604_25775_amd._lib import SvmcError
    from paper_2604_25775_amd.api import ScaleVMC
    lat = LATS[0]
    ctx = ScaleVMC([lat], MODEL.n_conv, MODEL.channels, MODEL.act, MODEL.conv_prec, MODEL.refresh_every)
    ctx.set_params_from(wl.random_params([lat], MODEL, seed=0))
    # (an empty occupation tensor has no data pointer: refused as a null
    # argument, else as "no walkers"; either way an invalid argument)
    with pytest.raises(SvmcError, match="invalid argument"):
        ctx.load([0], np.zeros(0, dtype=np.int8))


@pytest.mark.parametrize("lat", [
    wl.Lattice(64, 64, 1, 1, 1.0, -0.2, 4.0, 40, 40),
    wl.Lattice(64, 32, 0, 1, 1.0, 0.2, 0.0, 40, 40, tj=1, J=1.0 / 3.0, h_pin=0.5),
], ids=["hubbard_64x64", "tj_64x32"])
def test_connection_code_site_limits(lat):
    from gpu_util import hop_code
    from oracle_par import local_energies
    model = wl.Model(1, 8, "tanh", "f64", 32)
    say(f"[edge] {lat.Lx}x{lat.Ly} {'t-J' if lat.tj else 'Hubbard'} {lat.n_up}+{lat.n_dn}: codes at the 16-bit limit")
    # a walker with electrons on the last sites, so the largest codes occur
    occ = wl.random_occupations(lat, 2, seed=8)
    for o in occ:
        for sp, bit in ((0, 1), (1, 2)):
            if not (o[lat.N - 1 - sp] & bit):
                k = np.nonzero((o & bit) != 0)[0][0]
                if lat.tj and o[lat.N - 1 - sp] != 0:
                    continue
                o[k] &= ~bit
                o[lat.N - 1 - sp] |= bit
    ctx, params, _ = build([lat], model, [2], occ_list=[occ], backflow=0.3)
    assert not ctx.flags().cpu().numpy().any()
    eloc, nh, code, rat = (t.cpu().numpy() for t in ctx.local_energy(ratios=True))
    sign, la = (t.cpu().numpy() for t in ctx.log_psi())
    e_ref, cs, R_ref, (s_ref, l_ref) = local_energies(lat, params, [occ[0]], 0, model.act)[0]
    assert sign[0] == s_ref
    assert abs(la[0] - l_ref) <= 1e-10 * max(1.0, abs(l_ref))
    codes = [hop_code(c, lat.N) for c in cs]
    assert nh[0] == len(cs) and list(code[0, :len(cs)]) == codes
    assert max(codes) >= (((2 * lat.N if lat.tj else lat.N) - 64) << 4)
    floor = 1e-3 * np.sqrt(np.mean(R_ref ** 2))
    err = max(abs(r - rr) / max(abs(rr), floor) for r, rr in zip(rat[0, :len(cs)], R_ref))
    assert err <= 1e-10, err
    assert abs(eloc[0] - e_ref) <= 1e-10 * max(1.0, abs(e_ref))
    say(f"  {len(cs)} connections (largest code {max(codes)}), max ratio err {err:.1e}")
    n_acc = ctx.sweep(1, SEED, 0).cpu().numpy()
    assert n_acc.sum() > 0
    assert not (ctx.flags().cpu().numpy() & (1 | 2 | 8)).any()
    o, _ = ctx.state()
    o = o.cpu().numpy().reshape(2, lat.N)
    e1 = ctx.local_energy().cpu().numpy()
    l1 = ctx.log_psi()[1].cpu().numpy()
    ctx2, _, _ = build([lat], model, [2], occ_list=[o], backflow=0.3)
    e2 = ctx2.local_energy().cpu().numpy()
    l2 = ctx2.log_psi()[1].cpu().numpy()
    assert np.max(np.abs(l1 - l2) / np.maximum(1.0, np.abs(l2))) <= 1e-10
    assert np.max(np.abs(e1 - e2) / np.maximum(1.0, np.abs(e2))) <= 1e-9
    say(f"  sweep: accepted {n_acc.tolist()}, maintained state equals a fresh load")
