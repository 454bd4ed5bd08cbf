"""Symmetry-projected amplitudes (App. B) on the GPU, against the oracle.

* FP64: E_sym, sign and log|psi_sym| of every walker against the oracle's
  plain definition (psi_sym of every connected configuration recomputed over
  the whole group) at 1e-10, on a Hubbard torus (mirrors and a spin flip
  with character -1) and a t-J cylinder (translations around the width,
  both mirrors, an odd character).
* The group checks of svmc_set_symmetry and the batch layout checks.
* A batch whose copies are not images of copy 0 gives NaN and the SYMMETRY
  flag for that walker only.
* f16x2 at the 16x16 bench lattice with D2 x spin inversion (8 elements):
  sampled walkers against the oracle's copies (local energies, log|psi|)
  combined with its fermion signs, at 1e-4.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, say  # noqa: E402
from oracle.symmetry import fermion_sign, local_energy_sym, log_psi_sym  # noqa: E402
from oracle_par import local_energies  # noqa: E402

CASES = [
    ("4x4_torus_mirrors_flip_odd", wl.Lattice(4, 4, 1, 1, 1.0, -0.2, 4.0, 5, 5),
     [("mx", 1.0), ("my", 1.0), ("flip", -1.0)], wl.Model(1, 8, "silu", "f64", 4, n_mlp=2)),
    ("8x4_tj_cylinder_ty_mirrors", wl.Lattice(8, 4, 0, 1, 1.0, 0.2, 0.0, 14, 14, tj=1, J=1.0 / 3.0),
     [("ty", 1.0), ("my", -1.0), ("mx", 1.0)], wl.Model(2, 8, "tanh", "f64", 4)),
]


def sym_ctx(lat, model, G, chi, occ, **kw):
    """Context holding the copies of the base walkers occ [W, N]."""
    ctx, params, _ = build([lat], model, [len(occ) * len(G)], occ_list=[np.repeat(occ, len(G), axis=0)], **kw)
    ctx.set_symmetry(G, chi)
    cp = ctx.sym_expand(torch.from_numpy(occ).cuda())
    ctx.load([len(occ) * len(G)], cp.cpu().numpy())
    torch.cuda.synchronize()
    return ctx, params, cp.cpu().numpy()


@pytest.mark.parametrize("name,lat,gens,model", CASES, ids=[c[0] for c in CASES])
def test_sym_fp64_matches_plain_definition(name, lat, gens, model):
    G, chi = wl.symmetry_group(lat, gens)
    occ = wl.random_occupations(lat, 3, seed=11)
    say(f"[sym f64] {name}: |G| = {len(G)}")
    ctx, params, cp = sym_ctx(lat, model, G, chi, occ, backflow=0.5)
    # the expansion is the group action
    from oracle.symmetry import apply_symmetry
    for k in range(len(occ)):
        for g, (perm, flip) in enumerate(G):
            assert np.array_equal(cp[k * len(G) + g], apply_symmetry(occ[k], perm, flip))
    e, sg, la = (x.cpu().numpy() for x in ctx.local_energy_sym())
    worst = 0.0
    for k in range(len(occ)):
        s_ref, l_ref = log_psi_sym(lat, params, occ[k], G, chi, 0, model.act)
        e_ref = local_energy_sym(lat, params, occ[k], G, chi, 0, model.act)
        assert sg[k] == s_ref, k
        assert abs(la[k] - l_ref) <= 1e-10 * max(1.0, abs(l_ref)), (k, la[k], l_ref)
        worst = max(worst, abs(e[k] - e_ref) / max(1.0, abs(e_ref)))
    say(f"  worst E_sym {worst:.2e}")
    assert worst <= 1e-10
    assert not (ctx.flags().cpu().numpy() & 16).any()


def test_sym_refusals_and_layout():
    lat, gens, model = CASES[0][1], CASES[0][2], wl.Model(1, 8, "tanh", "f64", 4)
    G, chi = wl.symmetry_group(lat, gens)
    occ = wl.random_occupations(lat, 2, seed=3)
    ctx, _, _ = sym_ctx(lat, model, G, chi, occ)
    N = lat.N
    ident = tuple(range(N))
    bad_perm = tuple(np.random.default_rng(0).permutation(N).tolist())
    for group, why in [([(bad_perm, False)] + G[1:], "identity not first"),
                       (G + [(bad_perm, False)], "not a symmetry"),
                       ([(ident, False), ((1,) * N, False)], "not a permutation")]:
        with pytest.raises(RuntimeError):
            ctx.set_symmetry(group, [1.0] * len(group))
        say(f"  refused: {why}")
    # spin flip needs equal counts; the pinning field must be kept
    lat2 = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 4)
    ctx2, _, _ = build([lat2], model, [2])
    with pytest.raises(RuntimeError):
        ctx2.set_symmetry(*wl.symmetry_group(lat2, [("flip", 1.0)]))
    lat3 = wl.Lattice(8, 4, 0, 1, 1.0, 0.0, 0.0, 14, 14, tj=1, J=0.3, h_pin=0.5)
    ctx3, _, _ = build([lat3], model, [2])
    with pytest.raises(RuntimeError):
        ctx3.set_symmetry(*wl.symmetry_group(lat3, [("mx", 1.0)]))
    ctx3.set_symmetry(*wl.symmetry_group(lat3, [(("ty", 2), 1.0)]))      # keeps the staggered field
    # walker count not a multiple of the group order
    ctx.load([len(occ) * len(G) - 1], np.repeat(occ, len(G), axis=0)[:-1])
    with pytest.raises(RuntimeError):
        ctx.local_energy_sym()


def test_sym_inconsistent_copies_flagged():
    lat, gens, model = CASES[0][1], CASES[0][2], wl.Model(1, 8, "tanh", "f64", 4)
    G, chi = wl.symmetry_group(lat, gens)
    occ = wl.random_occupations(lat, 3, seed=4)
    ctx, _, cp = sym_ctx(lat, model, G, chi, occ)
    cp = cp.copy()
    c = cp[1 * len(G) + 2]
    a = int(np.nonzero(c == 1)[0][0])
    b = int(np.nonzero(c == 0)[0][0])
    c[a], c[b] = 0, 1                                  # walker 1, copy 2: one electron moved
    ctx.load([len(cp)], cp)
    e, _, _ = (x.cpu().numpy() for x in ctx.local_energy_sym())
    f = ctx.flags().cpu().numpy()
    assert np.isnan(e[1]) and np.isfinite(e[[0, 2]]).all()
    assert f[len(G)] & 16 and not (f[0] & 16) and not (f[2 * len(G)] & 16)


def test_sym_f16x2_16x16_d2_spin_inversion():
    w = wl.get("c3")
    lat = w.lattices[0]
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    G, chi = wl.symmetry_group(lat, [("mx", 1.0), ("my", 1.0), ("flip", 1.0)])
    assert len(G) == 8
    occ = wl.occupations(w, 0, n_walkers=32)
    say(f"[sym f16x2] 16x16, |G| = 8, 32 walkers")
    ctx, params, cp = sym_ctx(lat, model, G, chi, occ)
    e, sg, la = (x.cpu().numpy() for x in ctx.local_energy_sym())
    assert np.isfinite(e).all()
    for k in (0, 17):
        ref = local_energies(lat, params, [cp[k * 8 + g] for g in range(8)], 0, model.act)
        lmax = max(r[3][1] for r in ref)
        a = np.array([fermion_sign(occ[k], perm, flip) * c * r[3][0] * np.exp(r[3][1] - lmax)
                      for (perm, flip), c, r in zip(G, chi, ref)])
        e_ref = float(np.sum(a * np.array([r[0] for r in ref])) / np.sum(a))
        l_ref = lmax + np.log(abs(np.sum(a)))
        say(f"  walker {k}: E_sym {e[k]:.8f} oracle {e_ref:.8f}")
        assert sg[k] == np.sign(np.sum(a))
        assert abs(la[k] - l_ref) <= 1e-6 * abs(l_ref)
        assert abs(e[k] - e_ref) <= 1e-4 * max(1.0, abs(e_ref))


@pytest.mark.parametrize("name,lat,gens,model", CASES, ids=[c[0] for c in CASES])
def test_sym_sampler_chain_matches_oracle(name, lat, gens, model):
    """svmc_sweep_sym against the oracle's |psi_sym|^2 chain (plain psi_sym
    ratios): copy 0's occupations, labels and accept counts bit-exact; every
    copy accepted the same moves and stays the image of copy 0; E_sym after
    the sweeps against the plain definition."""
    from oracle.sampler import initial_labels
    from oracle.symmetry import metropolis_sym
    from test_gpu_sweep import SEED, STEP0
    G, chi = wl.symmetry_group(lat, gens)
    occ = wl.random_occupations(lat, 3, seed=12)
    say(f"[sym sweep f64] {name}: |G| = {len(G)}")
    ctx, params, _ = sym_ctx(lat, model, G, chi, occ, backflow=0.5)
    n_acc = ctx.sweep_sym(2, SEED, STEP0).cpu().numpy()
    o, pos = ctx.state()
    o = o.cpu().numpy().reshape(-1, lat.N)
    pos = pos.cpu().numpy()
    total = 0
    new = []
    for k in range(len(occ)):
        o_ref, p_ref, a_ref = metropolis_sym(lat, params, occ[k], initial_labels(lat, occ[k]), k, SEED, STEP0, 2,
                                             G, chi, act=model.act)
        w0 = k * len(G)
        assert np.array_equal(o[w0], o_ref), k
        for sp, n in ((0, lat.n_up), (1, lat.n_dn)):
            assert np.array_equal(pos[w0, sp, :n].astype(np.int64), p_ref[sp]), (k, sp)
        assert (n_acc[w0:w0 + len(G)] == a_ref).all(), (k, n_acc[w0:w0 + len(G)], a_ref)
        total += a_ref
        new.append(o_ref)
    assert total > 0
    say(f"  {total} accepted moves")
    e, sg, la = (x.cpu().numpy() for x in ctx.local_energy_sym())
    assert not (ctx.flags().cpu().numpy() & 16).any()
    for k in range(len(occ)):
        e_ref = local_energy_sym(lat, params, new[k], G, chi, 0, model.act)
        assert abs(e[k] - e_ref) <= 1e-9 * max(1.0, abs(e_ref)), (k, e[k], e_ref)


def test_sym_gradient_weights_match_finite_differences():
    """d log|psi_sym| / d theta from svmc_grad_logpsi with the copies'
    weights (vjp = w_g) against central differences of the oracle's plain
    log|psi_sym| on a sample of parameters of every kind."""
    from oracle.grad import pack, unpack
    name, lat, gens, model = CASES[0]
    G, chi = wl.symmetry_group(lat, gens)
    occ = wl.random_occupations(lat, 2, seed=21)
    ctx, params, _ = sym_ctx(lat, model, G, chi, occ, backflow=0.5)
    _, _, _, wts = ctx.local_energy_sym(weights=True)
    theta = pack(params)
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([rng.choice(theta.size, 60, replace=False), [0, theta.size - 1]]))
    for k in range(len(occ)):
        v = torch.zeros(ctx.num_walkers, dtype=torch.float64, device="cuda")
        v[k * len(G):(k + 1) * len(G)] = wts[k * len(G):(k + 1) * len(G)]
        g = ctx.grad_logpsi(v).cpu().numpy()
        h = 1e-5
        fd = np.empty(len(idx))
        for n, j in enumerate(idx):
            tp, tm = theta.copy(), theta.copy()
            tp[j] += h
            tm[j] -= h
            fd[n] = (log_psi_sym(lat, unpack(tp, params), occ[k], G, chi, 0, model.act)[1]
                     - log_psi_sym(lat, unpack(tm, params), occ[k], G, chi, 0, model.act)[1]) / (2 * h)
        scale = max(1.0, float(np.max(np.abs(fd))))
        err = float(np.max(np.abs(g[idx] - fd))) / scale
        say(f"  walker {k}: gradient vs finite differences {err:.2e}")
        assert err <= 1e-7
