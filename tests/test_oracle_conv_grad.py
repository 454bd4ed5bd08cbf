"""Library pins of the oracle's network forward and its gradient.

* The residual conv stack (Sec. II.B, conv equation, padding that follows the
  lattice boundary) must equal torch.nn.functional.conv2d in FP64 with
  circular padding on periodic axes and zero padding on open axes.
* The finite-difference gradient of log|psi| must equal the gradient that
  torch autograd gives for the same amplitude written with torch primitives
  (conv2d, slogdet) - an independent library route.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import workloads as wl
from oracle.ansatz import features, log_psi, occupied_sites
from oracle.grad import autograd_grad, fd_grad


def torch_features(lat, p, occ, act="tanh"):
    H = torch.from_numpy(p.embed)[torch.from_numpy(np.asarray(occ, dtype=np.int64))]
    x = H.T.reshape(1, -1, lat.Ly, lat.Lx)        # [1, C, Ly, Lx]
    W = torch.from_numpy(p.conv_w)                  # [L, ky, kx, cin, cout]
    b = torch.from_numpy(p.conv_b)
    for l in range(W.shape[0]):
        xp = x
        xp = F.pad(xp, (1, 1, 0, 0), mode="circular") if lat.pbc_x else F.pad(xp, (1, 1, 0, 0))
        xp = F.pad(xp, (0, 0, 1, 1), mode="circular") if lat.pbc_y else F.pad(xp, (0, 0, 1, 1))
        w = W[l].permute(3, 2, 0, 1)                # [cout, cin, ky, kx]
        y = F.conv2d(xp, w, b[l])
        x = x + (torch.tanh(y) if act == "tanh" else F.silu(y))
    return x.reshape(-1, lat.N).T


@pytest.mark.parametrize("lat", [
    wl.Lattice(4, 4, 1, 1, n_up=5, n_dn=5),
    wl.Lattice(6, 4, 1, 0, n_up=3, n_dn=4),
    wl.Lattice(3, 5, 0, 1, n_up=2, n_dn=2),
    wl.Lattice(5, 3, 0, 0, n_up=4, n_dn=1),
])
@pytest.mark.parametrize("act", ["tanh", "silu"])
def test_conv_stack_matches_torch(lat, act):
    p = wl.random_params([lat], wl.Model(3, 6), seed=9)
    p.conv_w *= 8.0                                 # make the layers matter
    for o in wl.random_occupations(lat, 3, seed=4):
        ours = features(lat, p, o, act)[-1]
        ref = torch_features(lat, p, o, act).numpy()
        assert np.max(np.abs(ours - ref)) < 1e-12


@pytest.mark.parametrize("lat", [
    wl.Lattice(4, 4, 1, 1, n_up=5, n_dn=5),
    wl.Lattice(4, 3, 1, 0, n_up=3, n_dn=2),
])
def test_fd_gradient_matches_autograd(lat):
    p = wl.random_params([lat], wl.Model(2, 4), seed=12, backflow=0.8)
    occ = wl.random_occupations(lat, 1, seed=3)[0]
    lp, g_ref = autograd_grad(lat, p, occ)
    assert lp == pytest.approx(log_psi(lat, p, occ)[1], abs=1e-12)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(g_ref.size, 60, replace=False))
    g_fd = fd_grad(lat, p, occ, indices=idx)
    assert np.max(np.abs(g_fd - g_ref[idx])) < 2e-7 * (1 + np.max(np.abs(g_ref)))


@pytest.mark.parametrize("act", ["tanh", "silu"])
def test_autograd_gradient_mixed_lattices(act):
    """Second lattice of a mixed set: its own projection block carries the
    gradient (FD-checked on every projection entry and on sampled conv
    entries), the first lattice's block is exactly zero."""
    lats = [wl.Lattice(4, 4, 1, 1, n_up=3, n_dn=2), wl.Lattice(3, 5, 0, 1, n_up=2, n_dn=3)]
    p = wl.random_params(lats, wl.Model(2, 4), seed=5, backflow=0.8)
    occ = wl.random_occupations(lats[1], 1, seed=8)[0]
    lp, g = autograd_grad(lats[1], p, occ, lat_index=1, act=act)
    assert lp == pytest.approx(log_psi(lats[1], p, occ, 1, act)[1], abs=1e-12)
    C, L = 4, 2
    o1 = 4 * C + 9 * L * C * C + L * C
    o2 = o1 + C * (3 + 2) + 3 + 2
    assert not g[o1:o2].any()
    rng = np.random.default_rng(2)
    idx = np.concatenate([np.arange(o2, g.size), np.sort(rng.choice(o1, 30, replace=False))])
    g_fd = fd_grad(lats[1], p, occ, lat_index=1, act=act, indices=idx)
    assert np.max(np.abs(g_fd - g[idx])) < 2e-7 * (1 + np.max(np.abs(g)))


def test_conv_input_rounding_matches_torch_bf16_inputs():
    """With conv_input_round = BF16 rounding, each layer equals conv2d applied
    to the BF16-rounded layer input plus the unrounded residual."""
    from oracle.ansatz import round_bf16
    lat = wl.Lattice(6, 4, 1, 0, n_up=3, n_dn=4)
    p = wl.random_params([lat], wl.Model(2, 8), seed=9)
    o = wl.random_occupations(lat, 1, seed=4)[0]
    Hs = features(lat, p, o, "tanh", conv_input_round=round_bf16)
    W = torch.from_numpy(p.conv_w)
    b = torch.from_numpy(p.conv_b)
    for l in range(2):
        x = torch.from_numpy(round_bf16(Hs[l])).T.reshape(1, -1, lat.Ly, lat.Lx)
        xp = F.pad(F.pad(x, (1, 1, 0, 0), mode="circular"), (0, 0, 1, 1))
        y = F.conv2d(xp, W[l].permute(3, 2, 0, 1), b[l]).reshape(-1, lat.N).T.numpy()
        assert np.max(np.abs(Hs[l + 1] - (Hs[l] + np.tanh(y)))) < 1e-12
    # the rounding does change the result (the hook is live)
    assert np.max(np.abs(Hs[-1] - features(lat, p, o, "tanh")[-1])) > 1e-6


# ---------------------------------------------------------------------------
# per-site embedding tables (Sec. II.B writes the embedding layer with one
# table E_i per site i)
# ---------------------------------------------------------------------------
def torch_features_site(lat, p, occ, li, act="tanh"):
    """The same conv stack as torch_features with H_0[s] gathered from the
    site's own table by torch indexing."""
    E = torch.from_numpy(p.embed_site[li])                       # [N, 4, C]
    o = torch.from_numpy(np.asarray(occ, dtype=np.int64))
    H = E[torch.arange(lat.N), o]
    q = p.copy()
    q.embed_site = None
    x = H.T.reshape(1, -1, lat.Ly, lat.Lx)
    W = torch.from_numpy(q.conv_w)
    b = torch.from_numpy(q.conv_b)
    for l in range(W.shape[0]):
        xp = F.pad(x, (1, 1, 0, 0), mode="circular") if lat.pbc_x else F.pad(x, (1, 1, 0, 0))
        xp = F.pad(xp, (0, 0, 1, 1), mode="circular") if lat.pbc_y else F.pad(xp, (0, 0, 1, 1))
        y = F.conv2d(xp, W[l].permute(3, 2, 0, 1), b[l])
        x = x + (torch.tanh(y) if act == "tanh" else F.silu(y))
    return x.reshape(-1, lat.N).T


def test_per_site_tables_equal_to_shared_reduce_to_shared():
    """Per-site tables that all equal the shared table give the shared
    network's features bit for bit."""
    lat = wl.Lattice(4, 3, 1, 0, n_up=3, n_dn=2)
    p = wl.random_params([lat], wl.Model(2, 6), seed=3)
    q = p.copy()
    q.embed_site = [np.tile(p.embed[None], (lat.N, 1, 1))]
    for o in wl.random_occupations(lat, 3, seed=2):
        for a, b in zip(features(lat, p, o), features(lat, q, o)):
            assert np.array_equal(a, b)
        assert log_psi(lat, p, o) == log_psi(lat, q, o)


@pytest.mark.parametrize("li", [0, 1])
def test_per_site_embedding_matches_torch(li):
    lats = [wl.Lattice(4, 4, 1, 1, n_up=5, n_dn=5), wl.Lattice(3, 5, 0, 1, n_up=2, n_dn=3)]
    p = wl.random_params(lats, wl.Model(3, 6, per_site_embed=True), seed=9)
    assert p.embed_site is not None and [e.shape for e in p.embed_site] == [(16, 4, 6), (15, 4, 6)]
    p.conv_w *= 8.0
    for o in wl.random_occupations(lats[li], 3, seed=4):
        ours = features(lats[li], p, o, "silu", lat_index=li)
        # H_0 is the site's own row: a site-dependent embedding
        assert np.array_equal(ours[0], p.embed_site[li][np.arange(lats[li].N), o])
        ref = torch_features_site(lats[li], p, o, li, "silu").numpy()
        assert np.max(np.abs(ours[-1] - ref)) < 1e-12


def test_per_site_embedding_gradient_fd_and_autograd():
    """Mixed lattices with per-site tables: d log|psi| of a walker of lattice 1
    by autograd equals central differences on every entry of its own table
    block (each site's row of its occupation carries the gradient, the other
    three rows and lattice 0's block are exactly zero)."""
    lats = [wl.Lattice(4, 4, 1, 1, n_up=3, n_dn=2), wl.Lattice(3, 4, 0, 1, n_up=2, n_dn=3)]
    p = wl.random_params(lats, wl.Model(2, 4, per_site_embed=True), seed=6, backflow=0.8)
    occ = wl.random_occupations(lats[1], 1, seed=8)[0]
    lp, g = autograd_grad(lats[1], p, occ, lat_index=1)
    assert lp == pytest.approx(log_psi(lats[1], p, occ, 1)[1], abs=1e-12)
    C = 4
    o0, o1 = 16 * 4 * C, 16 * 4 * C + 12 * 4 * C
    assert not g[:o0].any()
    blk = g[o0:o1].reshape(12, 4, C)
    for s in range(12):
        for o in range(4):
            if o != occ[s]:
                assert not blk[s, o].any()
    idx = np.arange(o0, o1)
    g_fd = fd_grad(lats[1], p, occ, lat_index=1, indices=idx)
    assert np.max(np.abs(g_fd - g[idx])) < 2e-7 * (1 + np.max(np.abs(g)))
    assert np.abs(g[idx]).max() > 1e-3
