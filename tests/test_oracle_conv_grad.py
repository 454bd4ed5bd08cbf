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
from oracle.grad import fd_grad, pack


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


def torch_log_psi(lat, theta, p, occ, act="tanh"):
    C, L = p.embed.shape[1], p.conv_w.shape[0]
    off = 0

    def take(shape):
        nonlocal off
        n = int(np.prod(shape))
        a = theta[off:off + n].reshape(shape)
        off += n
        return a
    E = take((4, C))
    W = take((L, 3, 3, C, C))
    b = take((L, C))
    pw = [take((C, lat.n_up)), take((C, lat.n_dn))]
    pb = [take((lat.n_up,)), take((lat.n_dn,))]
    x = E[torch.from_numpy(np.asarray(occ, dtype=np.int64))].T.reshape(1, C, lat.Ly, lat.Lx)
    for l in range(L):
        xp = F.pad(x, (1, 1, 0, 0), mode="circular") if lat.pbc_x else F.pad(x, (1, 1, 0, 0))
        xp = F.pad(xp, (0, 0, 1, 1), mode="circular") if lat.pbc_y else F.pad(xp, (0, 0, 1, 1))
        y = F.conv2d(xp, W[l].permute(3, 2, 0, 1), b[l])
        x = x + (torch.tanh(y) if act == "tanh" else F.silu(y))
    HL = x.reshape(C, lat.N).T
    tot = 0.0
    for s in (0, 1):
        rows = torch.from_numpy(p.base[0][s]) + HL @ pw[s] + pb[s][None, :]
        idx = torch.from_numpy(occupied_sites(occ, s))
        tot = tot + torch.linalg.slogdet(rows[idx])[1]
    return tot


@pytest.mark.parametrize("lat", [
    wl.Lattice(4, 4, 1, 1, n_up=5, n_dn=5),
    wl.Lattice(4, 3, 1, 0, n_up=3, n_dn=2),
])
def test_fd_gradient_matches_autograd(lat):
    p = wl.random_params([lat], wl.Model(2, 4), seed=12, backflow=0.8)
    occ = wl.random_occupations(lat, 1, seed=3)[0]
    theta = torch.from_numpy(pack(p)).requires_grad_(True)
    lp = torch_log_psi(lat, theta, p, occ)
    assert lp.item() == pytest.approx(log_psi(lat, p, occ)[1], abs=1e-12)
    lp.backward()
    g_ref = theta.grad.numpy()
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(theta.numel(), 60, replace=False))
    g_fd = fd_grad(lat, p, occ, indices=idx)
    assert np.max(np.abs(g_fd - g_ref[idx])) < 2e-7 * (1 + np.max(np.abs(g_ref)))


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
