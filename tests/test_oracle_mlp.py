"""Pins of the oracle's site-wise MLP layers after the conv stack (Sec. II.B,
site-wise MLP equation: H <- act(H W + b) per site, no residual).

* Library routine: the features equal torch conv2d (padding that follows the
  lattice boundary) followed by torch.nn.functional.linear, in FP64.
* Independent gradient route: central differences of log|psi| equal torch
  autograd of the amplitude written with torch primitives, MLP weights
  included.
* Locality (Sec. II.C): the MLP is site-wise, so changing one site's
  occupation changes the final features only within Chebyshev distance L
  (the number of conv layers) of it, however many MLP layers follow.
* Hamiltonian: E_loc(n) psi(n) = (H psi)(n) on a lattice small enough to
  build H by brute force, with the MLP head.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import workloads as wl
from oracle.ansatz import features, log_psi
from oracle.energy import local_energy
from oracle.grad import autograd_grad, fd_grad, pack
from oracle.lattice import neighbour

from test_oracle_bruteforce import hamiltonian, sector, to_occ
from test_oracle_conv_grad import torch_features


def torch_mlp_features(lat, p, occ, act):
    x = torch_features(lat, p, occ, act)             # [N, C] after the conv stack
    for W, b in zip(p.mlp_w, p.mlp_b):
        y = F.linear(x, torch.from_numpy(W).T.contiguous(), torch.from_numpy(b))
        x = torch.tanh(y) if act == "tanh" else F.silu(y)
    return x


@pytest.mark.parametrize("lat", [
    wl.Lattice(4, 4, 1, 1, n_up=5, n_dn=5),
    wl.Lattice(6, 4, 1, 0, n_up=3, n_dn=4),
    wl.Lattice(5, 3, 0, 0, n_up=4, n_dn=1),
])
@pytest.mark.parametrize("act", ["tanh", "silu"])
@pytest.mark.parametrize("n_mlp", [1, 4])
def test_mlp_features_match_torch(lat, act, n_mlp):
    p = wl.random_params([lat], wl.Model(2, 8, n_mlp=n_mlp), seed=9)
    p.conv_w *= 8.0
    for o in wl.random_occupations(lat, 3, seed=4):
        ours = features(lat, p, o, act)
        assert len(ours) == 1 + 2 + n_mlp
        ref = torch_mlp_features(lat, p, o, act).numpy()
        assert np.max(np.abs(ours[-1] - ref)) < 1e-12
        # a wrong layer order or a residual on the MLP would differ
        assert np.max(np.abs(ours[-1] - ours[2])) > 1e-3


def test_fd_gradient_matches_autograd_with_mlp():
    lat = wl.Lattice(4, 3, 1, 0, n_up=3, n_dn=2)
    p = wl.random_params([lat], wl.Model(1, 8, "silu", n_mlp=2), seed=13, backflow=0.8)
    occ = wl.random_occupations(lat, 1, seed=3)[0]
    lp, g_ref = autograd_grad(lat, p, occ, 0, "silu")
    assert lp == pytest.approx(log_psi(lat, p, occ, 0, "silu")[1], abs=1e-12)
    # every MLP parameter plus a sample of the rest
    n_before = p.embed.size + p.conv_w.size + p.conv_b.size
    n_mlp = sum(w.size for w in p.mlp_w) + sum(b.size for b in p.mlp_b)
    idx = np.concatenate([np.arange(n_before, n_before + n_mlp, 3),
                          np.random.default_rng(2).choice(len(pack(p)), 40, replace=False)])
    g = fd_grad(lat, p, occ, 0, "silu", indices=idx)
    assert np.max(np.abs(g - g_ref[idx])) < 1e-8 * max(1.0, np.max(np.abs(g_ref)))
    assert np.max(np.abs(g_ref[n_before:n_before + n_mlp])) > 1e-3


@pytest.mark.parametrize("n_conv", [1, 2])
def test_receptive_field_set_by_conv_layers_only(n_conv):
    lat = wl.Lattice(8, 7, 1, 0, n_up=10, n_dn=10)
    p = wl.random_params([lat], wl.Model(n_conv, 8, n_mlp=4), seed=21)
    rng = np.random.default_rng(5)
    for o in wl.random_occupations(lat, 4, seed=6):
        i = int(rng.integers(lat.N))
        o2 = o.copy()
        o2[i] = (o2[i] + 1) % 4
        d = np.max(np.abs(features(lat, p, o2)[-1] - features(lat, p, o)[-1]), axis=1)
        xi, yi = i % lat.Lx, i // lat.Lx
        for s in range(lat.N):
            dx = abs(s % lat.Lx - xi)
            dx = min(dx, lat.Lx - dx)                 # periodic x
            dy = abs(s // lat.Lx - yi)                # open y
            if max(dx, dy) > n_conv:
                assert d[s] == 0.0, (i, s)
        assert d[i] > 0.0
        # the nearest-neighbour ring at distance n_conv changes too
        assert d[neighbour(lat, i, n_conv, 0)] > 0.0


def test_local_energy_equals_h_psi_with_mlp():
    lat = wl.Lattice(2, 4, 0, 1, 1.0, 0.3, 6.0, 2, 2)
    p = wl.random_params([lat], wl.Model(1, 4, n_mlp=3), seed=5, backflow=0.5)
    states = sector(lat)
    H = hamiltonian(lat, states)
    psi = np.empty(len(states))
    for k, b in enumerate(states):
        s, la = log_psi(lat, p, to_occ(lat, b))
        psi[k] = s * np.exp(la)
    Hpsi = H @ psi
    scale = np.max(np.abs(psi))
    for k in range(len(states)):
        e = local_energy(lat, p, to_occ(lat, states[k]))
        assert e * psi[k] == pytest.approx(Hpsi[k], abs=1e-11 * scale * (1 + abs(e)))
