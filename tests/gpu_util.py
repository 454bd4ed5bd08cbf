"""Helpers shared by the GPU parity tests: build a library context from a
workloads description and compare its outputs with the oracle."""
from __future__ import annotations

import sys

import numpy as np

import workloads as wl
from oracle.ansatz import log_psi
from oracle.energy import local_energy

CODE_DIRS = 8


def hop_code(h, N):
    """The library's code of a connected configuration: (i << 4) | (spin << 3)
    | d for a hop, ((N + i) << 4) | d for a spin exchange from up site i."""
    from oracle.lattice import Exchange
    if isinstance(h, Exchange):
        return ((N + h.i) << 4) | h.d
    return (h.i << 4) | (h.spin << 3) | h.d


def build(lats, model: wl.Model, walkers, seed_params=0, seed_occ=1, backflow=0.1, occ_list=None):
    """(ctx, params (quantised like the library), occupations per lattice)."""
    import torch
    from paper_2604_25775_amd.api import ScaleVMC
    params = wl.random_params(lats, model, seed=seed_params, backflow=backflow)
    params = wl.quantise_params(params, model.conv_prec)
    occs = occ_list or [wl.random_occupations(l, n, seed=seed_occ + 100 * k)
                        for k, (l, n) in enumerate(zip(lats, walkers))]
    ctx = ScaleVMC(lats, model.n_conv, model.channels, model.act, model.conv_prec, model.refresh_every,
                   per_site_embed=model.per_site_embed, n_mlp=model.n_mlp)
    ctx.set_params_from(params)
    flat = np.concatenate([o.reshape(-1) for o in occs]).astype(np.int8)
    ctx.load(list(walkers), flat)
    torch.cuda.synchronize()
    return ctx, params, occs


def rel_err(a, b, floor):
    return abs(a - b) / max(abs(b), floor)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check_walkers(ctx, lats, params, occs, model, tol_ratio, tol_eloc, path="lowrank", sample=None,
                  check_logpsi=True, conv_input_round=None, tol_logpsi=None):
    """Compare log|psi|, sign, every hop ratio (code by code) and E_loc of
    the library with the oracle; returns the max errors."""
    import torch
    eloc, nh, code, rat = ctx.local_energy(path, ratios=True)
    sign, la = ctx.log_psi()
    torch.cuda.synchronize()
    eloc, nh, code, rat = eloc.cpu().numpy(), nh.cpu().numpy(), code.cpu().numpy(), rat.cpu().numpy()
    sign, la = sign.cpu().numpy(), la.cpu().numpy()
    worst = {"ratio": 0.0, "eloc": 0.0, "logpsi": 0.0}
    w0 = 0
    for li, (lat, occ) in enumerate(zip(lats, occs)):
        idx = range(len(occ)) if sample is None else sample[li]
        for k in idx:
            w = w0 + k
            o = occ[k]
            e_ref, hs, R_ref = local_energy(lat, params, o, li, model.act, return_ratios=True,
                                            conv_input_round=conv_input_round)
            if check_logpsi:
                s_ref, l_ref = log_psi(lat, params, o, li, model.act, conv_input_round)
                assert sign[w] == s_ref, (li, k, sign[w], s_ref)
                worst["logpsi"] = max(worst["logpsi"], abs(la[w] - l_ref) / max(1.0, abs(l_ref)))
            assert nh[w] == len(hs), (li, k, nh[w], len(hs))
            codes = [hop_code(h, lat.N) for h in hs]
            assert list(code[w, :len(hs)]) == codes, (li, k)
            floor = 1e-3 * np.sqrt(np.mean(R_ref ** 2)) if len(hs) else 1.0
            for r, rr in zip(rat[w, :len(hs)], R_ref):
                worst["ratio"] = max(worst["ratio"], rel_err(r, rr, floor))
            worst["eloc"] = max(worst["eloc"], rel_err(eloc[w], e_ref, 1.0))
        w0 += len(occ)
    assert worst["logpsi"] <= (tol_ratio if tol_logpsi is None else tol_logpsi), worst
    assert worst["ratio"] <= tol_ratio, worst
    assert worst["eloc"] <= tol_eloc, worst
    return worst
