#!/usr/bin/env python
"""Benchmark of the SCALE local-energy hot path on one MI355X.

Workload (default): Hubbard 16x16, periodic-x / open-y, t = 1, U = 8,
112 + 112 electrons (1/8 hole doping), 4 residual 3x3 conv layers x 32
channels, 8192 walkers, seeded synthetic parameters and occupations.

Before timing, --therm Metropolis sweeps (default 8) move the walkers from
the random start and leave the caches (features, G, P) as sampling does.
One timed step = one local-energy evaluation of the whole batch: per-walker
precompute (orbital rows, G = M Phi^-1, P = W Phi^-1) + the low-rank
local-energy kernel (hop enumeration, incremental conv on the matrix units,
FP64 determinant-lemma ratios, reduction).  Inputs are resident in HBM
before the timed region.  Also measured: the time per sweep, one gradient
VJP of log|psi| over the batch, the full-recompute path on the same walkers
(speed-up), the oracle on host cores (cpu_baseline), and the roofline
position of the dominant kernel from HIP events on its stream.

The conv runs in f16x2 by default: the workload's BF16 weights (exact in
FP16) on the FP16 matrix units, features carried as FP16 pairs (22
significant bits), FP32 accumulation; --prec bf16x3 gives exact FP32
activations at one more pass.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--prec f16x2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import replace

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16 = 2.5e15      # dense MFMA, FLOP/s
PEAK_FP64 = 78.6e12
PEAK_FP32 = 157.3e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# HBM traffic of the E_loc launch from counter runs (profiles/)
# ---------------------------------------------------------------------------
COPY_PROBE_BYTES = 1 << 30      # the known-size copy of the traffic probe


def kernel_src_sha1() -> str:
    """SHA-1 over the HIP/C++ sources of the library (names and contents in
    name order): a counter record holds for the sources it was taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2604_25775_amd", "csrc")
    h = hashlib.sha1()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def traffic_record(workload: str, walkers: int, prec: str, slices: int, row_form_max: int = 16):
    """HBM bytes per E_loc launch from a committed counter summary
    (a `traffic-record:` line under profiles/): FETCH_SIZE and WRITE_SIZE of
    the launch, each scaled by bytes / counter of a plain copy of known size
    in the same run.  None when no record matches this workload and launch
    shape (slices per walker, row-form limit), or the sources have changed
    since the counters were taken."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    sha = kernel_src_sha1()
    for f in sorted(os.listdir(d)):
        if not f.endswith((".md", ".txt")):
            continue
        with open(os.path.join(d, f)) as fh:
            for ln in fh:
                if not ln.startswith("traffic-record:"):
                    continue
                r = json.loads(ln.split(":", 1)[1])
                if (r.get("src_sha1") == sha and r.get("workload") == workload
                        and r.get("walkers") == walkers and r.get("prec") == prec
                        and r.get("slices") == slices and r.get("row_form_max", 16) == row_form_max):
                    fetch = r["fetch_kib"] * COPY_PROBE_BYTES / r["copy_fetch_kib"]
                    write = r["write_kib"] * COPY_PROBE_BYTES / r["copy_write_kib"]
                    return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write, "file": f,
                            "slices": r.get("slices")}
    return None


# ---------------------------------------------------------------------------
# algorithmic work of the low-rank kernel (accounting only, numpy)
# ---------------------------------------------------------------------------
def lowrank_flops(lat, occ: np.ndarray, L: int, C: int, n_mlp: int = 0):
    """(conv FLOPs, FP64 determinant FLOPs) of one low-rank local-energy
    launch: per hop, layer l recomputes the sites within Chebyshev distance l
    of the two changed sites (9 C^2 multiply-adds each), and each of the
    n_mlp site-wise layers the sites of layer L (C^2 each; counted with the
    conv work, same precision); per spin, k electrons
    of the new configuration lie within distance L, the determinant-lemma
    matrix has rank r = min(k, C + [moving spin]), its assembly costs k C r
    and its LU r^3 / 3 multiply-adds.  t-J lattices: hops only onto empty
    sites, and the spin exchanges, with both spins moving."""
    W, N = occ.shape
    Lx, Ly = lat.Lx, lat.Ly
    nd = 8 if lat.tp != 0.0 else 4
    DX = [1, -1, 0, 0, 1, 1, -1, -1]
    DY = [0, 0, 1, -1, 1, -1, 1, -1]
    grid = occ.reshape(W, Ly, Lx)
    ups = (grid & 1).astype(np.int64)
    dns = ((grid >> 1) & 1).astype(np.int64)

    def sat(a):
        # summed-area table of a tiled 3x3 copy (handles wrap on periodic axes)
        t = np.tile(a, (1, 3, 3))
        s = np.zeros((W, 3 * Ly + 1, 3 * Lx + 1), np.int64)
        s[:, 1:, 1:] = t.cumsum(1).cumsum(2)
        return s

    sat_u, sat_d = sat(ups), sat(dns)
    xs, ys = np.meshgrid(np.arange(Lx), np.arange(Ly))
    xs, ys = xs.ravel(), ys.ravel()
    conv = 0.0
    det = 0.0

    def axis_range(c0, c1, l, La, per):
        lo, hi = np.minimum(c0, c1) - l, np.maximum(c0, c1) + l
        if per:
            w = np.minimum(hi - lo + 1, La)
            return lo, w
        lo2, hi2 = np.maximum(lo, 0), np.minimum(hi, La - 1)
        return lo2, hi2 - lo2 + 1

    def ball_mask(l):
        """[N, N] bool: site s2 within Chebyshev distance l of site s (wrapped
        on periodic axes, clipped on open ones)."""
        dxm = np.abs(xs[:, None] - xs[None, :])
        dym = np.abs(ys[:, None] - ys[None, :])
        if lat.pbc_x:
            dxm = np.minimum(dxm, Lx - dxm)
        if lat.pbc_y:
            dym = np.minimum(dym, Ly - dym)
        return (dxm <= l) & (dym <= l)

    balls = {}

    def box_count(s, x0, wx, y0, wy):
        # x0, y0 may be negative on periodic axes: shift into the middle copy
        X0 = x0 + Lx
        Y0 = y0 + Ly
        wi = np.arange(W)[:, None]
        return (s[wi, Y0 + wy, X0 + wx] - s[wi, Y0, X0 + wx] - s[wi, Y0 + wy, X0] + s[wi, Y0, X0])

    occ2 = occ.reshape(W, N)
    # kinds of connection: hops of spin 0 and 1, then (t-J) spin exchanges,
    # whose two moving spins both take the larger column form
    kinds = [(0, d) for d in range(nd)] + [(1, d) for d in range(nd)]
    if lat.tj:
        kinds += [(2, d) for d in range(4)]
    for sp, d in kinds:
        xj, yj = xs + DX[d], ys + DY[d]
        okx = (xj >= 0) & (xj < Lx) if not lat.pbc_x else np.ones_like(xj, bool)
        oky = (yj >= 0) & (yj < Ly) if not lat.pbc_y else np.ones_like(yj, bool)
        ok = okx & oky
        xjw, yjw = xj % Lx, yj % Ly
        jsite = np.where(ok, xjw + Lx * yjw, 0)
        if sp == 2:
            valid = (occ2 == 1) & ok[None, :] & (occ2[:, jsite] == 2)
        else:
            src = (ups if sp == 0 else dns).reshape(W, N)
            free = (occ2[:, jsite] == 0) if lat.tj else (src[:, jsite] == 0)
            valid = (src == 1) & ok[None, :] & free                # [W, N]
        nh = valid.sum()
        if nh == 0:
            continue
        # conv work: layer l recomputes the union of the two Chebyshev
        # balls of radius l (a rectangle for nearest-neighbour hops; for
        # diagonal hops counted from per-site masks)
        diag = DX[d] != 0 and DY[d] != 0
        for l in range(1, L + 1):
            if diag:
                if l not in balls:
                    balls[l] = ball_mask(l)
                sites = (balls[l] | balls[l][jsite]).sum(axis=1)
            else:
                _, wx = axis_range(xs, xj, l, Lx, lat.pbc_x)
                _, wy = axis_range(ys, yj, l, Ly, lat.pbc_y)
                sites = wx * wy
            conv += float((valid * sites[None, :]).sum()) * 9 * C * C * 2
            if l == L:
                conv += float((valid * sites[None, :]).sum()) * n_mlp * C * C * 2
        if diag:
            if L not in balls:
                balls[L] = ball_mask(L)
            uni = (balls[L] | balls[L][jsite]).astype(np.int64)          # [N(site i), N]
            ku = ups.reshape(W, N) @ uni.T
            kd = dns.reshape(W, N) @ uni.T
        else:
            x0, wx = axis_range(xs, xj, L, Lx, lat.pbc_x)
            y0, wy = axis_range(ys, yj, L, Ly, lat.pbc_y)
            ku = box_count(sat_u, x0[None, :], wx[None, :], y0[None, :], wy[None, :])
            kd = box_count(sat_d, x0[None, :], wx[None, :], y0[None, :], wy[None, :])
        for tau, k in ((0, ku), (1, kd)):
            r = np.minimum(k, C + (1 if tau == sp or sp == 2 else 0))
            fma = k * C * r + r ** 3 / 3.0
            det += 2.0 * float((valid * fma).sum())
    return conv, det


# ---------------------------------------------------------------------------
# oracle baseline on host cores
# ---------------------------------------------------------------------------
_CPU = {}


def ctx_hops(lat, occ):
    """Number of connected configurations (hops) per walker, counted on the host."""
    W, N = occ.shape
    nd = 8 if lat.tp != 0.0 else 4
    DX = [1, -1, 0, 0, 1, 1, -1, -1]
    DY = [0, 0, 1, -1, 1, -1, 1, -1]
    xs, ys = np.meshgrid(np.arange(lat.Lx), np.arange(lat.Ly))
    xs, ys = xs.ravel(), ys.ravel()
    cnt = np.zeros(W, np.int64)

    def target(d):
        xj, yj = xs + DX[d], ys + DY[d]
        ok = np.ones(N, bool)
        if not lat.pbc_x:
            ok &= (xj >= 0) & (xj < lat.Lx)
        if not lat.pbc_y:
            ok &= (yj >= 0) & (yj < lat.Ly)
        return ok, (xj % lat.Lx) + lat.Lx * (yj % lat.Ly)

    for sp in (0, 1):
        mine = ((occ >> sp) & 1).astype(bool)
        for d in range(nd):
            ok, j = target(d)
            free = (occ[:, j] == 0) if lat.tj else ~mine[:, j]
            cnt += np.sum(mine & ok[None, :] & free, axis=1)
    if lat.tj:
        for d in range(4):
            ok, j = target(d)
            cnt += np.sum((occ == 1) & ok[None, :] & (occ[:, j] == 2), axis=1)
    return cnt


def _cpu_init(lat, params, act):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    _CPU.update(lat=lat, params=params, act=act)


def _cpu_eloc(o):
    from oracle.energy import local_energy
    return local_energy(_CPU["lat"], _CPU["params"], o, 0, _CPU["act"])


def cpu_baseline(lat, params, occ, act, n_sample):
    import multiprocessing as mp
    cores = max(1, min(os.cpu_count() or 1, 16, n_sample))
    sample = occ[:n_sample]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_cpu_init, initargs=(lat, params, act)) as pool:
        e = pool.map(_cpu_eloc, list(sample), chunksize=1)
    dt = time.perf_counter() - t0
    return np.array(e), dt, cores


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# low-rank vs full recompute on other workloads (same GPU, same precision)
# ---------------------------------------------------------------------------
SPEEDUP_ROWS = [
    # name, workload, conv layers (None: the workload's), walkers (low-rank),
    # walkers for the full path (a prefix of the same batch), other model fields
    ("16x16, 1 conv layer", "c3", 1, 8192, 1024, {}),
    ("16x16, 1 conv layer + 4 site-wise layers, SiLU", "c3", 1, 8192, 1024, {"n_mlp": 4, "act": "silu"}),
    ("32x32 448+448, 4 conv layers", "c5", None, 1024, 4, {}),
    ("16x8 t-J cylinder 56+56, 1 conv layer + 4 site-wise layers, SiLU", "tj", None, 8192, 1024, {}),
]


def speedup_table(prec, log):
    """E_loc/s of the low-rank and the full-recompute path on the same GPU
    for each row of SPEEDUP_ROWS (seeded synthetic walkers as in the main
    workload; the full path on a prefix of the batch), with each path's
    roofline fraction from the same FLOP models as the headline."""
    import torch
    import workloads as wls
    from paper_2604_25775_amd.api import ScaleVMC
    out = []
    for name, wname, layers, W, FW, more in SPEEDUP_ROWS:
        wl = wls.get(wname)
        lat = wl.lattices[0]
        model = replace(wl.model, conv_prec=prec, **({"n_conv": layers} if layers else {}), **more)
        params = wls.quantise_params(wls.random_params([lat], model, seed=wl.seed_params), prec)
        occ = wls.occupations(wl, 0, n_walkers=W)
        ctx = ScaleVMC([lat], model.n_conv, model.channels, model.act, prec, model.refresh_every,
                       n_mlp=model.n_mlp)
        ctx.set_params_from(params)
        ctx.load([W], occ)
        e = torch.empty(W, dtype=torch.float64, device="cuda")
        ctx.tune()
        ctx.local_energy(out=e)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(3):
            ctx.prepare()
            ctx.local_energy(out=e)
        t1.record()
        torch.cuda.synchronize()
        low_ms = t0.elapsed_time(t1) / 3
        del ctx
        fctx = ScaleVMC([lat], model.n_conv, model.channels, model.act, prec, model.refresh_every,
                        n_mlp=model.n_mlp)
        fctx.set_params_from(params)
        fctx.load([FW], occ[:FW])
        fe = torch.empty(FW, dtype=torch.float64, device="cuda")
        fctx.local_energy("full", out=fe)
        e2 = torch.empty(FW, dtype=torch.float64, device="cuda")
        fctx.local_energy(out=e2)
        t0.record()
        fctx.local_energy("full", out=fe)
        t1.record()
        torch.cuda.synchronize()
        full_ms = t0.elapsed_time(t1)
        agree = float(np.max(np.abs(fe.cpu().numpy() - e2.cpu().numpy()) / np.maximum(1.0, np.abs(e2.cpu().numpy()))))
        del fctx
        low_rate, full_rate = W / (low_ms / 1e3), FW / (full_ms / 1e3)
        conv_f, det_f = lowrank_flops(lat, occ, model.n_conv, model.channels, model.n_mlp)
        conv_peak = PEAK_BF16 if prec in ("bf16", "bf16x3", "f16x2") else (PEAK_FP32 if prec == "f32" else PEAK_FP64)
        t_low = conv_f / conv_peak + det_f / PEAK_FP64
        nhop = float(np.sum(ctx_hops(lat, occ[:FW])))
        conv_full = nhop * (9 * model.n_conv + model.n_mlp) * lat.N * model.channels ** 2 * 2
        fp64_full = nhop * sum(2.0 * n * n * model.channels + 2.0 / 3.0 * n ** 3 for n in (lat.n_up, lat.n_dn))
        t_full = conv_full / conv_peak + fp64_full / PEAK_FP64
        row = {"workload": f"{name} ({wname}, Hubbard {lat.Lx}x{lat.Ly}, {model.channels} ch, {prec})",
               "lowrank_eloc_per_s": round(low_rate, 1), "lowrank_walkers": W,
               "lowrank_roofline_frac": round(t_low / (low_ms / 1e3), 4),
               "full_recompute_eloc_per_s": round(full_rate, 2), "full_recompute_walkers": FW,
               "full_recompute_roofline_frac": round(t_full / (full_ms / 1e3), 4),
               "speedup_vs_full": round(low_rate / full_rate, 2),
               "speedup_at_equal_roofline_frac": round((t_full / FW) / (t_low / W), 2),
               "lowrank_vs_full_max_rel_diff": agree}
        log(f"[bench] {name}: low-rank {low_rate:.1f} E_loc/s ({row['lowrank_roofline_frac']:.3f} of roofline), "
            f"full {full_rate:.2f} E_loc/s ({row['full_recompute_roofline_frac']:.3f}), "
            f"speed-up {row['speedup_vs_full']:.1f}x (model at equal efficiency "
            f"{row['speedup_at_equal_roofline_frac']:.1f}x)")
        out.append(row)
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# one launch over a mixed batch of lattices (ragged hop counts)
# ---------------------------------------------------------------------------
def symmetric_eloc(prec, log, wname="c3", W=1024):
    """Local energy of the symmetry-projected amplitude at the bench lattice:
    D2 (both mirrors) x spin inversion, 8 elements, on W base walkers (the
    seeded occupations), i.e. 8 W copies through the low-rank kernels plus
    the combination; base walkers per second."""
    import torch
    import workloads as wls
    from paper_2604_25775_amd.api import ScaleVMC
    wl = wls.get(wname)
    lat = wl.lattices[0]
    model = replace(wl.model, conv_prec=prec)
    params = wls.quantise_params(wls.random_params([lat], model, seed=wl.seed_params), prec)
    G, chi = wls.symmetry_group(lat, [("mx", 1.0), ("my", 1.0), ("flip", 1.0)])
    occ = wls.occupations(wl, 0, n_walkers=W)
    ctx = ScaleVMC([lat], model.n_conv, model.channels, model.act, prec, model.refresh_every, n_mlp=model.n_mlp)
    ctx.set_params_from(params)
    ctx.set_symmetry(G, chi)
    cp = ctx.sym_expand(torch.from_numpy(occ).cuda())
    ctx.load([W * len(G)], cp)
    ctx.tune()
    ctx.local_energy_sym()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(3):
        ctx.prepare()
        e, _, _ = ctx.local_energy_sym()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 3
    ok = bool(torch.isfinite(e).all().item())
    # one sweep of |psi_sym|^2 (N proposals per walker, every copy moved)
    t0.record()
    n_acc = ctx.sweep_sym(1, wl.seed_mc, 0)
    t1.record()
    torch.cuda.synchronize()
    sweep_ms = t0.elapsed_time(t1)
    acc_rate = float(n_acc[::len(G)].sum().item()) / (W * lat.N)
    e2, _, _ = ctx.local_energy_sym()
    ok = ok and bool(torch.isfinite(e2).all().item())
    del ctx
    row = {"workload": f"{wname} lattice, {W} walkers x |G| = {len(G)} (mirrors x, y; spin inversion)",
           "group_order": len(G), "walkers": W, "ms": round(ms, 3),
           "eloc_sym_per_s": round(W / (ms / 1e3), 1), "copies_eloc_per_s": round(W * len(G) / (ms / 1e3), 1),
           "sym_sweep_ms": round(sweep_ms, 2), "sym_accept_rate": round(acc_rate, 4), "all_finite": ok}
    log(f"[bench] symmetric E_loc (|G| = {len(G)}): {ms:.2f} ms for {W} walkers -> "
        f"{row['eloc_sym_per_s']:.1f} E_sym/s ({row['copies_eloc_per_s']:.1f} copies/s); "
        f"one |psi_sym|^2 sweep {sweep_ms:.1f} ms, accept rate {acc_rate:.3f}")
    return row


def mixed_launch(log, wname="c4"):
    """E_loc/s of the mixed-lattice workload in one launch (after the
    workload's thermalising sweeps), against the same walkers evaluated one
    lattice per launch, with the launch's roofline fraction (conv at the
    precision's peak, determinant work at FP64 peak)."""
    import torch
    import workloads as wls
    from paper_2604_25775_amd.api import ScaleVMC
    wl = wls.get(wname)
    lats, counts, model = list(wl.lattices), list(wl.walkers), wl.model
    params = wls.quantise_params(wls.random_params(lats, model, seed=wl.seed_params), model.conv_prec)
    occs = [wls.occupations(wl, k, n_walkers=n) for k, n in enumerate(counts)]

    def timed(ctx, W):
        e = torch.empty(W, dtype=torch.float64, device="cuda")
        ctx.tune()
        ctx.local_energy(out=e)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(3):
            ctx.prepare()
            ctx.local_energy(out=e)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / 3, ctx.get_launch()

    ctx = ScaleVMC(lats, model.n_conv, model.channels, model.act, model.conv_prec, model.refresh_every)
    ctx.set_params_from(params)
    ctx.load(counts, np.concatenate([o.reshape(-1) for o in occs]).astype(np.int8))
    if wl.sweeps:
        ctx.sweep(wl.sweeps, wl.seed_mc, 0)
    occ_all, _ = ctx.state()
    occ_all = occ_all.cpu().numpy()
    mixed_ms, launch = timed(ctx, sum(counts))
    del ctx
    single_ms, off, conv_f, det_f, hops = [], 0, 0.0, 0.0, []
    for k, (lat, n) in enumerate(zip(lats, counts)):
        occ_k = occ_all[off: off + n * lat.N].reshape(n, lat.N)
        off += n * lat.N
        c1, d1 = lowrank_flops(lat, occ_k, model.n_conv, model.channels)
        conv_f, det_f = conv_f + c1, det_f + d1
        hops.append(float(np.mean(ctx_hops(lat, occ_k))))
        sctx = ScaleVMC([lat], model.n_conv, model.channels, model.act, model.conv_prec, model.refresh_every)
        sctx.set_params_from(params_for(params, k))
        sctx.load([n], occ_k)
        single_ms.append(timed(sctx, n)[0])
        del sctx
    conv_peak = {"f32": PEAK_FP32, "f64": PEAK_FP64}.get(model.conv_prec, PEAK_BF16)
    t_peak = conv_f / conv_peak + det_f / PEAK_FP64
    W = sum(counts)
    row = {"workload": f"{wname}: " + " + ".join(f"{l.Lx}x{l.Ly} ({n} walkers, {h:.0f} hops each)"
                                                 for l, n, h in zip(lats, counts, hops))
           + f", {model.n_conv} conv x {model.channels} ch, conv {model.conv_prec}",
           "eloc_per_s": round(W / (mixed_ms / 1e3), 1), "launch_ms": round(mixed_ms, 3),
           "launch": launch, "roofline_frac": round(t_peak / (mixed_ms / 1e3), 4),
           "one_lattice_per_launch_ms": [round(t, 3) for t in single_ms],
           "mixed_vs_separate": round(sum(single_ms) / mixed_ms, 3)}
    log(f"[bench] {wname} mixed batch: one launch {mixed_ms:.2f} ms ({row['eloc_per_s']:.0f} E_loc/s, "
        f"{row['roofline_frac']:.3f} of roofline) vs {sum(single_ms):.2f} ms one lattice per launch")
    return row


def params_for(params, k):
    """The parameters of a mixed batch restricted to lattice k (shared conv,
    that lattice's projection, base orbitals and per-site embedding)."""
    q = params.copy()
    q.proj_w, q.proj_b, q.base = [params.proj_w[k]], [params.proj_b[k]], [params.base[k]]
    if q.embed_site is not None:
        q.embed_site = [params.embed_site[k]]
    return q


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--prec", default="f16x2", choices=["bf16", "bf16x3", "f16x2", "f32", "f64"])
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--full-walkers", type=int, default=None,
                    help="walkers for the full-recompute timing (default: all)")
    ap.add_argument("--cpu-sample", type=int, default=288)
    ap.add_argument("--therm", type=int, default=8, help="thermalising sweeps before timing (untimed)")
    ap.add_argument("--no-full", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-speedup-table", action="store_true",
                    help="skip the low-rank vs full-recompute rows of the other workloads "
                         "and the mixed-lattice launch")
    ap.add_argument("--launch", default=None, metavar="SLICES,ROWFORM",
                    help="fixed E_loc launch shape (svmc_set_launch) instead of the autotuner")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (default: tune, do not store)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="after the sweeps and the tuner: one E_loc step and one copy of "
                         "COPY_PROBE_BYTES, then exit (the program for rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE runs)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {a.gpus}); the walker-parallel "
              f"multi-GPU design is described in DESIGN.md but not run here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wls
    from paper_2604_25775_amd.api import ScaleVMC

    wl = wls.get(a.workload)
    lat = wl.lattices[0]
    model = replace(wl.model, conv_prec=a.prec)
    W = a.walkers or wl.walkers[0]
    log(f"[bench] workload {wl.name}: {wl.description}; walkers {W}, conv {a.prec}")
    params = wls.quantise_params(wls.random_params([lat], model, seed=wl.seed_params), a.prec)
    occ = wls.occupations(wl, 0, n_walkers=W)

    ctx = ScaleVMC([lat], model.n_conv, model.channels, model.act, a.prec, model.refresh_every)
    ctx.set_params_from(params)
    ctx.load([W], occ)
    torch.cuda.synchronize()
    eloc = torch.empty(W, dtype=torch.float64, device="cuda")
    extra = {}
    if a.therm > 0:
        # Metropolis sweeps from the random start; E_loc is then measured on
        # the caches the sweeps leave (features, G and P maintained in place)
        t0 = time.perf_counter()
        nacc = ctx.sweep(a.therm, wl.seed_mc, 0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rate = float(nacc.double().mean().item()) / (a.therm * lat.N)
        extra.update({"therm_sweeps": a.therm, "therm_sweep_ms": round(dt * 1e3 / a.therm, 2),
                      "accept_rate": round(rate, 4)})
        log(f"[bench] {a.therm} sweeps: {dt * 1e3 / a.therm:.1f} ms per sweep of {W} walkers, "
            f"accept rate {rate:.3f}")
        occ_t, _ = ctx.state()
        occ = occ_t.cpu().numpy().reshape(W, lat.N)

    if a.launch:
        sl_, rf_ = (int(v) for v in a.launch.split(","))
        ctx.set_launch(sl_, rf_)
        slices = sl_
    else:
        slices = ctx.tune(a.tune_cache)
    rfm = ctx.get_launch()["row_form_max"]
    extra["eloc_slices_per_walker"] = slices
    extra["eloc_row_form_max"] = rfm
    log(f"[bench] autotuner: {slices} workgroups per walker, row form up to {rfm} changed rows")
    if a.traffic_probe:
        ctx.prepare()
        ctx.local_energy(out=eloc)
        torch.cuda.synchronize()
        x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"[bench] traffic probe: one E_loc step, then a copy of {COPY_PROBE_BYTES} bytes "
            f"(sources {kernel_src_sha1()})")
        return
    for _ in range(a.warmup):
        ctx.prepare()
        ctx.local_energy(out=eloc)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({a.warmup} steps)")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        evs[k][0].record()
        ctx.prepare()
        evs[k][1].record()
        ctx.local_energy(out=eloc)
        evs[k][2].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / a.steps * 1e3
    prep_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    kern_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    value = W / (ms_step / 1e3)
    log(f"[bench] {a.steps} steps: {ms_step:.3f} ms/step, precompute {prep_ms:.3f} ms, "
        f"E_loc kernel {kern_ms:.3f} ms -> {value:.1f} E_loc/s")
    e_gpu = eloc.cpu().numpy()
    flags = ctx.flags().cpu().numpy()

    conv_f, det_f = lowrank_flops(lat, occ, model.n_conv, model.channels)
    conv_peak = PEAK_BF16 if a.prec in ("bf16", "bf16x3", "f16x2") else (PEAK_FP32 if a.prec == "f32" else PEAK_FP64)
    passes = {"bf16x3": 3, "f16x2": 2}.get(a.prec, 1)
    # the method's own work, each conv product counted once at the 16-bit
    # MFMA peak (the extra passes of the split modes only carry precision)
    t_peak = conv_f / conv_peak + det_f / PEAK_FP64
    t_peak_passes = conv_f * passes / conv_peak + det_f / PEAK_FP64
    kern_s = kern_ms / 1e3
    achieved = (conv_f + det_f) / kern_s / 1e12
    peak = (conv_f + det_f) / t_peak / 1e12
    tr = traffic_record(wl.name, W, a.prec, slices, rfm)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": round(peak, 3),
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": round(tr["bytes"]) if tr else None,
                "traffic_note": (f"HBM bytes per launch, FETCH_SIZE + WRITE_SIZE scaled by a "
                                 f"{COPY_PROBE_BYTES}-byte copy ({tr['file']}, {slices} slices per walker)")
                                if tr else f"no counter record for these sources at {slices} slices per walker",
                "kernel": "k_eloc_lowrank",
                "flops_conv_per_launch": conv_f, "flops_fp64_per_launch": det_f,
                "peak_model": "time at peak = conv/(%.4g) + fp64/(%.4g), conv counted once"
                              % (conv_peak, PEAK_FP64),
                "t_peak_ms": round(t_peak * 1e3, 4),
                "conv_passes": passes,
                "frac_pass_inclusive": round(t_peak_passes / kern_s, 4)}
    log(f"[bench] roofline: conv {conv_f / 1e12:.3f} TFLOP + fp64 {det_f / 1e12:.3f} TFLOP per launch; "
        f"t_peak {t_peak * 1e3:.3f} ms vs {kern_ms:.3f} ms -> frac {t_peak / kern_s:.4f} "
        f"({t_peak_passes / kern_s:.4f} with all {passes} conv passes counted)")

    extra.update({"prepare_ms": round(prep_ms, 4), "eloc_kernel_ms": round(kern_ms, 4),
                  "walkers_flagged": {"singular": int(np.count_nonzero(flags & 1)),
                                      "nonfinite": int(np.count_nonzero(flags & 2)),
                                      "drift": int(np.count_nonzero(flags & 4)),
                                      "badcount": int(np.count_nonzero(flags & 8))}})
    if not a.no_graph:
        # the same step recorded once as a HIP graph and replayed
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.prepare()
            ctx.local_energy(out=eloc)
        g.replay()
        torch.cuda.synchronize()
        t0g = time.perf_counter()
        for _ in range(a.steps):
            g.replay()
        torch.cuda.synchronize()
        extra["graph_ms_per_step"] = round((time.perf_counter() - t0g) / a.steps * 1e3, 4)
        log(f"[bench] graph replay: {extra['graph_ms_per_step']:.3f} ms/step")
    if not a.no_grad:
        v = torch.ones(W, dtype=torch.float64, device="cuda")
        ctx.grad_logpsi(v)
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record()
        ctx.grad_logpsi(v)
        g1.record()
        torch.cuda.synchronize()
        extra["grad_vjp_ms"] = round(g0.elapsed_time(g1), 3)
        log(f"[bench] gradient VJP over {W} walkers: {extra['grad_vjp_ms']:.1f} ms")
    if not a.no_full:
        FW = a.full_walkers or W
        if FW == W:
            fctx = ctx
        else:
            fctx = ScaleVMC([lat], model.n_conv, model.channels, model.act, a.prec, model.refresh_every)
            fctx.set_params_from(params)
            fctx.load([FW], occ[:FW])
        feloc = torch.empty(FW, dtype=torch.float64, device="cuda")
        log(f"[bench] full-recompute path on {FW} walkers ...")
        fctx.local_energy("full", out=feloc)      # warm
        torch.cuda.synchronize()
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record()
        fctx.local_energy("full", out=feloc)
        f1.record()
        torch.cuda.synchronize()
        full_ms = f0.elapsed_time(f1)
        full_rate = FW / (full_ms / 1e3)
        ef = feloc.cpu().numpy()
        agree = float(np.max(np.abs(ef - e_gpu[:FW]) / np.maximum(1.0, np.abs(ef))))
        # the full path's own algorithmic work: per hop a full forward of all
        # N sites (conv passes as above), both spins' N_s rows (C MACs each
        # per orbital) and an LU of each N_s x N_s block
        occ_f = occ[:FW]
        nhop = float(np.sum(ctx_hops(lat, occ_f)))
        N = lat.N
        conv_full = nhop * model.n_conv * N * 9 * model.channels ** 2 * 2
        fp64_full = nhop * sum(2.0 * n * n * model.channels + 2.0 / 3.0 * n ** 3 for n in (lat.n_up, lat.n_dn))
        tpk_full = conv_full / conv_peak + fp64_full / PEAK_FP64
        tpk_low = t_peak * FW / W
        extra.update({"full_recompute_roofline_frac": round(tpk_full / (full_ms / 1e3), 4),
                      "speedup_at_equal_roofline_frac": round(tpk_full / tpk_low, 2)})
        extra.update({"full_recompute_eloc_per_s": round(full_rate, 1), "full_recompute_walkers": FW,
                      "full_recompute_ms": round(full_ms, 3),
                      "speedup_vs_full": round(value / full_rate, 3),
                      "speedup_kernel_only": round((FW / (full_ms / 1e3)) and (W / (kern_ms / 1e3)) / full_rate, 3),
                      "lowrank_vs_full_max_rel_diff": agree})
        log(f"[bench] full path: {full_ms:.1f} ms for {FW} walkers -> {full_rate:.1f} E_loc/s; "
            f"speed-up {value / full_rate:.2f}x; max |dE|/E lowrank vs full {agree:.2e}")

    if not a.no_speedup_table:
        extra["speedup_table"] = speedup_table(a.prec, log)
        extra["mixed_lattice_launch"] = mixed_launch(log)
        extra["symmetric_eloc"] = symmetric_eloc(a.prec, log)

    cpu = None
    if not a.no_cpu and a.cpu_sample > 0:
        log(f"[bench] oracle on host cores, {a.cpu_sample} walkers ...")
        e_ref, dt, cores = cpu_baseline(lat, params, occ, model.act, a.cpu_sample)
        err = float(np.max(np.abs(e_gpu[:len(e_ref)] - e_ref) / np.maximum(1.0, np.abs(e_ref))))
        cpu = {"value": round(len(e_ref) / dt, 3), "unit": "E_loc/s", "cores": cores, "kind": "oracle",
               "sample": f"first {len(e_ref)} walkers of the same batch, full FP64 recompute per hop "
                         f"({dt:.1f} s wall on {cores} processes, {cpu_model()})"}
        extra["max_rel_err_eloc_vs_oracle"] = err
        log(f"[bench] oracle {len(e_ref) / dt:.3f} E_loc/s on {cores} cores; max rel err of GPU E_loc {err:.2e}")

    line = {
        "metric": "local-energy evals/sec at 16x16 1/8-doped; speedup vs full-recompute",
        "value": round(value, 1), "unit": "E_loc/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{a.prec}+f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: Hubbard {lat.Lx}x{lat.Ly} pbc_x={lat.pbc_x} pbc_y={lat.pbc_y} "
                               f"U={lat.U} t'={lat.tp} n={lat.n_up}+{lat.n_dn}, {model.n_conv} conv x "
                               f"{model.channels} ch, {W} walkers",
                   "walkers": W, "conv_prec": a.prec, **extra},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
