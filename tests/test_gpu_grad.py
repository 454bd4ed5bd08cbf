"""GPU gradient of log|psi| with respect to the flat parameter vector,
through the C ABI, against the oracle's autograd gradient (torch FP64 conv2d
+ slogdet on the CPU, itself pinned by central differences).

FP64 conv: per walker, |g - g_ref| <= 1e-10 max(1, max|g_ref|) on every
entry.  FP32-feature paths (f32, bf16x3) carry the FP32 rounding of the
cached activations: 2e-5 of the same scale.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, say  # noqa: E402
from oracle.grad import autograd_grad  # noqa: E402

CASES = [
    ("4x4pbc_L2C8", [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)], wl.Model(2, 8, "tanh", "f64"), [4]),
    ("3x5open_x_L1C8_silu", [wl.Lattice(3, 5, 0, 1, 1.0, 0.3, 4.0, 4, 3)], wl.Model(1, 8, "silu", "f64"), [4]),
    ("6x4open_y_L3C16", [wl.Lattice(6, 4, 1, 0, 1.0, 0.0, 8.0, 9, 10)], wl.Model(3, 16, "tanh", "f64"), [3]),
    ("mixed_4x4_5x3open_L2C8", [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 8.0, 5, 5),
                                wl.Lattice(5, 3, 0, 1, 1.0, 0.0, 8.0, 4, 2)], wl.Model(2, 8, "tanh", "f64"), [2, 3]),
]


def jac_ref(lats, params, occs, act):
    rows = []
    for li, (lat, occ) in enumerate(zip(lats, occs)):
        for o in occ:
            rows.append(autograd_grad(lat, params, o, li, act)[1])
    return np.stack(rows)


def check_rows(J, R, tol):
    worst = 0.0
    for w in range(R.shape[0]):
        scale = max(1.0, float(np.max(np.abs(R[w]))))
        err = float(np.max(np.abs(J[w] - R[w]))) / scale
        worst = max(worst, err)
        assert err <= tol, (w, err, int(np.argmax(np.abs(J[w] - R[w]))))
    return worst


@pytest.mark.parametrize("name,lats,model,counts", CASES, ids=[c[0] for c in CASES])
def test_jacobian_fp64_matches_oracle(name, lats, model, counts):
    say(f"[grad f64] {name}")
    ctx, params, occs = build(lats, model, counts, backflow=0.5)
    J = ctx.grad_logpsi().cpu().numpy()
    assert J.shape == (sum(counts), ctx.num_params)
    worst = check_rows(J, jac_ref(lats, params, occs, model.act), 1e-10)
    say(f"  worst {worst:.3e}")


def test_gradient_after_sweeps_and_vjp():
    """After Metropolis moves (stale inverses) the gradient is taken at the
    new configurations; the VJP equals the weighted row sum; LogPsi.backward
    gives the same vector."""
    from paper_2604_25775_amd.api import LogPsi, pack_params
    lat = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 4)
    model = wl.Model(2, 8, "tanh", "f64", 4)
    say("[grad f64 after sweeps / vjp]")
    ctx, params, occs = build([lat], model, [5], backflow=0.5)
    ctx.sweep(2, 77, 0)
    occ, _ = ctx.state()
    new = occ.cpu().numpy().reshape(5, lat.N)
    J = ctx.grad_logpsi().cpu().numpy()
    check_rows(J, jac_ref([lat], params, [new], model.act), 1e-10)
    v = torch.linspace(-1.0, 2.0, 5, dtype=torch.float64, device="cuda")
    g = ctx.grad_logpsi(v).cpu().numpy()
    ref = v.cpu().numpy() @ J
    assert np.max(np.abs(g - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    theta = torch.from_numpy(pack_params(params, [lat])).cuda().requires_grad_(True)
    la = LogPsi.apply(theta, ctx)
    (la * v).sum().backward()
    assert np.max(np.abs(theta.grad.cpu().numpy() - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
    _, la_ref = ctx.log_psi()
    assert torch.allclose(la, la_ref)


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f16x2"])
def test_jacobian_fp32_features(prec):
    lat = wl.Lattice(6, 6, 1, 0, 1.0, 0.0, 8.0, 15, 15)
    model = wl.Model(3, 16, "tanh", prec)
    say(f"[grad {prec}]")
    ctx, params, occs = build([lat], model, [3], backflow=0.3)
    J = ctx.grad_logpsi().cpu().numpy()
    worst = check_rows(J, jac_ref([lat], params, occs, model.act), 2e-5)
    say(f"  worst {worst:.3e}")


def test_flagged_walker_rows():
    lat = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)
    model = wl.Model(1, 8, "tanh", "f64")
    occ = wl.random_occupations(lat, 3, seed=6)
    occ[2, np.nonzero(occ[2] & 2)[0][0]] -= 2          # one down electron missing
    ctx, params, _ = build([lat], model, [3], occ_list=[occ])
    J = ctx.grad_logpsi().cpu().numpy()
    assert np.isnan(J[2]).all() and np.isfinite(J[:2]).all()
    v = torch.ones(3, dtype=torch.float64, device="cuda")
    g = ctx.grad_logpsi(v).cpu().numpy()
    assert np.max(np.abs(g - (J[0] + J[1]))) <= 1e-12 * max(1.0, np.max(np.abs(J[:2])))
