"""svmc_local_energy_noalloc (the local-energy entry point that allocates
nothing; its partial sums live in a fixed per-device array) against
svmc_local_energy(LOWRANK) through the C ABI: bit-identical E_loc on two
calls in a row, the second with a smaller batch (another context with fewer
walkers on the same device, so the shared array keeps the first call's
contents), also after a Metropolis sweep; a batch whose partial sums would
not fit the array is refused with SVMC_ERR_UNSUPPORTED."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, say  # noqa: E402


def both(ctx):
    W = ctx.num_walkers
    ref = ctx.local_energy()
    out = torch.full((W,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.local_energy_noalloc(out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_equals_lowrank_two_calls_smaller_second():
    lat = wl.Lattice(10, 10, 1, 0, 1.0, 0.0, 8.0, 44, 44)
    model = wl.Model(4, 32, "tanh", "f16x2", 32)
    say("[noalloc] 10x10 f16x2, 300 walkers then 37")
    ctx, params, occs = build([lat], model, [300], backflow=0.1)
    a, b = both(ctx)
    assert np.isfinite(a).all() and np.array_equal(a, b)
    ctx2, _, _ = build([lat], model, [37], seed_occ=5, backflow=0.1)
    a2, b2 = both(ctx2)
    assert np.array_equal(a2, b2)
    assert not np.array_equal(a2, a[:37])
    ctx2.sweep(1, 3, 0)
    a3, b3 = both(ctx2)
    assert np.array_equal(a3, b3)
    # the first context again, after the smaller one used the array
    a4, b4 = both(ctx)
    assert np.array_equal(a4, a) and np.array_equal(b4, a)


def test_noalloc_mixed_lattices_fp64():
    lats = [wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5), wl.Lattice(5, 3, 0, 1, 1.0, 0.3, 6.0, 4, 3)]
    model = wl.Model(2, 8, "tanh", "f64")
    ctx, _, _ = build(lats, model, [5, 6], backflow=0.5)
    a, b = both(ctx)
    assert np.array_equal(a, b)


def test_noalloc_refuses_oversized_batch():
    from paper_2604_25775_amd._lib import SvmcError
    lat = wl.Lattice(3, 3, 1, 1, 1.0, 0.0, 4.0, 2, 2)
    model = wl.Model(1, 8, "tanh", "f64")
    W = (1 << 20) // 8 + 1            # default launch: 8 slices per walker
    ctx, _, _ = build([lat], model, [W])
    out = torch.empty(W, dtype=torch.float64, device="cuda")
    with pytest.raises(SvmcError) as ei:
        ctx.local_energy_noalloc(out)
    assert ei.value.status == 5
