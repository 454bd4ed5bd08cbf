"""FP16-pair rounding of the f16x2 mode's parameters (workloads.f16_rtz /
f16_pair), checked against torch's FP16 conversion and the pair's
definition: hi = x rounded toward zero to FP16, lo = (x - hi) rounded toward
zero to FP16, value hi + lo."""
import numpy as np
import torch

import workloads as wl


def _rtz_reference(x: np.ndarray) -> np.ndarray:
    # FP16 round-to-nearest, stepped one FP16 ulp toward zero where it rounded
    # away from zero
    t = torch.from_numpy(x).to(torch.float16)
    away = t.to(torch.float32).abs() > torch.from_numpy(x).abs()
    step = torch.nextafter(t, torch.zeros_like(t))
    return torch.where(away, step, t).to(torch.float32).numpy()


def test_rtz_matches_fp16_toward_zero():
    rng = np.random.default_rng(11)
    x = np.concatenate([
        rng.standard_normal(20000),
        rng.standard_normal(5000) * 1e-5,          # FP16 subnormal range
        rng.uniform(-60000, 60000, 2000),
        [0.0, -0.0, 1.0, -1.0, 2.0 ** -14, 2.0 ** -24, 3 * 2.0 ** -25, 65504.0, -65504.0],
    ]).astype(np.float32)
    got = wl.f16_rtz(x)
    ref = _rtz_reference(x)
    assert np.array_equal(got, ref)
    assert np.all(np.abs(got) <= np.abs(x))


def test_pair_terms_and_error():
    rng = np.random.default_rng(12)
    x = (rng.standard_normal(20000) * rng.choice([1e-3, 0.1, 1.0, 30.0], 20000)).astype(np.float32)
    p = wl.f16_pair(x)
    h = wl.f16_rtz(x)
    lo = (p - h).astype(np.float32)
    # lo is itself an FP16 value and hi + lo is exact in FP32
    assert np.array_equal(wl.f16_rtz(lo), lo)
    assert np.array_equal(p.astype(np.float32).astype(np.float64), p)
    # error: 2^-21 relative in FP16's normal range for lo, 2^-24 absolute below
    err = np.abs(p - x.astype(np.float64))
    bound = np.maximum(np.abs(x.astype(np.float64)) * 2.0 ** -20, 2.0 ** -24)
    assert np.all(err <= bound)
    # pair values are fixed points (the device splits them exactly)
    assert np.array_equal(wl.f16_pair(p.astype(np.float32)), p)


def test_quantised_f16x2_params_are_pairs():
    lat = wl.Lattice(4, 4, 1, 1, 1.0, 0.0, 4.0, 5, 5)
    model = wl.Model(2, 8, "tanh", "f16x2")
    prm = wl.quantise_params(wl.random_params([lat], model, seed=3), "f16x2")
    assert np.array_equal(wl.f16_pair(prm.embed.astype(np.float32)), prm.embed)
    w = torch.from_numpy(prm.conv_w)
    assert torch.equal(w.to(torch.float16).to(torch.float64), w)
