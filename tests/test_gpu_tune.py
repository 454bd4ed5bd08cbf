"""The launch-shape autotuner: it times the low-rank E_loc launch for several
slice counts, keeps the fastest, stores it in a cache file and reuses it; the
result does not depend on the choice beyond summation order."""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_util import build, say  # noqa: E402


def test_tune_cache_and_results(tmp_path):
    lat = wl.Lattice(8, 8, 1, 1, 1.0, 0.0, 8.0, 28, 28)
    model = wl.Model(2, 16, "tanh", "f64")
    ctx, params, occs = build([lat], model, [64], backflow=0.5)
    e0 = ctx.local_energy().cpu().numpy()
    cache = tmp_path / "tune.txt"
    s1 = ctx.tune(str(cache))
    say(f"[tune] chose {s1} slices; cache: {cache.read_text().strip()}")
    assert s1 in (1, 2, 4, 8, 16, 24, 32)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and f"slices={s1}" in lines[0]
    e1 = ctx.local_energy().cpu().numpy()
    assert np.max(np.abs(e1 - e0) / np.maximum(1.0, np.abs(e0))) < 1e-12
    # a second context with the same shape reads the cache (no new line)
    ctx2, _, _ = build([lat], model, [64], backflow=0.5)
    assert ctx2.tune(str(cache)) == s1
    assert len(cache.read_text().splitlines()) == 1
