"""Autotuner on a small system: every search returns parameters the library
accepts, the cache records what was tried, and a context built with the
chosen parameters reproduces the default context's results to the parity
tolerance (launch shape changes only the summation order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def sg():
    _need_gpu()
    from paper_1807_08116_amd import sphgrav
    sphgrav.lib()
    return sphgrav


@pytest.fixture(scope="module")
def small():
    from paper_1807_08116_amd import ic
    return ic.make("c0", scale=0.25)             # 1024 gas + 1024 halo


def _accel(eng, sg):
    eng.build_neighbors()
    eng.ctx.compute_density()
    eng.ctx.compute_accel(sg.SG_SPH | sg.SG_GRAV | sg.SG_POT)
    eng.ctx.sync()
    return np.stack([eng.numpy(f) for f in ("ax", "ay", "az")], 1)


@pytest.mark.parametrize("form", ["fp32c", "fp64"])
def test_tune_gravity_and_cells(sg, small, form, tmp_path):
    from paper_1807_08116_amd import autotune
    p = sg.SG_FP32C if form == "fp32c" else sg.SG_FP64
    cache = str(tmp_path / "cache.json")
    best = autotune.tune_gravity(small, p, reps=1, path=cache)
    cell = autotune.tune_cells(small, p, reps=1, path=cache)
    assert cell in autotune.CELL_SCALES
    n = len(small["x"])
    assert autotune.lookup("grav", p, n, cache) == best
    assert autotune.lookup("cells", p, small["ng"], cache) == cell
    tried = autotune.load_cache(cache)["grav:%d:%d" % (p, 2048)]["tried"]
    assert len(tried) >= 5 and all(r["ms"] > 0 for r in tried)
    ref = _accel(sg.Engine(small, precision=p), sg)
    got = _accel(sg.Engine(small, precision=p, cell_scale_log2=cell, **best), sg)
    tol = 1e-12 if form == "fp64" else 1e-6
    assert np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2)) < tol


def test_tune_ensemble(sg, tmp_path):
    from paper_1807_08116_amd import autotune, ic
    states = ic.ensemble(nsys=3, scale=0.02)
    cache = str(tmp_path / "cache.json")
    shape = autotune.tune_ensemble(states, reps=1, path=cache)
    assert shape["grav_ipl"] in autotune.IPLS and shape["grav_tile"] in autotune.TILES
    ens = sg.Ensemble(states, **shape)
    ens.gravity(sg.SG_GRAV | sg.SG_POT)
    ens.torch.cuda.synchronize()
    for st, eng in zip(states, ens.engines):
        single = sg.Engine(st, precision=sg.SG_FP32C, grav_split=1, **shape)
        single.ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)
        single.ctx.sync()
        np.testing.assert_array_equal(eng.numpy("ax"), single.numpy("ax"))
