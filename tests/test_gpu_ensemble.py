"""Ensembles: gravity of several systems in one persistent launch equals
each system's own gravity (same kernel body, same targets per workgroup);
ensemble steps equal per-system steps; graph replays equal eager ensemble
steps."""
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
def states():
    from paper_1807_08116_amd import ic
    return ic.ensemble(nsys=5, scale=0.05)          # 5 systems of ~400..13000 particles


@pytest.mark.parametrize("ipl,tile", [(2, 256), (1, 128), (4, 512)])
def test_ensemble_gravity_matches_single(sg, orc, states, ipl, tile):
    ens = sg.Ensemble(states, grav_ipl=ipl, grav_tile=tile)
    ens.gravity(sg.SG_GRAV | sg.SG_POT)
    ens.torch.cuda.synchronize()
    for st, eng in zip(states, ens.engines):
        single = sg.Engine(st, precision=sg.SG_FP32C, grav_split=1, grav_ipl=ipl, grav_tile=tile)
        single.ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)
        single.ctx.sync()
        for f in ("ax", "ay", "az", "pot"):
            np.testing.assert_array_equal(eng.numpy(f), single.numpy(f), err_msg=f)
        # and against the oracle on a few targets
        t = np.arange(0, len(st["x"]), 97)
        gx, gy, gz, gp = orc.gravity(st["x"], st["y"], st["z"], st["m"], 1.0, 0.01, t)
        ref = np.stack([gx, gy, gz], 1)
        got = np.stack([eng.numpy(f)[t] for f in ("ax", "ay", "az")], 1)
        assert np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2)) < 1e-6


def test_ensemble_steps_match_single_and_graph(sg, states):
    dt = 1e-3
    eager = sg.Ensemble(states, grav_ipl=2)
    eager.run(dt, 4, sg.SG_POT, use_graph=False)
    graph = sg.Ensemble(states, grav_ipl=2)
    graph.run(dt, 4, sg.SG_POT, use_graph=True)
    for st, e1, e2 in zip(states, eager.engines, graph.engines):
        single = sg.Engine(st, precision=sg.SG_FP32C, grav_split=1, grav_ipl=2)
        for _ in range(4):
            single.ctx.step(dt, sg.SG_POT)
        single.ctx.sync()
        for f in ("x", "y", "z", "vx", "vy", "vz", "e", "ax", "pot"):
            a, b, c = e1.numpy(f), e2.numpy(f), single.numpy(f)
            np.testing.assert_array_equal(a, b, err_msg="graph " + f)
            np.testing.assert_array_equal(a, c, err_msg="single " + f)
