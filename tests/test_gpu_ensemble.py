"""Ensembles: gravity of several systems in one persistent launch equals
each system's own gravity (same kernel body, same targets per workgroup);
ensemble steps equal per-system steps; graph replays equal eager ensemble
steps.  At the full ensemble size (64 systems, 4659360 particles), in the
tuned launch: batched gravity equals the systems' own launches bit for bit
on four systems (largest, smallest, two others) and the oracle on 256
seeded targets of each; one ensemble step keeps every system's momentum."""
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


@pytest.mark.parametrize("other", [dict(eps=0.02), dict(grav_reorder=4), dict(precision="fp64"),
                                   dict(stream="new")])
def test_ensemble_create_rejects_mismatched_contexts(sg, states, other):
    # every context of an ensemble must be FP32C and share G, eps, the
    # Morton-order period and the stream; anything else is SG_EINVAL
    import ctypes as C
    import torch
    stream = torch.cuda.Stream()
    kw = dict(other)
    prec = sg.SG_FP64 if kw.pop("precision", None) == "fp64" else sg.SG_FP32C
    st2 = "new" if kw.pop("stream", None) else stream
    a = sg.Engine(states[0], precision=sg.SG_FP32C, stream=stream)
    b = sg.Engine(states[1], precision=prec, stream=st2, **kw)
    L = sg.lib()
    nbytes = L.sg_ensemble_bytes(2, a.n + b.n)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (ws.data_ptr() + 255) & ~255
    handles = (C.c_void_p * 2)(a.ctx.h.value, b.ctx.h.value)
    h = C.c_void_p()
    torch.cuda.synchronize()
    rc = L.sg_ensemble_create(handles, 2, C.c_void_p(ptr), nbytes, None, C.byref(h))
    assert rc == sg.SG_EINVAL and not h.value
    # the same two systems with matching contexts are accepted
    b_ok = sg.Engine(states[1], precision=sg.SG_FP32C, stream=stream)
    handles = (C.c_void_p * 2)(a.ctx.h.value, b_ok.ctx.h.value)
    assert L.sg_ensemble_create(handles, 2, C.c_void_p(ptr), nbytes, None,
                                C.byref(h)) == sg.SG_OK
    L.sg_ensemble_destroy(h)


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
        # the batched launch's automatic tile is 512 sources
        single = sg.Engine(st, precision=sg.SG_FP32C, grav_split=1, grav_ipl=2, grav_tile=512)
        for _ in range(4):
            single.ctx.step(dt, sg.SG_POT)
        single.ctx.sync()
        for f in ("x", "y", "z", "vx", "vy", "vz", "e", "ax", "pot"):
            a, b, c = e1.numpy(f), e2.numpy(f), single.numpy(f)
            np.testing.assert_array_equal(a, b, err_msg="graph " + f)
            np.testing.assert_array_equal(a, c, err_msg="single " + f)


def _small_state(rng, ng, nh):
    n = ng + nh
    pos = rng.normal(size=(n, 3))
    return {"ng": ng, "x": pos[:, 0].copy(), "y": pos[:, 1].copy(), "z": pos[:, 2].copy(),
            "vx": rng.normal(size=n) * 0.1, "vy": rng.normal(size=n) * 0.1,
            "vz": rng.normal(size=n) * 0.1, "m": rng.uniform(0.5, 1.5, n) / max(n, 1),
            "e": rng.uniform(0.02, 0.08, ng),
            "h": rng.uniform(0.1, 0.4, ng) * (1 + np.abs(pos[:ng, 0])) * (50.0 / max(ng, 50)) ** (1 / 3)}


def test_ensemble_edge_systems(sg):
    # systems at the edges of the segmented launches' block prefixes: one
    # gas particle and no halo, no gas at all, fewer gas particles than one
    # workgroup of any stage, and sizes that end mid-workgroup; steps of the
    # ensemble (eager and graph-captured) equal each system's own steps
    rng = np.random.default_rng(2024)
    sizes = [(1, 0), (0, 7), (33, 0), (257, 40), (2000, 500), (4097, 3)]
    states = [_small_state(rng, ng, nh) for ng, nh in sizes]
    dt = 1e-3
    eager = sg.Ensemble(states, grav_ipl=2)
    eager.run(dt, 3, sg.SG_POT, use_graph=False)
    graph = sg.Ensemble(states, grav_ipl=2)
    graph.run(dt, 3, sg.SG_POT, use_graph=True)
    for (ng, nh), st, e1, e2 in zip(sizes, states, eager.engines, graph.engines):
        single = sg.Engine(st, precision=sg.SG_FP32C, grav_split=1, grav_ipl=2, grav_tile=512)
        if ng > 0:
            single.build_neighbors()          # capacities for the initial state, as the ensemble
        for _ in range(3):
            single.ctx.step(dt, sg.SG_POT)
        single.ctx.sync()
        fields = ("x", "y", "z", "vx", "vy", "vz", "ax", "pot") + (("e", "rho") if ng else ())
        for f in fields:
            a, b, c = e1.numpy(f), e2.numpy(f), single.numpy(f)
            assert np.all(np.isfinite(a)), (ng, nh, f)
            np.testing.assert_array_equal(a, b, err_msg="graph %d/%d %s" % (ng, nh, f))
            np.testing.assert_array_equal(a, c, err_msg="single %d/%d %s" % (ng, nh, f))


def test_ensemble_reports_a_system_overflow(sg):
    # a system whose gas spreads far beyond what its grid capacity was sized
    # for latches SG_ECAPACITY in its own status word; the ensemble run
    # reports it with the system's index
    rng = np.random.default_rng(5)
    states = [_small_state(rng, 300, 10) for _ in range(3)]
    ens = sg.Ensemble(states, grav_ipl=2)
    eng = ens.engines[1]
    eng.dev["x"][:eng.ng] *= 10.0          # about 4.6e5 cells needed, 6496 sized
    eng.dev["y"][:eng.ng] *= 10.0
    with pytest.raises(sg.SGError) as ei:
        ens.run(1e-3, 1, sg.SG_POT, use_graph=False)
    assert ei.value.code == sg.SG_ECAPACITY
    assert ei.value.system == 1 and ei.value.need[0] > eng.caps.cell_cap


# ------------------------------------------------- full ensemble size --

@pytest.fixture(scope="module")
def c4():
    from paper_1807_08116_amd import ic
    return ic.ensemble()          # 64 systems, N log-uniform in [8192, 262144]: 4659360 particles


def test_c4_fullsize(sg, orc, c4):
    # the launch the ensemble benchmark tunes to (IPL 2, j-tile 512)
    ens = sg.Ensemble(c4, grav_ipl=2, grav_tile=512)
    ens.gravity(sg.SG_GRAV | sg.SG_POT)
    ens.torch.cuda.synchronize()
    ns = [len(s["x"]) for s in c4]
    print("c4: %d systems, %d particles" % (len(c4), sum(ns)), flush=True)
    rng = np.random.default_rng(7)
    for k in sorted({int(np.argmax(ns)), int(np.argmin(ns)), 17, 40}):
        st, eng = c4[k], ens.engines[k]
        single = sg.Engine(st, precision=sg.SG_FP32C, grav_split=1, grav_ipl=2, grav_tile=512)
        single.ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)
        single.ctx.sync()
        for f in ("ax", "ay", "az", "pot"):
            np.testing.assert_array_equal(eng.numpy(f), single.numpy(f), err_msg="%d %s" % (k, f))
        single.ctx.close()
        t = np.sort(rng.choice(ns[k], 256, replace=False))
        gx, gy, gz, gp = orc.gravity(st["x"], st["y"], st["z"], st["m"], 1.0, 0.01, t)
        ref = np.stack([gx, gy, gz], 1)
        got = np.stack([eng.numpy(f)[t] for f in ("ax", "ay", "az")], 1)
        e_acc = np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2))
        e_pot = np.sqrt(np.sum((eng.numpy("pot")[t] - gp) ** 2) / np.sum(gp ** 2))
        print("system %d N %d gravity err %.2e pot err %.2e" % (k, ns[k], e_acc, e_pot))
        assert e_acc < 1e-6 and e_pot < 1e-6
    # one whole ensemble step: every system's momentum is kept to the
    # rounding of its FP32 pair sums (forces are pairwise antisymmetric)
    p0 = [np.array([np.sum(s["m"] * s[f]) for f in ("vx", "vy", "vz")]) for s in c4]
    ens.run(1e-3, 1, sg.SG_POT, use_graph=False)
    for s, eng, q0 in zip(c4, ens.engines, p0):
        m = s["m"]
        scale = np.sum(m * np.sqrt(s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2))
        q1 = np.array([np.sum(m * eng.numpy(f)) for f in ("vx", "vy", "vz")])
        assert np.all(np.isfinite(q1))
        assert np.all(np.abs(q1 - q0) < 1e-7 * scale)
