"""Graph-captured steps (sg_run with use_graph) against eager steps.

The captured step replays the same kernels on the same buffers, so every
replay must reproduce the eager trajectory bit for bit, also when eager
work and synchronisations sit between graph runs.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "e", "ax", "dedt", "rho", "pot")


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
def c0():
    from paper_1807_08116_amd import ic
    return ic.make("c0", scale=0.5)


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_graph_steps_bitwise_equal_eager(sg, c0, form):
    p = sg.SG_FP64 if form == "fp64" else sg.SG_FP32C
    dt = 2e-3
    eager = sg.Engine(c0, precision=p, stream="new")
    h_e = eager.ctx.run(dt, 6, sg.SG_POT, use_graph=False).cpu().numpy()
    graph = sg.Engine(c0, precision=p, stream="new")
    h_g = graph.ctx.run(dt, 6, sg.SG_POT, use_graph=True).cpu().numpy()
    np.testing.assert_array_equal(h_g, h_e)
    for f in FIELDS:
        np.testing.assert_array_equal(graph.numpy(f), eager.numpy(f), err_msg=f)
    # energy bookkeeping is sane: total energy changes little over 6 steps
    assert abs(h_e[-1, 3] - h_e[0, 3]) < 1e-3 * abs(h_e[0, 3])


@pytest.fixture(scope="module")
def c0_full():
    from paper_1807_08116_amd import ic
    return ic.make("c0")


# Bounds of a graph-captured run of 6 steps against the oracle's
# predictor-corrector.  FP64: only summation order differs.  FP32C: the
# accelerations carry a normwise error of about 2e-7; over k steps of dt it
# moves velocities by about k dt |da| and positions by about k dt^2 |da|
# (measured on one MI355X: FP64 x 2.5e-18, v 3.9e-17, e 3.0e-17, E 1.4e-16;
# FP32C x 7.9e-13, v 2.9e-9, e 1.5e-9, E 3.3e-8).
GRAPH_ORACLE_TOL = {"fp64": {"x": 1e-12, "v": 1e-12, "e": 1e-12, "E": 1e-12},
                    "fp32c": {"x": 1e-10, "v": 3e-8, "e": 1e-8, "E": 1e-6}}


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_graph_steps_match_oracle(sg, orc, c0_full, form):
    # sg_run with a captured step (1 eager step + 5 replays) against the
    # oracle's predictor-corrector (Sec. 2.2) on the full 4096 + 4096
    # workload: positions, velocities, energies and the conserved sums.
    from paper_1807_08116_amd import ic
    prm = ic.DEFAULT_PARAMS
    p = sg.SG_FP64 if form == "fp64" else sg.SG_FP32C
    tol = GRAPH_ORACLE_TOL[form]
    dt, nsteps = 2e-3, 6
    eng = sg.Engine(c0_full, precision=p, stream="new")
    hist = eng.ctx.run(dt, nsteps, sg.SG_POT, use_graph=True).cpu().numpy()
    st, cache = c0_full, None
    for _ in range(nsteps):
        st, cache = orc.pc_step(st, prm, dt, cache)
    ng = st["ng"]

    def err(a, b):
        return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))

    ex = err(np.stack([eng.numpy(f) for f in ("x", "y", "z")]),
             np.stack([st[f] for f in ("x", "y", "z")]))
    ev = err(np.stack([eng.numpy(f) for f in ("vx", "vy", "vz")]),
             np.stack([st[f] for f in ("vx", "vy", "vz")]))
    ee = err(eng.numpy("e")[:ng], st["e"])
    d = orc.diagnostics(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"],
                        st["e"], cache["pot"], ng)
    eE = abs(hist[-1, 3] - d[3]) / abs(d[3])
    print(form, "graph run vs oracle after %d steps: x %.2e v %.2e e %.2e E %.2e"
          % (nsteps, ex, ev, ee, eE))
    assert ex < tol["x"] and ev < tol["v"] and ee < tol["e"] and eE < tol["E"]


def test_graph_replays_with_eager_work_between(sg, c0):
    dt = 2e-3
    ref = sg.Engine(c0, precision=sg.SG_FP64, stream="new")
    ref.ctx.run(dt, 8, sg.SG_POT, use_graph=False)
    eng = sg.Engine(c0, precision=sg.SG_FP64, stream="new")
    eng.ctx.run(dt, 3, sg.SG_POT, use_graph=True)
    eng.ctx.step(dt, sg.SG_POT)                       # eager step in between
    d = eng.ctx.diagnostics()
    eng.ctx.sync()
    assert np.all(np.isfinite(d.cpu().numpy()))
    eng.ctx.run(dt, 4, sg.SG_POT, use_graph=True)      # a fresh capture, replayed 3 times
    for f in FIELDS:
        np.testing.assert_array_equal(eng.numpy(f), ref.numpy(f), err_msg=f)


def test_graph_refuses_while_profiling(sg, c0):
    eng = sg.Engine(c0, precision=sg.SG_FP64, stream="new")
    eng.ctx.profile_enable(True)
    with pytest.raises(sg.SGError) as ei:
        eng.ctx.run(1e-3, 3, 0, use_graph=True)
    assert ei.value.code == sg.SG_ESTATE


def test_graph_refuses_the_null_stream(sg, c0):
    eng = sg.Engine(c0, precision=sg.SG_FP64)          # torch's current stream
    if eng.ctx.stream.cuda_stream != 0:
        pytest.skip("current stream is not the null stream")
    x0 = eng.numpy("x").copy()
    with pytest.raises(sg.SGError) as ei:
        eng.ctx.run(1e-3, 3, 0, use_graph=True)
    assert ei.value.code == sg.SG_EINVAL
    np.testing.assert_array_equal(eng.numpy("x"), x0)  # refused before any work
    eng.ctx.run(1e-3, 2, 0, use_graph=False)           # eager steps are fine there


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_checkpoint_resume_bitwise(sg, c0, form):
    # The state (r, v, e, h, m) is all a checkpoint needs: a fresh context
    # recomputes neighbours, density and gravity at r(t), which the running
    # context had cached from the previous corrector; all kernels are
    # deterministic, so the continued run matches bit for bit.
    p = sg.SG_FP64 if form == "fp64" else sg.SG_FP32C
    dt = 2e-3
    straight = sg.Engine(c0, precision=p)
    for _ in range(4):
        straight.ctx.step(dt, sg.SG_POT)
    first = sg.Engine(c0, precision=p)
    for _ in range(2):
        first.ctx.step(dt, sg.SG_POT)
    saved = {f: first.numpy(f).copy() for f in ("x", "y", "z", "vx", "vy", "vz", "m", "h", "e")}
    saved["ng"] = c0["ng"]
    saved["e"] = saved["e"][:c0["ng"]]
    saved["h"] = saved["h"][:c0["ng"]]
    resumed = sg.Engine(saved, precision=p)
    for _ in range(2):
        resumed.ctx.step(dt, sg.SG_POT)
    for f in ("x", "y", "z", "vx", "vy", "vz", "e", "ax", "pot"):
        np.testing.assert_array_equal(resumed.numpy(f), straight.numpy(f), err_msg=f)


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_overlapped_steps_equal_serial(sg, c0, form):
    # gravity beside the neighbour/SPH chain (default) and after it
    # (step_serial) give the same trajectory bit for bit, eager and captured
    p = sg.SG_FP32C if form == "fp32c" else sg.SG_FP64
    runs = []
    for serial in (0, 1):
        for graph in (False, True):
            eng = sg.Engine(c0, precision=p, step_serial=serial, stream="new")
            eng.ctx.run(1e-3, 4, sg.SG_POT, use_graph=graph)
            runs.append({f: eng.numpy(f) for f in FIELDS})
            eng.ctx.close()
    for r in runs[1:]:
        for f in FIELDS:
            np.testing.assert_array_equal(r[f], runs[0][f], err_msg=f)


def test_ensemble_overlapped_steps_equal_serial(sg):
    from paper_1807_08116_amd import ic
    states = ic.ensemble(nsys=4, scale=0.03)
    out = []
    for serial in (0, 1):
        ens = sg.Ensemble(states, step_serial=serial)
        ens.run(1e-3, 3, sg.SG_POT, use_graph=True)
        out.append([{f: e.numpy(f) for f in FIELDS} for e in ens.engines])
        ens.close()
    for a, b in zip(*out):
        for f in FIELDS:
            np.testing.assert_array_equal(a[f], b[f], err_msg=f)


# ------------------------------------------------ Morton-order period --

@pytest.mark.parametrize("form", ["fp32c", "fp64"])
def test_reorder_period_graph_equals_eager_and_stays_accurate(sg, orc, c0, form):
    # grav_reorder = 4: the Morton order is recomputed every 4th gravity
    # preparation (FP32C and the FP64 expanded kernel).  A captured chunk
    # holds 4 steps, so 1 eager + 2 chunks + 2 tail steps (9 steps) must
    # equal 9 eager steps bit for bit, and the gravity of one more step (in
    # the order recomputed two steps earlier) stays within the form's bound
    # of the oracle's.
    p = sg.SG_FP32C if form == "fp32c" else sg.SG_FP64
    tol = 1e-6 if form == "fp32c" else 1e-12
    dt = 2e-3
    eager = sg.Engine(c0, precision=p, grav_reorder=4, stream="new")
    h_e = eager.ctx.run(dt, 9, sg.SG_POT, use_graph=False).cpu().numpy()
    graph = sg.Engine(c0, precision=p, grav_reorder=4, stream="new")
    h_g = graph.ctx.run(dt, 9, sg.SG_POT, use_graph=True).cpu().numpy()
    np.testing.assert_array_equal(h_g, h_e)
    for f in FIELDS:
        np.testing.assert_array_equal(graph.numpy(f), eager.numpy(f), err_msg=f)
    # the step after the run reuses a stale order; gravity part vs oracle
    eager.ctx.step(dt, sg.SG_POT)
    eager.ctx.sync()
    x, y, z, m = (eager.numpy(f) for f in ("x", "y", "z", "m"))
    gx, gy, gz, _ = orc.gravity(x, y, z, m, 1.0, 0.01)
    ref = np.stack([gx, gy, gz], 1)
    got = eager.ctx.export(sg.SG_X_ACC_GRAV).T
    assert np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2)) < tol
    # a period of 1 (the default) recomputes every time: a different
    # trajectory only at rounding level
    fresh = sg.Engine(c0, precision=p, stream="new")
    fresh.ctx.run(dt, 9, sg.SG_POT, use_graph=False)
    for f in ("x", "vx"):
        a, b = graph.numpy(f), fresh.numpy(f)           # 9 steps each
        assert np.max(np.abs(a - b)) < 1e-5 * np.max(np.abs(b)), f


def test_reorder_period_ensemble_equals_single(sg):
    # ensembles follow each system's period: eager, captured (chunks of
    # 3 steps) and single-context runs agree bit for bit
    from paper_1807_08116_amd import ic
    states = ic.ensemble(nsys=4, scale=0.03)
    dt = 1e-3
    eager = sg.Ensemble(states, grav_reorder=3)
    eager.run(dt, 8, sg.SG_POT, use_graph=False)
    graph = sg.Ensemble(states, grav_reorder=3)
    graph.run(dt, 8, sg.SG_POT, use_graph=True)
    for st, e1, e2 in zip(states, eager.engines, graph.engines):
        single = sg.Engine(st, precision=sg.SG_FP32C, grav_split=1, grav_ipl=2, grav_tile=512,
                           grav_reorder=3)
        single.ctx.run(dt, 8, sg.SG_POT, use_graph=False)
        for f in FIELDS:
            a, b, c = e1.numpy(f), e2.numpy(f), single.numpy(f)
            np.testing.assert_array_equal(a, b, err_msg="graph " + f)
            np.testing.assert_array_equal(a, c, err_msg="single " + f)
