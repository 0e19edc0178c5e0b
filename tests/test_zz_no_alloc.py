"""The allocation-free context (sg_create_static: the library's own device
array as workspace) against a context over a caller-owned workspace
(sg_create), through the C ABI.  Both run the same kernels on the same
inputs, so every output must agree bit for bit (integer lists) and to the
same bits (FP64 sums in a fixed order): a full force evaluation and one
predictor-corrector step, on two calls in a row, the second with a smaller
input, in both precision forms."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

OUT = ("x", "y", "z", "vx", "vy", "vz", "e", "ax", "ay", "az", "dedt", "rho", "pot")


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


def _evaluate(sg, ctx, dev, st):
    """Force evaluation + one step on a bound context; host copies."""
    import torch
    ng, n = st["ng"], len(st["x"])
    ctx.bind_state(dev, ng, n - ng)
    ctx.build_neighbors()
    ctx.compute_density()
    ctx.compute_accel(sg.SG_SPH | sg.SG_GRAV | sg.SG_POT)
    ctx.sync()
    out = {"nbr_off": ctx.export(sg.SG_X_NBR_OFF), "nbr_idx": ctx.export(sg.SG_X_NBR_IDX),
           "perm": ctx.export(sg.SG_X_PERM)}
    torch.cuda.synchronize()
    out.update({"t0_" + f: dev[f].cpu().numpy()[: (ng if f in ("rho", "dedt") else n)].copy()
                for f in ("ax", "ay", "az", "rho", "dedt", "pot")})
    ctx.step(1e-3, sg.SG_POT)
    ctx.sync()
    torch.cuda.synchronize()
    for f in OUT:
        k = ng if f in ("e", "dedt", "rho") else n
        out[f] = dev[f].cpu().numpy()[:k].copy()
    return out


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_static_context_equals_workspace_context(sg, form):
    from paper_1807_08116_amd import ic
    p = sg.SG_FP32C if form == "fp32c" else sg.SG_FP64
    big = ic.make("c0")                    # 4096 gas + 4096 halo
    small = ic.make("c0", scale=0.375)     # 1536 gas + 1536 halo
    prm = sg.make_params(precision=p)
    caps = sg.default_caps(big["ng"], len(big["x"]) - big["ng"])
    assert sg.workspace_bytes(prm, caps) <= sg.SG_STATIC_WS_BYTES
    ref = sg.Context(prm, caps)                        # caller-owned workspace
    sta = sg.Context(prm, caps, static=True)           # the library's array
    try:
        for st in (big, small):                        # two calls, the second smaller
            print("static context", form, "N", len(st["x"]), flush=True)
            want = _evaluate(sg, ref, sg.to_device(st), st)
            got = _evaluate(sg, sta, sg.to_device(st), st)
            _same(got, want)
    finally:
        sta.close()
        ref.close()
    # a fresh static context on the freed slot, smaller capacities
    caps_s = sg.default_caps(small["ng"], len(small["x"]) - small["ng"])
    sta2 = sg.Context(prm, caps_s, static=True)
    ref2 = sg.Context(prm, caps_s)
    try:
        _same(_evaluate(sg, sta2, sg.to_device(small), small),
              _evaluate(sg, ref2, sg.to_device(small), small))
    finally:
        sta2.close()
        ref2.close()


def test_static_context_one_per_device(sg):
    prm = sg.make_params()
    caps = sg.default_caps(1000, 1000)
    a = sg.Context(prm, caps, static=True)
    try:
        with pytest.raises(sg.SGError) as ei:
            sg.Context(prm, caps, static=True)
        assert ei.value.code == sg.SG_ESTATE
    finally:
        a.close()
    b = sg.Context(prm, caps, static=True)     # the slot is free again
    b.close()
    # capacities beyond the array are refused before any device work
    L = sg.lib()
    h = C.c_void_p()
    big = sg.default_caps(100000, 100000)
    assert L.sg_create_static(C.byref(prm), C.byref(big), None, C.byref(h)) == sg.SG_ECAPACITY
    assert h.value is None
    assert b"exceeds the static array" in L.sg_last_error(None)
