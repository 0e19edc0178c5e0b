"""Python binding of libsphgrav.so: argument marshalling only.

Every step of the force evaluation runs in the HIP library; this module
loads it with ctypes, holds the device buffers (torch tensors on the GPU:
PyTorch is used only for device memory and the stream) and turns status
codes into exceptions.  Names follow the C ABI in ``include/sphgrav.h``.

There is no fallback: if the library is missing or no GPU is present the
calls fail loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphgrav.so")

SG_OK, SG_EINVAL, SG_ECAPACITY, SG_EDEVICE, SG_ESTATE, SG_ENONFINITE, SG_ERANGE = range(7)
SG_FP64, SG_FP32C = 0, 1
SG_SPH, SG_GRAV, SG_POT = 1, 2, 4
SG_PREDICT, SG_CORRECT = 0, 1
SG_MAX_LEVELS = 16
SG_STATIC_WS_BYTES = 64 << 20
(SG_X_KEYS, SG_X_COUNTS, SG_X_OFFSETS, SG_X_HMAX, SG_X_PERM, SG_X_NBR_OFF, SG_X_NBR_IDX,
 SG_X_GRID, SG_X_GORDER, SG_X_ACC_SPH, SG_X_ACC_GRAV) = range(11)

STATUS_NAMES = {0: "SG_OK", 1: "SG_EINVAL", 2: "SG_ECAPACITY", 3: "SG_EDEVICE", 4: "SG_ESTATE",
                5: "SG_ENONFINITE", 6: "SG_ERANGE"}

# Every entry point declared in include/sphgrav.h.
EXPORTED = ["sg_workspace_bytes", "sg_create", "sg_create_static", "sg_bind_state", "sg_build_neighbors",
            "sg_compute_density", "sg_compute_accel", "sg_kick_drift", "sg_step", "sg_run", "sg_cfl_dt", "sg_update_h",
            "sg_diagnostics", "sg_export", "sg_status_sync", "sg_profile_enable", "sg_profile_read",
            "sg_ensemble_bytes", "sg_ensemble_create", "sg_ensemble_gravity", "sg_ensemble_step",
            "sg_ensemble_run", "sg_ensemble_last_error", "sg_ensemble_destroy",
            "sg_last_error", "sg_destroy", "sg_version"]
STAGES = ["sort", "nbr", "density", "sph", "grav_prep", "grav", "update", "diag"]


class SGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("gamma", C.c_double),
                ("alpha", C.c_double), ("beta", C.c_double), ("eta", C.c_double),
                ("precision", C.c_int32), ("grav_ipl", C.c_int32), ("grav_split", C.c_int32),
                ("grav_variant", C.c_int32), ("grav_tile", C.c_int32),
                ("cell_scale_log2", C.c_int32), ("step_serial", C.c_int32),
                ("grav_reorder", C.c_int32)]


class Caps(C.Structure):
    _fields_ = [("n_gas_cap", C.c_int64), ("n_halo_cap", C.c_int64), ("cell_cap", C.c_int64),
                ("nnz_cap", C.c_int64)]


_STATE_FIELDS = ["x", "y", "z", "vx", "vy", "vz", "m", "h", "e", "ax", "ay", "az", "dedt",
                 "rho", "pot"]


class State(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in _STATE_FIELDS]


class GridInfo(C.Structure):
    _fields_ = [("L0", C.c_double), ("nlev", C.c_int32), ("pad", C.c_int32),
                ("L", C.c_double * SG_MAX_LEVELS), ("org", (C.c_double * 3) * SG_MAX_LEVELS),
                ("dim", (C.c_int64 * 3) * SG_MAX_LEVELS), ("base", C.c_int64 * SG_MAX_LEVELS),
                ("ncell", C.c_int64 * SG_MAX_LEVELS), ("npart", C.c_int64 * SG_MAX_LEVELS),
                ("hmax", C.c_double * SG_MAX_LEVELS), ("M", C.c_int64)]


_lib = None


def C_void(t):
    return C.c_void_p(t.data_ptr())


def lib():
    """Load libsphgrav.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsphgrav.so not built: run __graft_entry__.build() "
                          "(or python paper_1807_08116_amd/build.py)")
    # torch owns device memory and streams: bring its HIP runtime up first so
    # that the library binds to the runtime (and device list) torch uses.
    import torch
    torch.cuda.is_available()
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    L.sg_workspace_bytes.restype = C.c_size_t
    L.sg_workspace_bytes.argtypes = [C.POINTER(Params), C.POINTER(Caps)]
    L.sg_create.restype = C.c_int
    L.sg_create.argtypes = [C.POINTER(Params), C.POINTER(Caps), vp, C.c_size_t, vp, vp,
                            C.POINTER(vp)]
    L.sg_create_static.restype = C.c_int
    L.sg_create_static.argtypes = [C.POINTER(Params), C.POINTER(Caps), vp, C.POINTER(vp)]
    L.sg_bind_state.restype = C.c_int
    L.sg_bind_state.argtypes = [vp, i64, i64, C.POINTER(State)]
    for f in ("sg_build_neighbors", "sg_compute_density"):
        getattr(L, f).restype = C.c_int
        getattr(L, f).argtypes = [vp]
    L.sg_compute_accel.restype = C.c_int
    L.sg_compute_accel.argtypes = [vp, u32]
    L.sg_kick_drift.restype = C.c_int
    L.sg_kick_drift.argtypes = [vp, dbl, i32]
    L.sg_step.restype = C.c_int
    L.sg_step.argtypes = [vp, dbl, u32]
    L.sg_run.restype = C.c_int
    L.sg_run.argtypes = [vp, dbl, i64, u32, i32, vp]
    L.sg_cfl_dt.restype = C.c_int
    L.sg_cfl_dt.argtypes = [vp, dbl, vp]
    L.sg_update_h.restype = C.c_int
    L.sg_update_h.argtypes = [vp, dbl]
    L.sg_diagnostics.restype = C.c_int
    L.sg_diagnostics.argtypes = [vp, vp]
    L.sg_export.restype = C.c_int
    L.sg_export.argtypes = [vp, i32, vp, i64, C.POINTER(i64)]
    L.sg_status_sync.restype = C.c_int
    L.sg_status_sync.argtypes = [vp, C.POINTER(i64)]
    L.sg_profile_enable.restype = C.c_int
    L.sg_profile_enable.argtypes = [vp, i32]
    L.sg_profile_read.restype = C.c_int
    L.sg_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.sg_ensemble_bytes.restype = C.c_size_t
    L.sg_ensemble_bytes.argtypes = [i32, i64]
    L.sg_ensemble_create.restype = C.c_int
    L.sg_ensemble_create.argtypes = [C.POINTER(vp), i32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.sg_ensemble_gravity.restype = C.c_int
    L.sg_ensemble_gravity.argtypes = [vp, u32]
    L.sg_ensemble_step.restype = C.c_int
    L.sg_ensemble_step.argtypes = [vp, dbl, u32]
    L.sg_ensemble_run.restype = C.c_int
    L.sg_ensemble_run.argtypes = [vp, dbl, i64, u32, i32]
    L.sg_ensemble_last_error.restype = C.c_char_p
    L.sg_ensemble_last_error.argtypes = [vp]
    L.sg_ensemble_destroy.restype = None
    L.sg_ensemble_destroy.argtypes = [vp]
    L.sg_last_error.restype = C.c_char_p
    L.sg_last_error.argtypes = [vp]
    L.sg_destroy.restype = None
    L.sg_destroy.argtypes = [vp]
    L.sg_version.restype = C.c_char_p
    L.sg_version.argtypes = []
    _lib = L
    return L


def make_params(G=1.0, eps=0.01, gamma=5.0 / 3.0, alpha=1.0, beta=2.0, eta=0.1,
                precision=SG_FP64, grav_ipl=0, grav_split=0, grav_variant=0, grav_tile=0,
                cell_scale_log2=0, step_serial=0, grav_reorder=0):
    return Params(G, eps, gamma, alpha, beta, eta, precision, grav_ipl, grav_split, grav_variant,
                  grav_tile, cell_scale_log2, step_serial, grav_reorder)


def default_caps(n_gas, n_halo, cell_cap=None, nnz_cap=None):
    """Capacities with headroom for the smoothing-length grid and the lists."""
    if cell_cap is None:
        cell_cap = 8 * n_gas + 4096 if n_gas > 0 else 0
    if nnz_cap is None:
        nnz_cap = 96 * n_gas + 1024 if n_gas > 0 else 0
    return Caps(n_gas, n_halo, cell_cap, nnz_cap)


def workspace_bytes(params, caps):
    return lib().sg_workspace_bytes(C.byref(params), C.byref(caps))


def _torch_stream(torch, device, stream):
    if stream is None:
        return torch.cuda.current_stream(device)
    if stream == "new":
        # a stream of its own (default priority): needed for graph capture
        return torch.cuda.Stream(device=device)
    return stream


class Context:
    """One sg_ctx over a torch-allocated workspace on a torch stream (the
    current one by default), with a second torch stream for the gravity
    beside the neighbour/SPH chain of a step (aux_stream: "new" by default,
    None for none)."""

    def __init__(self, params: Params, caps: Caps, device="cuda", stream=None, aux_stream="new",
                 static=False):
        import torch
        self.torch = torch
        self.params = params
        self.caps = caps
        self.device = torch.device(device)
        L = lib()
        if static:
            # sg_create_static: the library's own workspace, no aux stream
            stream = _torch_stream(torch, self.device, stream)
            torch.cuda.synchronize(self.device)
            self.stream, self.aux_stream = stream, None
            h = C.c_void_p()
            with torch.cuda.device(self.device):
                rc = L.sg_create_static(C.byref(params), C.byref(caps),
                                        C.c_void_p(stream.cuda_stream), C.byref(h))
            if rc != SG_OK:
                raise SGError(rc, "sg_create_static failed: " + L.sg_last_error(None).decode())
            self.h = h
            self.state = None
            return
        nbytes = L.sg_workspace_bytes(C.byref(params), C.byref(caps))
        if nbytes == 0:
            raise SGError(SG_EINVAL, "invalid parameters or capacities")
        self.ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws_raw.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.ws_bytes = nbytes
        stream = _torch_stream(torch, self.device, stream)
        aux = None if aux_stream is None else _torch_stream(torch, self.device, aux_stream)
        torch.cuda.synchronize(self.device)     # state uploads on other streams are done
        self.stream = stream
        self.aux_stream = aux
        h = C.c_void_p()
        rc = L.sg_create(C.byref(params), C.byref(caps), C.c_void_p(self.ws_ptr),
                         C.c_size_t(nbytes), C.c_void_p(stream.cuda_stream),
                         C.c_void_p(aux.cuda_stream if aux is not None else None), C.byref(h))
        if rc != SG_OK:
            raise SGError(rc, "sg_create failed: " + L.sg_last_error(None).decode())
        self.h = h
        self.state = None

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().sg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != SG_OK:
            raise SGError(rc, "%s: %s" % (what, lib().sg_last_error(self.h).decode()))

    # -- entry points -------------------------------------------------------
    def bind_state(self, state: dict, n_gas: int, n_halo: int):
        """state: dict of float64 CUDA tensors (see sg_state); pot optional."""
        st = State()
        for f in _STATE_FIELDS:
            t = state.get(f)
            if t is not None:
                assert t.dtype == self.torch.float64 and t.is_cuda and t.is_contiguous(), f
            setattr(st, f, C.c_void_p(t.data_ptr()) if t is not None else None)
        self.state = state
        self.n_gas, self.n_halo = n_gas, n_halo
        self._check(lib().sg_bind_state(self.h, n_gas, n_halo, C.byref(st)), "sg_bind_state")

    def build_neighbors(self):
        self._check(lib().sg_build_neighbors(self.h), "sg_build_neighbors")

    def compute_density(self):
        self._check(lib().sg_compute_density(self.h), "sg_compute_density")

    def compute_accel(self, flags):
        self._check(lib().sg_compute_accel(self.h, flags), "sg_compute_accel")

    def kick_drift(self, dt, phase):
        self._check(lib().sg_kick_drift(self.h, float(dt), phase), "sg_kick_drift")

    def step(self, dt, flags=0):
        self._check(lib().sg_step(self.h, float(dt), flags), "sg_step")

    def run(self, dt, nsteps, flags=0, use_graph=True, hist=None):
        """nsteps steps (graph-replayed after the first when use_graph);
        returns the [nsteps, 10] device tensor of per-step diagnostics."""
        if hist is None:
            hist = self.torch.empty((max(nsteps, 1), 10), dtype=self.torch.float64,
                                    device=self.device)
        self._check(lib().sg_run(self.h, float(dt), int(nsteps), flags, 1 if use_graph else 0,
                                 C.c_void_p(hist.data_ptr())), "sg_run")
        self.sync()                 # sg_run has waited: report latched device conditions
        return hist

    def cfl_dt(self, C=0.5, out=None):
        """Eq. (dt-stability) time step at the current state (device tensor)."""
        if out is None:
            out = self.torch.empty(1, dtype=self.torch.float64, device=self.device)
        self._check(lib().sg_cfl_dt(self.h, float(C), C_void(out)), "sg_cfl_dt")
        return out

    def update_h(self, sigma):
        self._check(lib().sg_update_h(self.h, float(sigma)), "sg_update_h")

    def diagnostics(self, out=None):
        if out is None:
            out = self.torch.empty(10, dtype=self.torch.float64, device=self.device)
        self._check(lib().sg_diagnostics(self.h, C.c_void_p(out.data_ptr())), "sg_diagnostics")
        return out

    def profile_enable(self, on=True):
        self._check(lib().sg_profile_enable(self.h, 1 if on else 0), "sg_profile_enable")

    def profile_read(self):
        """{stage: (total ms, launches)} since the last profile_enable (syncs)."""
        ms = (C.c_double * len(STAGES))()
        cnt = (C.c_int64 * len(STAGES))()
        self._check(lib().sg_profile_read(self.h, ms, cnt), "sg_profile_read")
        return {name: (float(ms[k]), int(cnt[k])) for k, name in enumerate(STAGES)}

    def sync(self):
        """Wait for the stream; raise SGError (with .need) on a device-side error."""
        need = (C.c_int64 * 2)()
        rc = lib().sg_status_sync(self.h, need)
        if rc != SG_OK:
            e = SGError(rc, lib().sg_last_error(self.h).decode())
            e.need = (int(need[0]), int(need[1]))
            raise e

    _EXPORT_DTYPES = {SG_X_KEYS: "int32", SG_X_COUNTS: "int32", SG_X_OFFSETS: "int64",
                      SG_X_HMAX: "uint64", SG_X_PERM: "int32", SG_X_NBR_OFF: "int64",
                      SG_X_NBR_IDX: "int32", SG_X_GORDER: "int32", SG_X_ACC_SPH: "float64",
                      SG_X_ACC_GRAV: "float64"}

    def export(self, what):
        """Copy an internal array out (syncs the stream); returns a numpy array."""
        torch = self.torch
        if what == SG_X_GRID:
            info = GridInfo()
            n = C.c_int64()
            self._check(lib().sg_export(self.h, what, C.byref(info), C.sizeof(info), C.byref(n)),
                        "sg_export")
            return info
        dt = self._EXPORT_DTYPES[what]
        n = C.c_int64()
        cap = 16
        for _ in range(2):
            buf = torch.empty(max(cap, 1), dtype=torch.int64, device=self.device)
            rc = lib().sg_export(self.h, what, C.c_void_p(buf.data_ptr()), 8 * max(cap, 1),
                                 C.byref(n))
            if rc == SG_ECAPACITY:
                cap = int(n.value)
                continue
            self._check(rc, "sg_export")
            esz = 4 if dt == "int32" else 8
            raw = buf.cpu().numpy().view(np.uint8)[: esz * int(n.value)]
            arr = raw.view(np.dtype(dt))
            if what == SG_X_HMAX:
                arr = arr.view(np.float64)
            if what in (SG_X_ACC_SPH, SG_X_ACC_GRAV):
                arr = arr.reshape(3, -1)         # rows x, y, z
            return arr.copy()
        raise SGError(SG_ECAPACITY, "export size changed")


def grid_dict(info: GridInfo):
    nl = info.nlev
    return {
        "L0": info.L0, "nlev": nl, "M": info.M,
        "L": np.array(info.L[:nl]),
        "org": np.array([[info.org[l][d] for d in range(3)] for l in range(nl)]),
        "dim": np.array([[info.dim[l][d] for d in range(3)] for l in range(nl)], dtype=np.int64),
        "base": np.array(info.base[:nl], dtype=np.int64),
        "ncell": np.array(info.ncell[:nl], dtype=np.int64),
        "npart": np.array(info.npart[:nl], dtype=np.int64),
        "hmax": np.array(info.hmax[:nl]),
    }


def to_device(st: dict, device="cuda", with_pot=True):
    """SoA numpy state (gas first) -> dict of float64 device tensors + outputs."""
    import torch
    dev = torch.device(device)
    n = len(st["x"])
    ng = int(st["ng"])
    out = {}
    for f in ("x", "y", "z", "vx", "vy", "vz", "m"):
        out[f] = torch.tensor(np.ascontiguousarray(st[f], dtype=np.float64), device=dev)
    for f in ("h", "e"):
        a = np.ascontiguousarray(st[f], dtype=np.float64) if ng > 0 else np.zeros(1)
        out[f] = torch.tensor(a, device=dev)
    for f in ("ax", "ay", "az"):
        out[f] = torch.zeros(n, dtype=torch.float64, device=dev)
    out["dedt"] = torch.zeros(max(ng, 1), dtype=torch.float64, device=dev)
    out["rho"] = torch.zeros(max(ng, 1), dtype=torch.float64, device=dev)
    out["pot"] = torch.zeros(n, dtype=torch.float64, device=dev) if with_pot else None
    return out


class Engine:
    """Convenience owner of a context plus a bound state, with capacity retry."""

    def __init__(self, st: dict, precision=SG_FP64, device="cuda", params=None, caps=None,
                 with_pot=True, stream=None, aux_stream="new", static=False, **kw):
        self.ng = int(st["ng"])
        self.n = len(st["x"])
        self.nh = self.n - self.ng
        self.params = params if params is not None else make_params(precision=precision, **kw)
        self.caps = caps if caps is not None else default_caps(self.ng, self.nh)
        self.dev = to_device(st, device, with_pot=with_pot)
        self.device = device
        self.stream = stream
        self.aux_stream = aux_stream
        self.static = static
        self._make()

    def _make(self):
        self.ctx = Context(self.params, self.caps, self.device, stream=self.stream,
                           aux_stream=self.aux_stream, static=self.static)
        if self.stream == "new":
            self.stream = self.ctx.stream
        self.ctx.bind_state(self.dev, self.ng, self.nh)

    def grow(self, need):
        cells, nnz = need
        c = self.caps
        self.caps = Caps(c.n_gas_cap, c.n_halo_cap, max(c.cell_cap, int(cells * 1.25) + 1024),
                         max(c.nnz_cap, int(nnz * 1.25) + 1024))
        self.ctx.close()
        self._make()

    def build_neighbors(self, retry=True):
        for _ in range(3):
            self.ctx.build_neighbors()
            try:
                self.ctx.sync()
                return
            except SGError as e:
                if e.code != SG_ECAPACITY or not retry:
                    raise
                self.grow(e.need)
        raise SGError(SG_ECAPACITY, "could not size the workspace")

    def numpy(self, name):
        self.ctx.torch.cuda.synchronize()
        return self.dev[name].cpu().numpy()


class Ensemble:
    """Independent systems (one Engine each, FP32C, one shared stream) whose
    gravity runs as one persistent launch."""

    def __init__(self, states, device="cuda", chain_stream=None, **kw):
        import torch
        self.torch = torch
        dev = torch.device(device)
        self.stream = torch.cuda.Stream(device=dev)
        self.engines = [Engine(st, precision=SG_FP32C, device=device, stream=self.stream,
                               aux_stream=None, **kw) for st in states]
        # size each system's grid and list capacities for its initial state
        # (a build per system; the ensemble keeps the contexts' pointers, so
        # they cannot grow once it exists)
        for e in self.engines:
            if e.ng > 0:
                e.build_neighbors()
        total = sum(e.n for e in self.engines)
        L = lib()
        nbytes = L.sg_ensemble_bytes(len(self.engines), total)
        self.ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch.device(device))
        ptr = (self.ws_raw.data_ptr() + 255) & ~255
        handles = (C.c_void_p * len(self.engines))(*[e.ctx.h.value for e in self.engines])
        h = C.c_void_p()
        torch.cuda.synchronize()
        # chain_stream (the systems' corrector chains beside the batched
        # gravity): None = the library's CU-masked stream, "new" = a torch
        # stream, or a torch stream
        if chain_stream == "new":
            chain_stream = torch.cuda.Stream(device=dev)
        self.chain_stream = chain_stream
        gs = C.c_void_p(chain_stream.cuda_stream) if chain_stream is not None else None
        rc = L.sg_ensemble_create(handles, len(self.engines), C.c_void_p(ptr), nbytes, gs,
                                  C.byref(h))
        if rc != SG_OK:
            raise SGError(rc, "sg_ensemble_create failed")
        self.h = h

    def _check(self, rc, what):
        if rc != SG_OK:
            raise SGError(rc, "%s: %s" % (what, lib().sg_ensemble_last_error(self.h).decode()))

    def gravity(self, flags=SG_GRAV | SG_POT):
        self._check(lib().sg_ensemble_gravity(self.h, flags), "sg_ensemble_gravity")

    def step(self, dt, flags=0):
        self._check(lib().sg_ensemble_step(self.h, float(dt), flags), "sg_ensemble_step")

    def run(self, dt, nsteps, flags=0, use_graph=True):
        self._check(lib().sg_ensemble_run(self.h, float(dt), int(nsteps), flags,
                                          1 if use_graph else 0), "sg_ensemble_run")
        self.sync()

    def sync(self):
        """Wait for the stream and raise SGError (with .system, .need) for the
        first system whose device status word holds a condition."""
        for k, e in enumerate(self.engines):
            try:
                e.ctx.sync()
            except SGError as err:
                err.system = k
                raise

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().sg_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
