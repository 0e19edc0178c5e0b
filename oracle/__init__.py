"""CPU FP64 oracle for the SPH + direct-gravity force evaluation.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product path.  It
shares no code with the HIP library (``paper_1807_08116_amd``) and does not
import it.

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP over particles);
this module only marshals arrays and strings the C steps together in the
order of the paper's predictor-corrector scheme (Sec. 2.2, Eqs. v-predictor to
e-corrector, and the kernel sequence of Sec. 3).  Candidate neighbour pairs
for large inputs come from scipy's k-d tree (a library primitive); the exact
neighbour test is always the C predicate.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

MAX_LEVELS = 16


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2 -fopenmp, no contraction)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Grid(C.Structure):
    _fields_ = [
        ("L0", C.c_double),
        ("nlev", C.c_int32),
        ("pad", C.c_int32),
        ("L", C.c_double * MAX_LEVELS),
        ("org", (C.c_double * 3) * MAX_LEVELS),
        ("dim", (C.c_int64 * 3) * MAX_LEVELS),
        ("base", C.c_int64 * MAX_LEVELS),
        ("ncell", C.c_int64 * MAX_LEVELS),
        ("npart", C.c_int64 * MAX_LEVELS),
        ("hmax", C.c_double * MAX_LEVELS),
        ("M", C.c_int64),
    ]


_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64 = C.c_int64
_dbl = C.c_double


def _opt(t):
    """ndpointer that also accepts None."""
    class _P(t):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return t.from_param(obj)
    return _P


def lib():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.or_W.restype = _dbl
        L.or_W.argtypes = [_dbl, _dbl]
        L.or_Wp.restype = _dbl
        L.or_Wp.argtypes = [_dbl, _dbl]
        L.or_dWp_dxi.restype = _dbl
        L.or_dWp_dxi.argtypes = [_dbl, _dbl]
        L.or_pred.restype = C.c_int
        L.or_pred.argtypes = [_dbl] * 8
        L.or_grid.restype = C.c_int
        L.or_grid.argtypes = [_i64, _D, _D, _D, _D, C.c_int, C.POINTER(Grid)]
        L.or_keys.restype = None
        L.or_keys.argtypes = [_i64, _D, _D, _D, _D, C.POINTER(Grid), _I32, _opt(_I32)]
        L.or_count_sort.restype = None
        L.or_count_sort.argtypes = [_i64, _i64, _I32, _D, _I32, _I64, _D, _I32]
        L.or_nbrs_brute.restype = None
        L.or_nbrs_brute.argtypes = [_i64, _D, _D, _D, _D, _I64, _opt(_I32)]
        L.or_nbr_row_brute.restype = _i64
        L.or_nbr_row_brute.argtypes = [_i64, _D, _D, _D, _D, _i64, _I32, _i64]
        L.or_nbrs_from_candidates.restype = None
        L.or_nbrs_from_candidates.argtypes = [_i64, _D, _D, _D, _D, _I64, _I32, _I64, _opt(_I32)]
        L.or_rows_to_slots.restype = None
        L.or_rows_to_slots.argtypes = [_i64, _I32, _I64, _I32, _I64, _I32]
        L.or_density.restype = None
        L.or_density.argtypes = [_i64, _D, _D, _D, _D, _D, _I64, _I32, _D]
        L.or_eos.restype = None
        L.or_eos.argtypes = [_i64, _dbl, _D, _D, _D, _D]
        L.or_sph_force.restype = None
        L.or_sph_force.argtypes = [_i64] + [_D] * 10 + [_dbl] * 4 + [_I64, _I32] + [_D] * 4
        L.or_gravity.restype = None
        L.or_gravity.argtypes = [_i64, _D, _D, _D, _D, _dbl, _dbl, _i64, _I64, _D, _D, _D, _opt(_D)]
        L.or_predict.restype = None
        L.or_predict.argtypes = [_i64, _i64, _dbl] + [_D] * 15
        L.or_correct.restype = None
        L.or_correct.argtypes = [_i64, _i64, _dbl] + [_D] * 12
        L.or_diagnostics.restype = None
        L.or_diagnostics.argtypes = [_i64, _i64] + [_D] * 8 + [_opt(_D), _D]
        L.or_cfl_dt.restype = _dbl
        L.or_cfl_dt.argtypes = [_i64] + [_D] * 12 + [_dbl] * 4 + [_I64, _I32]
        L.or_update_h.restype = None
        L.or_update_h.argtypes = [_i64, _dbl, _D, _D, _D]
        L.or_max_levels.restype = C.c_int
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        L.or_grid_size.restype = C.c_size_t
        assert L.or_max_levels() == MAX_LEVELS
        assert L.or_grid_size() == C.sizeof(Grid), "Grid struct layout mismatch"
        _lib = L
        return _lib


def _c(a, dt=np.float64):
    return np.ascontiguousarray(a, dtype=dt)


# --------------------------------------------------------------------------
# Kernels and predicate (scalar, for pins)
# --------------------------------------------------------------------------

def W(r, h):
    return lib().or_W(float(r), float(h))


def Wp(r, h):
    return lib().or_Wp(float(r), float(h))


def dWp_dxi(r, h):
    return lib().or_dWp_dxi(float(r), float(h))


def pred(pi, hi, pj, hj):
    return bool(lib().or_pred(float(pi[0]), float(pi[1]), float(pi[2]), float(hi),
                              float(pj[0]), float(pj[1]), float(pj[2]), float(hj)))


# --------------------------------------------------------------------------
# Grid, keys, counting sort
# --------------------------------------------------------------------------

def set_threads(n):
    """Threads of the oracle's OpenMP loops."""
    lib().or_set_threads(int(n))


def get_threads():
    return int(lib().or_get_threads())


def grid(x, y, z, h, cell_scale_log2=0):
    g = Grid()
    rc = lib().or_grid(len(x), _c(x), _c(y), _c(z), _c(h), int(cell_scale_log2), C.byref(g))
    if rc != 0:
        raise ValueError("oracle grid error %d" % rc)
    return g


def grid_dict(g: Grid):
    nl = g.nlev
    return {
        "L0": g.L0, "nlev": nl, "M": g.M,
        "L": np.array(g.L[:nl]),
        "org": np.array([[g.org[l][d] for d in range(3)] for l in range(nl)]),
        "dim": np.array([[g.dim[l][d] for d in range(3)] for l in range(nl)], dtype=np.int64),
        "base": np.array(g.base[:nl], dtype=np.int64),
        "ncell": np.array(g.ncell[:nl], dtype=np.int64),
        "npart": np.array(g.npart[:nl], dtype=np.int64),
        "hmax": np.array(g.hmax[:nl]),
    }


def keys(x, y, z, h, g: Grid):
    n = len(x)
    key = np.empty(n, np.int32)
    lev = np.empty(n, np.int32)
    lib().or_keys(n, _c(x), _c(y), _c(z), _c(h), C.byref(g), key, lev)
    return key, lev


def count_sort(key, h, M):
    n = len(key)
    count = np.empty(M, np.int32)
    off = np.empty(M + 1, np.int64)
    hmax = np.empty(M, np.float64)
    perm = np.empty(n, np.int32)
    lib().or_count_sort(n, M, _c(key, np.int32), _c(h), count, off, hmax, perm)
    return count, off, hmax, perm


def sort_gas(x, y, z, h, cell_scale_log2=0):
    """Grid, keys, counts, offsets, hmax and stable permutation of the gas."""
    g = grid(x, y, z, h, cell_scale_log2)
    key, lev = keys(x, y, z, h, g)
    count, off, hmax, perm = count_sort(key, h, g.M)
    return {"grid": g, "key": key, "level": lev, "count": count, "off": off,
            "hmax": hmax, "perm": perm}


# --------------------------------------------------------------------------
# Neighbour lists
# --------------------------------------------------------------------------

def nbrs_brute(x, y, z, h):
    n = len(x)
    x, y, z, h = _c(x), _c(y), _c(z), _c(h)
    off = np.zeros(n + 1, np.int64)
    lib().or_nbrs_brute(n, x, y, z, h, off, None)
    idx = np.empty(int(off[-1]), np.int32)
    lib().or_nbrs_brute(n, x, y, z, h, off, idx)
    return off, idx


def nbr_row_brute(x, y, z, h, i):
    n = len(x)
    cap = 4096
    while True:
        out = np.empty(cap, np.int32)
        c = lib().or_nbr_row_brute(n, _c(x), _c(y), _c(z), _c(h), int(i), out, cap)
        if c <= cap:
            return out[:c].copy()
        cap = int(c)


def kdtree_workers():
    """Threads of the k-d tree queries: the OpenMP thread count the oracle's C
    code uses (OMP_NUM_THREADS, else all CPUs this process may run on)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    if hasattr(os, "sched_getaffinity"):
        return max(1, len(os.sched_getaffinity(0)))
    return os.cpu_count() or 1


def nbrs_kdtree(x, y, z, h, workers=None):
    """Exact rows via k-d tree candidates (radius 2 h_i (1 + 2^-10)) + C filter."""
    from scipy.spatial import cKDTree
    n = len(x)
    x, y, z, h = _c(x), _c(y), _c(z), _c(h)
    pts = np.stack([x, y, z], axis=1)
    tree = cKDTree(pts)
    w = workers if workers is not None else kdtree_workers()
    lists = tree.query_ball_point(pts, r=2.0 * h * (1.0 + 2.0 ** -10), workers=w,
                                  return_sorted=False)
    lens = np.fromiter((len(a) for a in lists), dtype=np.int64, count=n)
    coff = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=coff[1:])
    cidx = np.fromiter((j for a in lists for j in a), dtype=np.int32, count=int(coff[-1])) \
        if n < 200000 else np.concatenate([np.asarray(a, np.int32) for a in lists])
    del lists
    off = np.zeros(n + 1, np.int64)
    lib().or_nbrs_from_candidates(n, x, y, z, h, coff, cidx, off, None)
    idx = np.empty(int(off[-1]), np.int32)
    lib().or_nbrs_from_candidates(n, x, y, z, h, coff, cidx, off, idx)
    return off, idx


def nbrs(x, y, z, h, workers=None):
    """Exact id-space neighbour rows; brute force for small inputs."""
    if len(x) <= 20000:
        return nbrs_brute(x, y, z, h)
    return nbrs_kdtree(x, y, z, h, workers)


def rows_to_slots(perm, off, idx):
    n = len(perm)
    lens = np.diff(off)[perm]
    soff = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=soff[1:])
    sidx = np.empty(int(soff[-1]), np.int32)
    lib().or_rows_to_slots(n, _c(perm, np.int32), _c(off, np.int64), _c(idx, np.int32), soff, sidx)
    return soff, sidx


# --------------------------------------------------------------------------
# SPH and gravity
# --------------------------------------------------------------------------

def density(x, y, z, m, h, off, idx):
    n = len(x)
    rho = np.empty(n)
    lib().or_density(n, _c(x), _c(y), _c(z), _c(m), _c(h), _c(off, np.int64), _c(idx, np.int32), rho)
    return rho


def eos(rho, e, gamma):
    n = len(rho)
    p = np.empty(n)
    c = np.empty(n)
    lib().or_eos(n, float(gamma), _c(rho), _c(e), p, c)
    return p, c


def sph_force(x, y, z, vx, vy, vz, m, h, rho, e, gamma, alpha, beta, eta, off, idx):
    n = len(x)
    ax, ay, az, de = (np.empty(n) for _ in range(4))
    lib().or_sph_force(n, _c(x), _c(y), _c(z), _c(vx), _c(vy), _c(vz), _c(m), _c(h),
                       _c(rho), _c(e), float(gamma), float(alpha), float(beta), float(eta),
                       _c(off, np.int64), _c(idx, np.int32), ax, ay, az, de)
    return ax, ay, az, de


def gravity(x, y, z, m, G, eps, targets=None, with_pot=True):
    n = len(x)
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = _c(targets, np.int64)
    nt = len(targets)
    ax, ay, az = np.empty(nt), np.empty(nt), np.empty(nt)
    pot = np.empty(nt) if with_pot else None
    lib().or_gravity(n, _c(x), _c(y), _c(z), _c(m), float(G), float(eps), nt, targets,
                     ax, ay, az, pot)
    return ax, ay, az, pot


def diagnostics(x, y, z, vx, vy, vz, m, e, pot, ng):
    n = len(x)
    out = np.empty(10)
    lib().or_diagnostics(n, int(ng), _c(x), _c(y), _c(z), _c(vx), _c(vy), _c(vz), _c(m),
                         _c(e) if ng > 0 else np.zeros(1), None if pot is None else _c(pot), out)
    return out


def cfl_dt(x, y, z, vx, vy, vz, h, c, qx, qy, qz, E, C, alpha, beta, eta, off, idx):
    """Eq. (dt-stability) over the gas rows (see or_cfl_dt)."""
    n = len(x)
    return lib().or_cfl_dt(n, _c(x), _c(y), _c(z), _c(vx), _c(vy), _c(vz), _c(h), _c(c),
                           _c(qx), _c(qy), _c(qz), _c(E), float(C), float(alpha), float(beta),
                           float(eta), _c(off, np.int64), _c(idx, np.int32))


def update_h(m, rho, sigma):
    n = len(m)
    h = np.empty(n)
    lib().or_update_h(n, float(sigma), _c(m), _c(rho), h)
    return h


# --------------------------------------------------------------------------
# Whole force evaluation and predictor-corrector step
# --------------------------------------------------------------------------

def forces(st, prm, vel=None, ener=None, grav_targets=None, nb=None, rho=None):
    """Force evaluation at the positions in ``st``.

    st: dict with x,y,z,vx,vy,vz,m [N] and h,e [N_g], and ``ng``.
    prm: dict with G, eps, gamma, alpha, beta, eta.
    vel/ener: optional (vx,vy,vz) / e used by the SPH force instead of st's.
    Returns a dict with rho [N_g], the SPH part (asx.., dedt) [N_g], gravity
    gx.. (and pot) on grav_targets (all N by default), and the neighbour rows.
    """
    ng = int(st["ng"])
    x, y, z = st["x"], st["y"], st["z"]
    gx_ = slice(0, ng)
    if nb is None and ng > 0:
        nb = nbrs(x[gx_], y[gx_], z[gx_], st["h"])
    out = {"nb": nb}
    if ng > 0:
        if rho is None:
            rho = density(x[gx_], y[gx_], z[gx_], st["m"][gx_], st["h"], nb[0], nb[1])
        vx, vy, vz = vel if vel is not None else (st["vx"], st["vy"], st["vz"])
        e = ener if ener is not None else st["e"]
        asx, asy, asz, de = sph_force(x[gx_], y[gx_], z[gx_], vx[gx_], vy[gx_], vz[gx_],
                                      st["m"][gx_], st["h"], rho, e, prm["gamma"],
                                      prm["alpha"], prm["beta"], prm["eta"], nb[0], nb[1])
        out.update(rho=rho, asx=asx, asy=asy, asz=asz, dedt=de)
    if grav_targets is not False:
        gx, gy, gz, pot = gravity(x, y, z, st["m"], prm["G"], prm["eps"], grav_targets)
        out.update(gx=gx, gy=gy, gz=gz, pot=pot)
    return out


def total_accel(st, f):
    """a = a_SPH + g for gas, g for halo (Eq. dv_dt-SPH); all N particles."""
    ng = int(st["ng"])
    ax, ay, az = f["gx"].copy(), f["gy"].copy(), f["gz"].copy()
    if ng > 0:
        ax[:ng] += f["asx"]
        ay[:ng] += f["asy"]
        az[:ng] += f["asz"]
    return ax, ay, az


def pc_step(st, prm, dt, cache=None):
    """One predictor-corrector step (Sec. 2.2 steps I-III; Sec. 3 sequence).

    ``cache`` holds the force evaluation at the current positions with the
    current velocities (gravity is computed once per step and reused by the
    next predictor, Sec. 2.2).  Returns (new_state, new_cache).
    """
    ng = int(st["ng"])
    n = len(st["x"])
    st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    if cache is None:
        cache = forces(st, prm)
    else:
        # predictor right-hand side: SPH at (r(t), v(t), e(t)) on the rows and
        # density already built at r(t); gravity reused from the last step.
        f = forces(st, prm, nb=cache["nb"], rho=cache.get("rho"), grav_targets=False)
        f.update({k: cache[k] for k in ("gx", "gy", "gz", "pot")})
        cache = f
    qx, qy, qz = total_accel(st, cache)
    E = cache["dedt"] if ng > 0 else np.zeros(0)
    vtx, vty, vtz = np.empty(n), np.empty(n), np.empty(n)
    et = np.empty(ng)
    e = st["e"] if ng > 0 else np.zeros(1)
    lib().or_predict(n, ng, float(dt), st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"],
                     _c(e), qx, qy, qz, _c(E) if ng > 0 else np.zeros(1), vtx, vty, vtz,
                     et if ng > 0 else np.zeros(1))
    f2 = forces(st, prm, vel=(vtx, vty, vtz), ener=et if ng > 0 else None)
    qx2, qy2, qz2 = total_accel(st, f2)
    E2 = f2["dedt"] if ng > 0 else np.zeros(1)
    ee = st["e"] if ng > 0 else np.zeros(1)
    lib().or_correct(n, ng, float(dt), st["vx"], st["vy"], st["vz"], ee, vtx, vty, vtz,
                     et if ng > 0 else np.zeros(1), qx2, qy2, qz2, _c(E2))
    if ng > 0:
        st["e"] = ee
    return st, f2
