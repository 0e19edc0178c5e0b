"""Seeded synthetic initial conditions (inputs only; none of the method's arithmetic).

The paper's experiments collide two galaxies, each with N_g/2 gas (SPH)
particles and N_h/2 collisionless dark-halo particles (Sec. 2.1), built from a
quasi-isothermal halo and a King bulge whose parameters are not given in the
paper.  These generators stand in for them with Plummer spheres of the same
particle counts:

* gas: Plummer scale a = 1, total mass 0.1; halo: a = 3, mass 0.9 (G = 1);
* each component truncated at 5a and sampled by inverting the Plummer
  cumulative mass profile X(r) = r^3 / (r^2 + a^2)^{3/2} (Aarseth, Henon &
  Wielen 1974); equal particle masses that add up exactly to the component
  mass;
* velocities: each Cartesian component drawn from N(0, 0.1^2);
* gas specific internal energy 0.05;
* smoothing lengths found by bisection so that each gas particle has 32..64
  other gas particles within 2 h_i (k-d tree distances);
* a collision places system A at (-5, -b/2, 0) and B at (+5, +b/2, 0),
  moving towards each other along x with the given closing speed.

Particles are ordered gas first: [gas A, gas B, halo A, halo B].
All randomness comes from numpy's PCG64 generator seeded by the caller.
"""
from __future__ import annotations

import os

import numpy as np

SEED_BASE = 1807081160

DEFAULT_PARAMS = dict(G=1.0, eps=0.01, gamma=5.0 / 3.0, alpha=1.0, beta=2.0, eta=0.1)


def plummer(n, a, mass, rng, trunc=5.0):
    """n positions of a Plummer sphere of scale a truncated at trunc*a."""
    rt = trunc * a
    Xt = rt ** 3 / (rt * rt + a * a) ** 1.5
    X = Xt * (1.0 - rng.random(n))          # in (0, Xt]
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    u = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - u * u)
    pos = np.stack([r * s * np.cos(phi), r * s * np.sin(phi), r * u], axis=1)
    m = np.full(n, mass / n)
    return pos, m


def _workers():
    """OMP_NUM_THREADS when set (the CPU share of the process), else the CPUs
    this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, len(os.sched_getaffinity(0))) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def smoothing_lengths(pos, nmin=32, nmax=64, workers=None):
    """Bisection on h_i until #{j != i : |r_ij| < 2 h_i} lies in [nmin, nmax]."""
    from scipy.spatial import cKDTree
    n = len(pos)
    k = min(nmax + 2, n)                      # self + up to nmax + 1 others
    w = workers if workers is not None else _workers()
    d, _ = cKDTree(pos).query(pos, k=k, workers=w)
    d = d[:, 1:]                              # drop self
    lo = np.zeros(n)
    hi = 0.5 * d[:, -1]                       # count(hi) <= k-2 <= nmax
    h = np.empty(n)
    done = np.zeros(n, bool)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        cnt = (d < 2.0 * mid[:, None]).sum(axis=1)
        ok = (cnt >= nmin) & (cnt <= nmax) & ~done
        h[ok] = mid[ok]
        done |= ok
        if done.all():
            break
        low = cnt < nmin
        lo = np.where(~done & low, mid, lo)
        hi = np.where(~done & ~low, mid, hi)
    if not done.all():
        raise RuntimeError("smoothing-length bisection did not converge")
    return h


def galaxy(n_gas, n_halo, rng, gas_a=1.0, gas_m=0.1, halo_a=3.0, halo_m=0.9,
           sigma=0.1, e0=0.05):
    gp, gm = plummer(n_gas, gas_a, gas_m, rng)
    hp, hm = plummer(n_halo, halo_a, halo_m, rng)
    gv = rng.normal(0.0, sigma, (n_gas, 3))
    hv = rng.normal(0.0, sigma, (n_halo, 3))
    return dict(gp=gp, gm=gm, gv=gv, ge=np.full(n_gas, e0), hp=hp, hm=hm, hv=hv)


def assemble(systems, offsets, velocities, with_h=True):
    """Concatenate systems gas first; return the SoA state dict."""
    gp = np.concatenate([s["gp"] + o for s, o in zip(systems, offsets)])
    gv = np.concatenate([s["gv"] + v for s, v in zip(systems, velocities)])
    gm = np.concatenate([s["gm"] for s in systems])
    ge = np.concatenate([s["ge"] for s in systems])
    hp = np.concatenate([s["hp"] + o for s, o in zip(systems, offsets)])
    hv = np.concatenate([s["hv"] + v for s, v in zip(systems, velocities)])
    hm = np.concatenate([s["hm"] for s in systems])
    pos = np.concatenate([gp, hp])
    vel = np.concatenate([gv, hv])
    st = {
        "ng": len(gp),
        "x": np.ascontiguousarray(pos[:, 0]), "y": np.ascontiguousarray(pos[:, 1]),
        "z": np.ascontiguousarray(pos[:, 2]),
        "vx": np.ascontiguousarray(vel[:, 0]), "vy": np.ascontiguousarray(vel[:, 1]),
        "vz": np.ascontiguousarray(vel[:, 2]),
        "m": np.concatenate([gm, hm]),
        "e": ge.copy(),
    }
    st["h"] = smoothing_lengths(gp) if (with_h and len(gp) > 0) else np.zeros(len(gp))
    return st


def isolated(n_gas, n_halo, seed):
    """One Plummer gas sphere + halo at rest at the origin."""
    rng = np.random.default_rng(seed)
    g = galaxy(n_gas, n_halo, rng)
    return assemble([g], [np.zeros(3)], [np.zeros(3)])


def collision(n_gas_per, n_halo_per, seed, b=0.5, v=1.0, sep=10.0, mass_ratio=1.0):
    """Two systems on a collision course (head-on up to impact parameter b).

    With mass_ratio q != 1 system A holds q times the particles (and mass) of
    system B at equal particle mass; velocities keep the total momentum zero.
    """
    rng = np.random.default_rng(seed)
    if mass_ratio == 1.0:
        na_g, nb_g, na_h, nb_h = n_gas_per, n_gas_per, n_halo_per, n_halo_per
        fa = fb = 1.0
    else:
        tot_g, tot_h = 2 * n_gas_per, 2 * n_halo_per
        na_g = int(round(tot_g * mass_ratio / (1.0 + mass_ratio)))
        na_h = int(round(tot_h * mass_ratio / (1.0 + mass_ratio)))
        nb_g, nb_h = tot_g - na_g, tot_h - na_h
        fa, fb = na_g / n_gas_per, nb_g / n_gas_per
    A = galaxy(na_g, na_h, rng, gas_m=0.1 * fa, halo_m=0.9 * fa)
    B = galaxy(nb_g, nb_h, rng, gas_m=0.1 * fb, halo_m=0.9 * fb)
    va = v * fb / (fa + fb)
    vb = v * fa / (fa + fb)
    return assemble([A, B],
                    [np.array([-0.5 * sep, -0.5 * b, 0.0]), np.array([0.5 * sep, 0.5 * b, 0.0])],
                    [np.array([va, 0.0, 0.0]), np.array([-vb, 0.0, 0.0])])


# Workloads of the paper's shape: c0 isolated system; c1, c2 head-on
# collisions at 262144 and 2097152 particles; c3 off-axis 3:1 collision at
# 4194304 particles.
CONFIGS = {
    "c0": dict(kind="isolated", n_gas=4096, n_halo=4096),
    "c1": dict(kind="collision", n_gas_per=65536, n_halo_per=65536, b=0.5, v=1.0),
    "c2": dict(kind="collision", n_gas_per=524288, n_halo_per=524288, b=0.5, v=1.0),
    "c3": dict(kind="collision", n_gas_per=1048576, n_halo_per=1048576, b=2.0, v=1.0,
               mass_ratio=3.0),
}


def make(name, seed=None, scale=1.0):
    """State for a named workload; scale < 1 shrinks the particle counts."""
    cfg = CONFIGS[name]
    idx = int(name[1:])
    seed = SEED_BASE + idx if seed is None else seed
    if cfg["kind"] == "isolated":
        return isolated(max(1, int(cfg["n_gas"] * scale)), max(1, int(cfg["n_halo"] * scale)), seed)
    return collision(max(1, int(cfg["n_gas_per"] * scale)), max(1, int(cfg["n_halo_per"] * scale)),
                     seed, b=cfg["b"], v=cfg["v"], mass_ratio=cfg.get("mass_ratio", 1.0))


def ensemble(nsys=64, seed=SEED_BASE + 4, n_min=8192, n_max=262144, scale=1.0):
    """Independent two-system collisions: N per system log-uniform in
    [n_min, n_max] (a multiple of 4, gas:halo 1:1, two galaxies each), impact
    parameter U[0, 3], closing speed U[0.5, 2].  Returns a list of states."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(nsys):
        n = int(np.exp(rng.uniform(np.log(n_min), np.log(n_max))) * scale)
        n = max(8, n - n % 4)
        b = rng.uniform(0.0, 3.0)
        v = rng.uniform(0.5, 2.0)
        sub = int(rng.integers(0, 2 ** 31))
        st = collision(n // 4, n // 4, sub, b=b, v=v)
        st["meta"] = {"n": n, "b": b, "v": v, "seed": sub}
        out.append(st)
    return out
