"""Autotuner for the launch parameters of the force evaluation.

Tuned knobs (none changes results beyond summation order; the parity tests
cover every value):

* gravity: targets per lane (a workgroup of 256 lanes owns 256 * ipl
  targets: the "block" of targets), sources per LDS tile (the j-tile: 128,
  256 or 512), source-range splits and, in the FP64 form, the kernel
  variant (difference or expanded far field, FP32- or FP64-seeded rsqrt);
* neighbour grid: the cell size, as a power-of-two scale of the default
  rule (cell_scale_log2 in {-1, 0, 1});
* ensembles: targets per lane and j-tile of the persistent launch.

Each candidate is timed on the caller's particle set with the library's own
stage timing (HIP events around the kernels).  The gravity search is a
coordinate search (targets per lane, then tile, then splits, then variant),
each step keeping the best value so far.  Results are cached in a JSON file
keyed by what was tuned, the precision form and the particle count rounded
up to a power of two.

Usage: python -m paper_1807_08116_amd.autotune [--config c2] [--scale 1.0]
           [--forms fp32c,fp64] [--reps 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
IPLS = (1, 2, 4)
TILES = (128, 256, 512)
CELL_SCALES = (-1, 0, 1)


def _fill_split(n, ipl):
    """Splits that give about 8192 workgroups (the library's automatic rule)."""
    blocks = max(1, (n + 256 * ipl - 1) // (256 * ipl))
    return max(1, min(64, (8192 + blocks - 1) // blocks))


def candidates(precision, n):
    """Every gravity parameter set the search may visit (for validation)."""
    from . import sphgrav as sg
    out = []
    variants = (1, 2, 3, 4) if precision == sg.SG_FP64 else (0,)
    for ipl in IPLS:
        for tile in TILES:
            for split in sorted({1, 2, 4, _fill_split(n, ipl)}):
                for v in variants:
                    out.append(dict(grav_ipl=ipl, grav_tile=tile, grav_split=split, grav_variant=v))
    return out


def _key(kind, precision, n):
    b = 1
    while b < n:
        b <<= 1
    return "%s:%d:%d" % (kind, precision, b)


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, key, entry):
    cache = load_cache(path)
    cache[key] = entry
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)


def _stage_ms(prof, names):
    return sum(prof[k][0] / max(prof[k][1], 1) for k in names)


def time_gravity(st, precision, params, reps=2):
    """Mean ms of one gravity evaluation (preparation + pair kernel)."""
    from . import sphgrav as sg
    eng = sg.Engine(st, precision=precision, **params)
    ctx = eng.ctx
    ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)          # warm-up (code load, caches)
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.close()
    return _stage_ms(prof, ("grav", "grav_prep"))


def tune_gravity(st, precision, reps=2, path=CACHE, verbose=False):
    """Coordinate search over (ipl, tile, split, variant); returns the best dict."""
    from . import sphgrav as sg
    n = len(st["x"])
    best = dict(grav_ipl=0, grav_tile=0, grav_split=0, grav_variant=0)
    best_ms = time_gravity(st, precision, best, reps)
    rows = [dict(best, ms=best_ms)]

    def try_axis(name, values):
        nonlocal best, best_ms
        for v in values:
            cand = dict(best, **{name: v})
            if cand == best:
                continue
            ms = time_gravity(st, precision, cand, reps)
            rows.append(dict(cand, ms=ms))
            if verbose:
                print("  %s: %.3f ms" % (cand, ms), file=sys.stderr, flush=True)
            if ms < best_ms:
                best, best_ms = cand, ms

    try_axis("grav_ipl", IPLS)
    try_axis("grav_tile", TILES)
    ipl = best["grav_ipl"] or 2
    try_axis("grav_split", sorted({1, 2, 4, _fill_split(n, ipl)}))
    if precision == sg.SG_FP64:
        try_axis("grav_variant", (1, 2, 3, 4))
    _store(path, _key("grav", precision, n), dict(best=best, ms=best_ms, n=n, tried=rows))
    return best


def time_sph(st, precision, cell_scale_log2, reps=2):
    """Mean ms of neighbour build + density + SPH forces at a cell scale."""
    from . import sphgrav as sg
    eng = sg.Engine(st, precision=precision, cell_scale_log2=cell_scale_log2)
    ctx = eng.ctx
    eng.build_neighbors()
    ctx.compute_density()
    ctx.compute_accel(sg.SG_SPH)
    ctx.profile_enable(True)
    for _ in range(reps):
        eng.build_neighbors()
        ctx.compute_density()
        ctx.compute_accel(sg.SG_SPH)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.close()
    return sum(prof[k][0] for k in ("sort", "nbr", "density", "sph")) / reps


def tune_cells(st, precision, reps=2, path=CACHE, verbose=False):
    """Best cell_scale_log2 for the SPH part of the step."""
    rows = []
    for s in CELL_SCALES:
        ms = time_sph(st, precision, s, reps)
        rows.append(dict(cell_scale_log2=s, ms=ms))
        if verbose:
            print("  cell_scale_log2 %d: %.3f ms" % (s, ms), file=sys.stderr, flush=True)
    best = min(rows, key=lambda r: r["ms"])
    _store(path, _key("cells", precision, st["ng"]), dict(best=best["cell_scale_log2"],
                                                           ms=best["ms"], tried=rows))
    return best["cell_scale_log2"]


def tune_ensemble(states, reps=2, path=CACHE, verbose=False):
    """Best (ipl, tile) of the persistent ensemble gravity launch."""
    import torch
    from . import sphgrav as sg
    rows = []
    for ipl in IPLS:
        for tile in TILES:
            ens = sg.Ensemble(states, grav_ipl=ipl, grav_tile=tile)
            ens.gravity(sg.SG_GRAV | sg.SG_POT)                 # warm-up
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(ens.stream)
            for _ in range(reps):
                ens.gravity(sg.SG_GRAV | sg.SG_POT)
            b.record(ens.stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            rows.append(dict(grav_ipl=ipl, grav_tile=tile, ms=ms))
            if verbose:
                print("  ensemble ipl %d tile %d: %.3f ms" % (ipl, tile, ms), file=sys.stderr,
                      flush=True)
            ens.close()
    best = min(rows, key=lambda r: r["ms"])
    total = sum(len(s["x"]) for s in states)
    _store(path, _key("ens", sg.SG_FP32C, total),
           dict(best=dict(grav_ipl=best["grav_ipl"], grav_tile=best["grav_tile"]),
                ms=best["ms"], nsys=len(states), tried=rows))
    return dict(grav_ipl=best["grav_ipl"], grav_tile=best["grav_tile"])


def lookup(kind, precision, n, path=CACHE):
    """Cached best parameters ('grav', 'cells' or 'ens') for this size bucket, or None."""
    e = load_cache(path).get(_key(kind, precision, n))
    return None if e is None else e["best"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c2")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--forms", default="fp32c,fp64")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args()
    from . import ic
    from . import sphgrav as sg
    sg.lib()
    st = ic.make(args.config, scale=args.scale)
    out = {"config": args.config, "n_particles": len(st["x"]), "n_gas": st["ng"]}
    for form in args.forms.split(","):
        p = sg.SG_FP32C if form == "fp32c" else sg.SG_FP64
        print("tuning %s gravity" % form, file=sys.stderr, flush=True)
        g = tune_gravity(st, p, args.reps, args.cache, verbose=True)
        print("tuning %s cell size" % form, file=sys.stderr, flush=True)
        c = tune_cells(st, p, args.reps, args.cache, verbose=True)
        out[form] = dict(gravity=g, cell_scale_log2=c)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
