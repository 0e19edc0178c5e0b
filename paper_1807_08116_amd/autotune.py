"""Autotuner for the gravity launch shape.

Candidates are (variant, targets per lane, source splits); each is timed on
the caller's particle set with the library's own stage timing (HIP events
around the pair kernel) and the fastest is kept.  Results are cached in a
JSON file keyed by precision form and the particle count rounded to a power
of two, so later runs of similar size reuse them.

Only launch parameters are searched: every candidate computes the same sums
(up to summation order), which the parity tests check for each shape.
"""
from __future__ import annotations

import json
import os

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def candidates(precision, n):
    from . import sphgrav as sg
    out = []
    if precision == sg.SG_FP32C:
        blocks = max(1, (n + 63) // 64)
        for split in sorted({1, 2, 4, max(1, min(64, 2048 // blocks)), max(1, min(64, 4096 // blocks))}):
            out.append((2, 0, split))
        for ipl in (2, 4):
            out.append((1, ipl, 0))
    else:
        for ipl in (1, 2, 4):
            blocks = max(1, (n + 256 * ipl - 1) // (256 * ipl))
            for split in sorted({1, max(1, min(64, 2048 // blocks)), max(1, min(64, 4096 // blocks))}):
                out.append((1, ipl, split))
    return out


def _key(precision, n):
    b = 1
    while b < n:
        b <<= 1
    return "%d:%d" % (precision, b)


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def tune_gravity(st, precision, reps=2, path=CACHE, verbose=False):
    """Time each candidate on state `st`; return (variant, ipl, split)."""
    from . import sphgrav as sg
    n = len(st["x"])
    best = None
    rows = []
    for variant, ipl, split in candidates(precision, n):
        eng = sg.Engine(st, precision=precision, grav_variant=variant, grav_ipl=ipl,
                        grav_split=split)
        ctx = eng.ctx
        ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)          # warm-up (code load, caches)
        ctx.profile_enable(True)
        for _ in range(reps):
            ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        ms = prof["grav"][0] / max(prof["grav"][1], 1) + prof["grav_prep"][0] / max(prof["grav_prep"][1], 1)
        rows.append({"variant": variant, "ipl": ipl, "split": split, "ms": ms})
        if verbose:
            print("  variant %d ipl %d split %d: %.3f ms" % (variant, ipl, split, ms), flush=True)
        if best is None or ms < best[0]:
            best = (ms, variant, ipl, split)
        ctx.close()
        del eng
    cache = load_cache(path)
    cache[_key(precision, n)] = {"variant": best[1], "ipl": best[2], "split": best[3],
                                 "ms": best[0], "n": n, "tried": rows}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return best[1], best[2], best[3]


def lookup(precision, n, path=CACHE):
    """Cached (variant, ipl, split) for this size bucket, or None."""
    e = load_cache(path).get(_key(precision, n))
    if e is None:
        return None
    return e["variant"], e["ipl"], e["split"]
