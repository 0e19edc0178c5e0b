"""Batched ensemble: independent two-system collisions in one persistent
gravity launch, against running the systems one by one.

Default workload: 64 collisions, N per system log-uniform in [8192, 262144]
(gas:halo 1:1), impact parameter U[0, 3], closing speed U[0.5, 2];
FP32-compensated form.  Reports aggregate pair-interactions/s of the
batched gravity and of per-system launches, and steps/s of graph-captured
ensemble steps.

With --tune the persistent launch's targets per lane (the block of
targets) and j-tile are first picked by the autotuner on these systems,
and the neighbour-grid cell size on the largest of them.

Usage: python -m paper_1807_08116_amd.ensemble [--nsys 64] [--steps 50]
           [--reps 3] [--scale 1.0] [--tune]
"""
import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nsys", type=int, default=64)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--reorder", type=int, default=0,
                    help="gravity preparations per Morton-order recomputation (0 = every one)")
    ap.add_argument("--chain-stream", choices=["cu", "torch"], default="cu",
                    help="stream of the systems' corrector chains beside the batched gravity: "
                         "the library's CU-masked stream or a torch stream")
    args = ap.parse_args()
    import torch
    from paper_1807_08116_amd import ic
    from paper_1807_08116_amd import sphgrav as sg
    sg.lib()
    t = time.perf_counter()
    states = ic.ensemble(nsys=args.nsys, scale=args.scale)
    ns = np.array([len(s["x"]) for s in states], dtype=np.float64)
    pairs = float(np.sum(ns * ns))
    log("inputs: %d systems, %d particles, %.3e pairs per gravity pass (%.1fs)"
        % (len(states), int(ns.sum()), pairs, time.perf_counter() - t))
    shape = {}
    if args.tune:
        from paper_1807_08116_amd import autotune
        t = time.perf_counter()
        shape = autotune.tune_ensemble(states, reps=2, verbose=True)
        # cell size of the neighbour grid, tuned on the largest system
        big = max(states, key=lambda s: len(s["x"]))
        shape["cell_scale_log2"] = autotune.tune_cells(big, sg.SG_FP32C, reps=2, verbose=True)
        log("autotuned ensemble launch %s (%.1fs)" % (shape, time.perf_counter() - t))
    if args.reorder:
        shape["grav_reorder"] = args.reorder
    ens = sg.Ensemble(states, chain_stream=None if args.chain_stream == "cu" else "new", **shape)
    st = ens.stream
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()                                        # warm-up
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record(st)
        for _ in range(args.reps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.reps

    ms_batched = timed(lambda: ens.gravity(sg.SG_GRAV | sg.SG_POT))
    log("batched gravity: %.2f ms (%.3e pairs/s)" % (ms_batched, pairs / ms_batched * 1e3))

    def one_by_one():
        for e in ens.engines:
            e.ctx.compute_accel(sg.SG_GRAV | sg.SG_POT)
    ms_single = timed(one_by_one)
    log("one by one:      %.2f ms (%.3e pairs/s)" % (ms_single, pairs / ms_single * 1e3))

    # steps, graph-captured (one capture per run, chunks of one Morton-order
    # period) and eager (the host enqueues every launch of every step)
    sec = {}
    for graph in (True, False):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ens.run(args.dt, args.steps, sg.SG_POT, use_graph=graph)
        torch.cuda.synchronize()
        sec[graph] = time.perf_counter() - t
        log("%d %s ensemble steps: %.3f s/step"
            % (args.steps, "graph-captured" if graph else "eager", sec[graph] / args.steps))
    out = {
        "workload": "%d independent collisions, N log-uniform in [8192, 262144] x %g"
                    % (len(states), args.scale),
        "n_particles": int(ns.sum()), "pairs_per_gravity": pairs,
        "batched_gravity_ms": ms_batched, "batched_pairs_per_s": pairs / ms_batched * 1e3,
        "one_by_one_gravity_ms": ms_single, "one_by_one_pairs_per_s": pairs / ms_single * 1e3,
        "batched_speedup": ms_single / ms_batched,
        "steps": args.steps, "steps_per_s_graph": args.steps / sec[True],
        "steps_per_s_eager": args.steps / sec[False], "precision": "fp32c",
        "grav_reorder": args.reorder or 1, "chain_stream": args.chain_stream,
        "launch": shape or "automatic",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
