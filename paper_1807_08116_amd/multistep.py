"""Multi-step run with graph-captured steps: energy and momentum drift.

Runs the off-axis 3:1 collision (2097152 gas + 2097152 halo particles by
default) for a number of predictor-corrector steps in each precision form,
with the steady-state step captured into a HIP graph and replayed, and
reports steps/s plus the drift of the FP64 conserved-quantity sums:
|E(t) - E(0)| / |E(0)|, |P(t) - P(0)| / sum m|v|, and the gap between the
FP32-compensated and FP64 trajectories.

Usage: python -m paper_1807_08116_amd.multistep [--config c3] [--steps 50]
           [--chunk 10] [--forms fp32c,fp64] [--dt 1e-3] [--scale 1.0]
           [--save-hist DIR]
       python -m paper_1807_08116_amd.multistep --compare FP32C.npy FP64.npy
"""
import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(sg, st, precision, steps, chunk, dt):
    import torch
    eng = sg.Engine(st, precision=precision, stream="new")
    ctx = eng.ctx
    d0 = ctx.diagnostics()
    ctx.sync()
    # forces at t = 0 are needed for E_pot(0): one evaluation outside the steps
    eng.build_neighbors()
    ctx.compute_density()
    ctx.compute_accel(sg.SG_SPH | sg.SG_GRAV | sg.SG_POT)
    ctx.diagnostics(d0)
    ctx.sync()
    hist = [d0.cpu().numpy()[None, :]]
    done = 0
    t_total = 0.0
    while done < steps:
        k = min(chunk, steps - done)
        torch.cuda.synchronize()
        t = time.perf_counter()
        h = ctx.run(dt, k, sg.SG_POT, use_graph=True)
        torch.cuda.synchronize()
        t_total += time.perf_counter() - t
        hist.append(h.cpu().numpy())
        done += k
        e = hist[-1][-1]
        log("  step %d/%d  E=%.12e  dE/E0=%.3e  %.3f s/step" %
            (done, steps, e[3], abs(e[3] - hist[0][0][3]) / abs(hist[0][0][3]), t_total / done))
    ctx.sync()
    H = np.concatenate(hist, 0)
    ctx.close()
    del eng
    torch.cuda.empty_cache()
    return H, t_total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c3")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--chunk", type=int, default=10)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--forms", default="fp32c,fp64")
    ap.add_argument("--save-hist", default=None,
                    help="directory to write each form's per-step conserved sums "
                         "(hist_<form>_<config>.npy, rows E_kin, E_int, E_pot, E, P, L)")
    ap.add_argument("--compare", nargs=2, default=None, metavar=("FP32C_NPY", "FP64_NPY"),
                    help="compare two saved histories (no GPU work) and print the gaps")
    args = ap.parse_args()
    if args.compare:
        a, b = (np.load(f) for f in args.compare)
        k = min(len(a), len(b))
        print(json.dumps({"steps_compared": k - 1, **gaps(a[:k], b[:k])}), flush=True)
        return
    from paper_1807_08116_amd import ic
    from paper_1807_08116_amd import sphgrav as sg
    sg.lib()
    t = time.perf_counter()
    st = ic.make(args.config, scale=args.scale)
    n, ng = len(st["x"]), st["ng"]
    log("inputs %s: N=%d (gas %d) in %.1fs" % (args.config, n, ng, time.perf_counter() - t))
    m = st["m"]
    pscale = float(np.sum(m * np.sqrt(st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2)))
    out = {"config": args.config, "n_particles": n, "n_gas": ng, "steps": args.steps,
           "dt": args.dt, "graph": True, "forms": {}}
    hists = {}
    for form in args.forms.split(","):
        p = sg.SG_FP32C if form == "fp32c" else sg.SG_FP64
        log("form %s: %d steps in chunks of %d" % (form, args.steps, args.chunk))
        H, sec = run_form(sg, st, p, args.steps, args.chunk, args.dt)
        hists[form] = H
        E0 = H[0, 3]
        dE = np.abs(H[:, 3] - E0) / abs(E0)
        dP = np.linalg.norm(H[:, 4:7] - H[0, 4:7], axis=1) / pscale
        dL = np.linalg.norm(H[:, 7:10] - H[0, 7:10], axis=1)
        out["forms"][form] = {
            "steps_per_s": args.steps / sec, "s_per_step": sec / args.steps,
            "energy_drift_final": float(dE[-1]), "energy_drift_max": float(dE.max()),
            "momentum_drift_max": float(dP.max()), "angmom_change_max": float(dL.max()),
            "E0": float(E0), "E_final": float(H[-1, 3]),
        }
    if args.save_hist:
        import os
        os.makedirs(args.save_hist, exist_ok=True)
        for form, H in hists.items():
            np.save(os.path.join(args.save_hist, "hist_%s_%s.npy" % (form, args.config)), H)
    if "fp32c" in hists and "fp64" in hists:
        a, b = hists["fp32c"], hists["fp64"]
        k = min(len(a), len(b))
        out["fp32c_vs_fp64"] = gaps(a[:k], b[:k])
    print(json.dumps(out), flush=True)


def gaps(a, b):
    """Largest gaps between two histories of the conserved sums (same steps):
    total energy relative to |E(0)| of the second (values, and changes
    since step 0), momentum and angular momentum absolute."""
    return {
        "energy_gap_max": float(np.max(np.abs(a[:, 3] - b[:, 3]) / abs(b[0, 3]))),
        "energy_change_gap_max": float(np.max(np.abs((a[:, 3] - a[0, 3]) - (b[:, 3] - b[0, 3]))
                                              / abs(b[0, 3]))),
        "momentum_gap_max": float(np.max(np.linalg.norm(a[:, 4:7] - b[:, 4:7], axis=1))),
        "angmom_gap_max": float(np.max(np.linalg.norm(a[:, 7:10] - b[:, 7:10], axis=1))),
    }


if __name__ == "__main__":
    main()
