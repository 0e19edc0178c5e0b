"""Benchmark: force-steps/s of the SPH + direct-gravity step at 2M particles.

One step = one predictor-corrector step of the paper's scheme (neighbour
build, density, gravity once, SPH forces twice, two updates) plus the FP64
conserved-quantity reduction, over the head-on collision of two Plummer
gas+halo systems, 1048576 gas + 1048576 halo particles (synthetic, seeded).

The headline value is the FP32-compensated form's steps/s; the FP64 form is
timed beside it, and both forms' acceleration error against the FP64 CPU
oracle on a seeded 4096-particle subset is reported.  The gravity pair
kernel (the dominant kernel) is timed with HIP events on the library's
stream for the roofline figure.  The oracle is timed on the host on a
bounded sample (gravity of the 4096-particle subset plus the whole SPH part)
and extrapolated to one step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 22          # 20 for the acceleration, +2 for the potential
PEAK = {"fp32": 157.3, "fp64": 78.6}  # TFLOP/s, MI355X vector peaks
HBM_PEAK = 8000.0            # GB/s
DT = 1e-3
HBM_ROUNDS = 5               # rounds of the HBM-bound passes timed on their own


def radix_passes(cell_cap):
    """10-bit radix passes of the cell keys for keys below cell_cap."""
    return max(1, ((max(cell_cap - 1, 1)).bit_length() + 9) // 10)


def pass_bytes(stage, precision_form, ng, nnz, ncell):
    """Algorithmic HBM bytes of one launch group of an HBM-bound stage: every
    array the stage must read or write, counted once (per gas particle, per
    neighbour pair, per cell)."""
    if stage == "sort":
        # keys: x,y,z,h,m in (40 B), key out (4), count and max-h atomics
        # (12), the particle's 64-byte record out (for the gather); radix
        # passes: the first reads keys (histogram and scatter, 8 B) and
        # writes key and id (8), each later one reads and writes both
        # (4 + 16); gather: perm and the record in (68), sorted copies and
        # the density records out (104); cells: count, max h, offset (24)
        p = radix_passes(8 * ng + 4096)      # the binding's default cell capacity
        return (120 + 16 + 20 * (p - 1) + 172) * ng + 24 * ncell
    if stage == "nbr":         # own x,y,z,h; count + offset; one int32 per pair
        return 44 * ng + 4 * nnz
    if stage == "density":     # offset, record (64 B), rho out; one index per pair
        return 80 * ng + 4 * nnz
    if stage == "sph":         # v, e packed (32 B in, 32 out), EOS + record build
        #                        (reads the pack), then offsets, records, 4 outputs
        return (400 if precision_form == "fp64" else 336) * ng + 4 * nnz
    raise ValueError(stage)


def hbm_passes(precision_form, prof, ng, nnz, ncell):
    out = {}
    for stage in ("sort", "nbr", "density", "sph"):
        ms, launches = prof[stage]
        if launches == 0 or ms <= 0:
            continue
        b = pass_bytes(stage, precision_form, ng, nnz, ncell)
        gbs = b * launches / (ms * 1e-3) / 1e9
        out[stage] = {"ms_per_launch": ms / launches, "bytes_per_launch": b,
                      "achieved_GB_s": gbs, "frac_of_peak": gbs / HBM_PEAK}
    return out


def recorded_traffic(precision_form):
    """HBM bytes per gravity launch from committed rocprofv3 counter runs, or
    None when the kernel source changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "gravity_%s_c2_traffic.json" % precision_form)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, rec["kernel_source"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["kernel_source_sha256"]:
            return None
    return rec["traffic_bytes_per_launch"]


def nrm_err(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(sg, st, precision, steps, warmup, sample, tune):
    import torch
    eng = sg.Engine(st, precision=precision, **tune)
    ctx = eng.ctx
    # force evaluation at t = 0 (for the error check against the oracle)
    eng.build_neighbors()
    ctx.compute_density()
    ctx.compute_accel(sg.SG_SPH | sg.SG_GRAV | sg.SG_POT)
    ctx.sync()
    acc = np.stack([eng.dev[f][sample].cpu().numpy() for f in ("ax", "ay", "az")], 1)
    ng = st["ng"]
    parts = {"grav": ctx.export(sg.SG_X_ACC_GRAV)[:, sample].T,
             "sph": ctx.export(sg.SG_X_ACC_SPH)[:, sample[sample < ng]].T}
    diag = ctx.diagnostics()
    for _ in range(warmup):
        ctx.step(DT, sg.SG_POT)
        ctx.diagnostics(diag)
    ctx.sync()
    ctx.profile_enable(True)
    # per-step events on the context's stream (no host waits between steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(ctx.stream)
    for k in range(steps):
        ctx.step(DT, sg.SG_POT)
        ctx.diagnostics(diag)
        evs[k + 1].record(ctx.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.sync()
    # The HBM-bound passes on their own: inside a step the neighbour build,
    # density and corrector SPH forces run beside the gravity kernel, so
    # their stage times there include waiting for compute units.
    # HBM_ROUNDS rounds through the separate entry points (one pass after
    # another, no gravity) time them unobstructed.
    ctx.profile_enable(True)
    for _ in range(HBM_ROUNDS):
        eng.build_neighbors()
        ctx.compute_density()
        ctx.compute_accel(sg.SG_SPH)
    prof_serial = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.sync()
    d = diag.cpu().numpy()
    nnz = int(ctx.export(sg.SG_X_NBR_OFF)[-1])
    ncell = int(sg.grid_dict(ctx.export(sg.SG_X_GRID))["M"])
    eng.ctx.close()
    del eng
    torch.cuda.empty_cache()
    return {"sec": (t1 - t0), "step_ms": step_ms, "acc": acc, "parts": parts, "prof": prof,
            "prof_serial": prof_serial, "diag": d.tolist(), "nnz": nnz, "ncell": ncell}


def cpu_baseline(st, sample, prm):
    """Time the oracle on a bounded sample of the same workload."""
    import oracle
    oracle.lib()
    ng = st["ng"]
    n = len(st["x"])
    x, y, z = st["x"][:ng], st["y"][:ng], st["z"][:ng]
    t = time.perf_counter()
    oracle.sort_gas(x, y, z, st["h"])
    nb = oracle.nbrs(x, y, z, st["h"])
    t_nbr = time.perf_counter() - t
    t = time.perf_counter()
    rho = oracle.density(x, y, z, st["m"][:ng], st["h"], *nb)
    t_dens = time.perf_counter() - t
    t = time.perf_counter()
    asx, asy, asz, de = oracle.sph_force(x, y, z, st["vx"][:ng], st["vy"][:ng], st["vz"][:ng],
                                         st["m"][:ng], st["h"], rho, st["e"], prm["gamma"],
                                         prm["alpha"], prm["beta"], prm["eta"], *nb)
    t_sph = time.perf_counter() - t
    t = time.perf_counter()
    gx, gy, gz, gp = oracle.gravity(st["x"], st["y"], st["z"], st["m"], prm["G"], prm["eps"],
                                    sample)
    t_grav = time.perf_counter() - t
    gas = sample < ng
    ref_grav = np.stack([gx, gy, gz], 1)
    ref_sph = np.stack([asx[sample[gas]], asy[sample[gas]], asz[sample[gas]]], 1)
    ref = ref_grav.copy()
    ref[gas] += ref_sph
    step_s = t_nbr + t_dens + 2 * t_sph + t_grav * n / len(sample)
    cores = oracle.get_threads()
    host = {"nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "omp_threads": cores, "kdtree_workers": oracle.kdtree_workers(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}
    # one thread: density, forces and gravity of 256 of the targets (the
    # k-d tree neighbour search keeps its all-core time)
    oracle.set_threads(1)
    try:
        t = time.perf_counter()
        rho1 = oracle.density(x, y, z, st["m"][:ng], st["h"], *nb)
        t1_dens = time.perf_counter() - t
        t = time.perf_counter()
        oracle.sph_force(x, y, z, st["vx"][:ng], st["vy"][:ng], st["vz"][:ng], st["m"][:ng],
                         st["h"], rho1, st["e"], prm["gamma"], prm["alpha"], prm["beta"],
                         prm["eta"], *nb)
        t1_sph = time.perf_counter() - t
        s1 = sample[:: max(1, len(sample) // 256)]
        t = time.perf_counter()
        oracle.gravity(st["x"], st["y"], st["z"], st["m"], prm["G"], prm["eps"], s1)
        t1_grav = time.perf_counter() - t
    finally:
        oracle.set_threads(cores)
    step1_s = t_nbr + t1_dens + 2 * t1_sph + t1_grav * n / len(s1)
    return {"total": ref, "grav": ref_grav, "sph": ref_sph}, {
        "value": 1.0 / step_s, "unit": "force-steps/s", "cores": cores, "kind": "oracle",
        "sample": ("gravity of %d seeded targets over all %d sources (x%.0f to a step) + whole "
                   "SPH part (neighbours %.1fs, density %.1fs, forces %.1fs x2); gravity %.1fs"
                   % (len(sample), n, n / len(sample), t_nbr, t_dens, t_sph, t_grav)),
        "extrapolated": True,
        "host": host,
        "single_core": {"value": 1.0 / step1_s, "unit": "force-steps/s", "cores": 1,
                        "sample": ("one thread: gravity of %d of the targets (x%.0f) + "
                                   "density %.1fs + forces %.1fs x2; gravity %.1fs; the "
                                   "neighbour search's all-core time (%.1fs) is included"
                                   % (len(s1), n / len(s1), t1_dens, t1_sph, t1_grav, t_nbr))},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--only", choices=["fp32c", "fp64", "both"], default="both")
    ap.add_argument("--ipl", type=int, default=0, help="gravity targets per lane (0 = auto)")
    ap.add_argument("--split", type=int, default=0, help="gravity source splits (0 = auto)")
    ap.add_argument("--tile", type=int, default=0, help="gravity sources per LDS tile (0 = auto)")
    ap.add_argument("--variant", type=int, default=0,
                    help="FP64 gravity kernel: 0 automatic, 1/2 pair differences with FP32-/FP64-"
                         "seeded rsqrt, 3/4 expanded far field with the same seeds")
    ap.add_argument("--serial", action="store_true",
                    help="run each step's gravity after the neighbour/SPH chain instead of "
                         "beside it (kernel traces with unobstructed per-kernel durations)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_1807_08116_amd import ic
    from paper_1807_08116_amd import sphgrav as sg
    sg.lib()
    prm = ic.DEFAULT_PARAMS
    t = time.perf_counter()
    st = ic.make(args.config)
    n, ng = len(st["x"]), st["ng"]
    log("inputs %s: N=%d (gas %d) in %.1fs" % (args.config, n, ng, time.perf_counter() - t))
    sample = np.sort(np.random.default_rng(ic.SEED_BASE + 99).choice(n, 4096, replace=False))

    res = {}
    forms = ["fp32c", "fp64"] if args.only == "both" else [args.only]
    for form in forms:
        p = sg.SG_FP32C if form == "fp32c" else sg.SG_FP64
        log("timing %s: %d warmup + %d steps" % (form, args.warmup, args.steps))
        tune = dict(grav_ipl=args.ipl, grav_split=args.split, grav_tile=args.tile,
                    grav_variant=args.variant if p == sg.SG_FP64 else 0,
                    step_serial=1 if args.serial else 0)
        res[form] = run_form(sg, st, p, args.steps, args.warmup, sample, tune)
        log("  %s: %.3f s/step" % (form, res[form]["sec"] / args.steps))

    cpu = None
    errs = {}
    if not args.no_cpu:
        log("oracle baseline on the host ...")
        ref, cpu = cpu_baseline(st, sample, prm)
        for form in forms:
            r = res[form]
            errs[form] = nrm_err(r["acc"], ref["total"])
            rel = (np.linalg.norm(r["acc"] - ref["total"], axis=1)
                   / np.linalg.norm(ref["total"], axis=1))
            r["err_parts"] = {"gravity": nrm_err(r["parts"]["grav"], ref["grav"]),
                              "sph": nrm_err(r["parts"]["sph"], ref["sph"]),
                              "median_particle_rel": float(np.median(rel))}
        log("  oracle %.4g steps/s (extrapolated); errors %s" % (cpu["value"], errs))

    head = "fp32c" if "fp32c" in res else "fp64"
    sec = res[head]["sec"]
    gms, glaunch = res[head]["prof"]["grav"]
    grav_s = gms / 1e3 / max(glaunch, 1)
    achieved = FLOPS_PER_PAIR * float(n) * float(n) / grav_s / 1e12
    peak = PEAK["fp32" if head == "fp32c" else "fp64"]
    out = {
        "metric": "force-steps/s at 2M particles, FP32-compensated vs FP64, at 1e-6 accel err",
        "value": args.steps / sec,
        "unit": "force-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32c" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: head-on collision of two Plummer gas+halo systems, "
                               "%d gas + %d halo particles, one predictor-corrector step "
                               "+ FP64 energy/momentum sums" % (args.config, ng, n - ng),
                   "n_particles": n, "n_gas": ng, "precision_form": head, "seed": ic.SEED_BASE + int(args.config[1:])},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": recorded_traffic(head) if args.config == "c2" else None,
                     "kernel": "gravity pair kernel (%s), %d flops/pair x N^2 per launch, "
                               "%.1f ms/launch" % (head, FLOPS_PER_PAIR, 1e3 * grav_s)},
        "cpu_baseline": cpu,
        "accel_err_vs_oracle": errs,
        "pairs_per_s": float(n) * n / grav_s,
        "software": {"library": sg.lib().sg_version().decode(),
                     "hip": getattr(torch.version, "hip", None), "torch": torch.__version__},
    }
    for form in res:
        pr = res[form]["prof"]
        out[form] = {
            "steps_per_s": args.steps / res[form]["sec"],
            "ms_per_step": 1e3 * res[form]["sec"] / args.steps,
            "ms_per_step_events": res[form]["step_ms"],
            "ms_per_step_median": float(np.median(res[form]["step_ms"])),
            "stage_ms_per_step": {k: v[0] / args.steps for k, v in pr.items()},
            "stage_note": "stages of the timed steps; the neighbour, density and SPH stages "
                          "run beside the gravity kernel, so their times include waiting "
                          "for compute units (hbm_passes times them on their own)",
            "grav_ms_per_launch": pr["grav"][0] / max(pr["grav"][1], 1),
            "accel_err": errs.get(form),
            "accel_err_parts": res[form].get("err_parts"),
            "diagnostics_last": res[form]["diag"],
            "nnz": res[form]["nnz"],
            "hbm_passes": hbm_passes(form, res[form]["prof_serial"], ng, res[form]["nnz"],
                                     res[form]["ncell"]),
            "hbm_passes_measured": ("%d rounds of neighbours, density and SPH forces through "
                                    "the separate entry points after the timed steps" % HBM_ROUNDS),
        }
    if "fp64" in res and "fp32c" in res:
        out["fp32c_vs_fp64_speedup"] = res["fp64"]["sec"] / res["fp32c"]["sec"]
    if "fp64" in res and head != "fp64":
        ms64, n64 = res["fp64"]["prof"]["grav"]
        s64 = ms64 / 1e3 / max(n64, 1)
        a64 = FLOPS_PER_PAIR * float(n) * float(n) / s64 / 1e12
        out["roofline_fp64"] = {"bound": "alu", "achieved": a64, "peak": PEAK["fp64"],
                                "unit": "TFLOP/s", "frac": a64 / PEAK["fp64"],
                                "kernel": "gravity pair kernel (fp64), %.1f ms/launch" % (1e3 * s64)}
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = {"read": 1 << 30, "write": 1 << 30, "launches": 3}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
