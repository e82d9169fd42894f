"""Benchmark of the per-stage residual-and-update sweep on one MI355X.

Default workload: the batched case -- 256 independent 2D instances of uneven
size (64^2..512^2), f = (u^2/2, u^2/2), a = c u^m, limiter and point-value
projection on, FP32, SSP-RK3, all K steps in one HIP graph launch.  Prints one
JSON line.  ``value`` is cell-DoF updates per second per RK stage (all
instances, inputs resident in HBM before the timed region).

    python bench.py [--steps K] [--warmup W] [--workload c4|c2|c3|c3f32|c5|nodc|ek|c3out]
"""
import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-DOF updates/s per RK stage + %HBM roofline, FP32 batched vs FP64 plain"
UNIT = "cell-DoF updates/s per RK stage"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the HIP sources and the build script (its compiler flags); a
    traffic figure measured with other sources or flags is stale and not
    reported."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2510_11527_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "paper_2510_11527_amd", "build.py"))
    for f in files:
        if f.endswith((".hpp", ".hip", ".h", ".cpp", ".py")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(workload_name, tile):
    """The committed rocprofv3 summary of this workload and tile -- HBM bytes
    per stage launch (FETCH_SIZE / WRITE_SIZE) and VALU busy % -- if the
    kernel sources are the ones it was measured with; else an empty dict."""
    sha = kernel_source_sha()
    for f in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.txt")):
        kv = {}
        with open(f) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.strip().split("=", 1)
                    kv[k] = v
        if kv.get("workload") == workload_name and kv.get("tile") == tile and kv.get("source_sha") == sha:
            return kv
    return {}


def measured_traffic(workload_name, tile):
    """HBM bytes per stage launch (see measured_counters), or None."""
    kv = measured_counters(workload_name, tile)
    return float(kv["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in kv else None


def measured_valu_busy(workload_name, tile):
    """VALU busy % of the stage kernel (see measured_counters), or None."""
    kv = measured_counters(workload_name, tile)
    return float(kv["valu_busy_pct"]) if "valu_busy_pct" in kv else None


def workload(name):
    from paper_2510_11527_amd import workloads as W
    if name == "c4":
        items = W.config4()
        return "c4_batched_256x2d_pme_burgers_fp32", items
    if name == "c2":
        return "c2_burgers_deadzone_512x512_fp64", [W.config2()]
    if name == "c3":
        return "c3_buckley_leverett_gravity_1024x1024_fp64", [W.config3(precision=64)]
    if name == "c3f32":
        return "c3_buckley_leverett_gravity_1024x1024_fp32", [W.config3(precision=32)]
    if name == "c5":
        return "c5_degenerate_3d_256cubed_fp32_si", [W.config5()]
    if name == "nodc":
        return "nodc_ek_batched_1024x8192_1d_fp64", W.config_nodc()
    if name == "ek":
        return "ek_dirichlet_batched_1024x8192_1d_fp64", W.config_ek()
    if name == "c3out":
        spec, U = W.config3(precision=64)
        return ("c3_buckley_leverett_gravity_1024x1024_fp64_outflow",
                [(dict(spec, bcs=[("outflow", "outflow"), ("outflow", "outflow")]), U)])
    raise SystemExit("unknown workload " + name)


def make_ctx(items, precision=None, variant=None, integrator="ssprk3"):
    from paper_2510_11527_amd import af
    ctx = af.Context([s for s, _ in items], precision=precision, integrator=integrator)
    if variant is not None:
        ctx.set_variant(variant)
    for i, (_, U) in enumerate(items):
        ctx.set_state(i, U)
    return ctx


STAGES = {"ssprk3": 3, "ssprk54": 5, "euler": 1}


def cpu_model():
    """Host CPU model name (first processor of /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(items, target_cells, integrator="ssprk3"):
    """The FP64 oracle on a bounded sample, on all host cores: the first
    instances of the same workload up to target_cells cells, one SSP-RK3 step
    with CFL steps (an instance far larger than that: one forward-Euler stage
    of its first target_cells cells); and on one core, one forward-Euler
    stage of the first cells of the first instance."""
    import oracle
    oracle.build()
    sample, cells = [], 0
    for s, U in items:
        sample.append((s, U))
        cells += int(np.prod(s["n"][:s["dim"]]))
        if cells >= target_cells:
            break
    dofs_per_cell = 2 ** items[0][0]["dim"]
    cores = oracle.num_threads()
    s0, U0 = items[0]
    n0 = int(np.prod(s0["n"][:s0["dim"]]))
    if n0 > 4 * target_cells:
        # one instance far above the target (3D 256^3): one forward-Euler
        # stage of its first target_cells cells, on all cores
        P0 = oracle.problem(s0)
        dt0 = oracle.dt_cfl(P0, U0, s0["cfl"])
        t0 = time.perf_counter()
        oracle.fe_cells(P0, U0, dt0, np.arange(target_cells))
        el = time.perf_counter() - t0
        value = target_cells * dofs_per_cell / el
        what = "one forward-Euler stage of the first %d cells of the first instance, %.1f s" % (target_cells, el)
    else:
        t0 = time.perf_counter()
        for s, U in sample:
            P = oracle.problem(s)
            oracle.run(P, U, nsteps=1, cfl=s["cfl"], integrator=integrator)
        el = time.perf_counter() - t0
        value = cells * dofs_per_cell * STAGES[integrator] / el
        what = "first %d instances of the workload (%d cells), 1 %s step (%d stages), %.1f s" % (
            len(sample), cells, integrator, STAGES[integrator], el)
    # one core: one forward-Euler stage of the first cells of the first
    # instance (cell by cell, so the sample stays bounded for any grid)
    P0 = oracle.problem(s0)
    k = min(n0, 200_000)
    dt0 = oracle.dt_cfl(P0, U0, s0["cfl"])
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.fe_cells(P0, U0, dt0, np.arange(k))
    el1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    return {"value": value, "unit": UNIT, "cores": cores, "kind": "oracle", "sample": what, "cpu": cpu_model(),
            "single_core": {"value": k * dofs_per_cell / el1, "unit": UNIT, "cores": 1,
                            "sample": "one forward-Euler stage of the first %d cells of the first instance, %.1f s"
                                      % (k, el1)}}


def fp64_plain(items, steps, integrator="ssprk3"):
    """The same instances in FP64, one context per instance, stepped one after
    the other (no batching): the 'plain' form.  Each context is warmed up like
    the batched one (one step, then one K-step graph launch, which captures
    the graph) before the timed K-step launches."""
    from paper_2510_11527_amd import af
    ctxs = []
    for s, U in items:
        c = af.Context(dict(s, precision=64), integrator=integrator)
        c.set_state(0, U)
        c.step(1)
        c.step(steps)
        ctxs.append(c)
    t0 = time.perf_counter()
    for c in ctxs:
        c.step(steps)
    el = time.perf_counter() - t0
    cells = sum(int(np.prod(s["n"][:s["dim"]])) for s, _ in items)
    dpc = 2 ** items[0][0]["dim"]
    return ctxs, {"value": cells * dpc * STAGES[integrator] * steps / el, "unit": UNIT, "dtype": "f64",
                  "instances": len(items), "cells": cells, "steps": steps, "seconds": el}


def rel_l1(a, b):
    """max over DoF kinds of ||a - b||_1 / ||b||_1 (uniform cells)."""
    return max(float(np.abs(np.asarray(x) - np.asarray(y)).sum() / max(np.abs(y).sum(), 1e-300))
               for x, y in zip(a, b))


def restrict(spec, U):
    """DoFs of a fine grid on the grid of half as many cells per axis: an
    average is the mean of the 2^d fine averages it covers; every point value
    of the coarse grid is a fine corner point value (all coarse DoF points lie
    on fine faces along every axis)."""
    d = spec["dim"]
    n = spec["n"][:d]
    shp = tuple(reversed(n))
    A = np.asarray(U[0]).reshape(shp)
    for ax in range(d):
        A = A.reshape(A.shape[:ax] + (A.shape[ax] // 2, 2) + A.shape[ax + 1:]).mean(axis=ax + 1)
    C = np.asarray(U[-1]).reshape(shp)   # the corner kind (all axes on faces)
    from paper_2510_11527_amd import workloads as W
    out = [A.reshape(-1)]
    for mask in W.ZETA_MASKS[d][1:]:
        sl = tuple(slice(1 if (mask >> (d - 1 - a)) & 1 else 0, None, 2) for a in range(d))
        out.append(C[sl].reshape(-1))
    return out


def coarse_fourier(spec, U):
    """The instance's Fourier initial data on half as many cells per axis,
    rescaled with the fine grid's map to [0, 1] (so that both grids sample one
    and the same function)."""
    from paper_2510_11527_amd import workloads as W
    d = spec["dim"]
    g = W.fourier_dofs(spec, spec["modes"])
    g0, g1 = min(float(x.min()) for x in g), max(float(x.max()) for x in g)
    sc = dict(spec, n=[v // 2 for v in spec["n"][:d]] + list(spec["n"][d:]), precision=64)
    gc = W.fourier_dofs(sc, spec["modes"])
    return sc, [(x - g0) / (g1 - g0) for x in gc]


def run_to(ctx, t_end, chunk=500):
    """Steps every instance of ctx to t_end (CFL steps, the last one clipped)."""
    while True:
        ctx.step(chunk, t_end=t_end)
        if all(ctx.norms(i)["t"] >= t_end * (1 - 1e-12) for i in range(len(ctx.specs))):
            return


def c4_accuracy(items, fp64_ctxs, steps, fp32_ctx, n_coarse=16):
    """Equal stated accuracy of the FP32 batched and FP64 plain forms on the
    batched workload: both from the initial state for `steps` CFL steps;
    max over instances of the relative l1 difference, against the
    discretisation error estimated on a subset by the same run on half as
    many cells per axis to the same time (relative l1 of the restricted fine
    FP64 solution against the coarse one)."""
    from paper_2510_11527_amd import af
    for i, (s, U) in enumerate(items):
        fp32_ctx.set_state(i, U)
        fp64_ctxs[i].set_state(0, U)
    fp32_ctx.step(steps)
    worst, tdiff = 0.0, 0.0
    u64s, t64s = [], []
    for i, c in enumerate(fp64_ctxs):
        c.step(steps)
        V64, t64 = c.get_state(0)
        V32, t32 = fp32_ctx.get_state(i)
        worst = max(worst, rel_l1(V32, V64))
        tdiff = max(tdiff, abs(t32 - t64) / t64)
        t64s.append(t64)
        u64s.append(V64 if i < 4 * n_coarse else None)
    # discretisation error on a subset: instances of >= 128^2 cells
    sub = [i for i, (s, _) in enumerate(items) if s["n"][0] >= 128 and u64s[i] is not None][:n_coarse]
    disc = []
    for i in sub:
        s, U = items[i]
        sc, Uc = coarse_fourier(s, U)
        cc = af.Context(sc)
        cc.set_state(0, Uc)
        run_to(cc, t64s[i], chunk=64)
        Vc, _ = cc.get_state(0)
        cc.close()
        disc.append(rel_l1(restrict(s, u64s[i]), Vc))
    med = float(np.median(disc)) if disc else None
    # fourth order: the error on N cells is about the N/2-vs-N difference / 15
    est = med / 15.0 if disc else None
    return {"steps": steps, "fp32_vs_fp64_rel_l1_max": worst, "time_rel_diff_max": tdiff,
            "stated_fp32_tolerance": 1e-5, "fp32_within_stated": worst <= 1e-5,
            "disc_n_vs_half_n_rel_l1_median": med, "disc_n_vs_half_n_rel_l1_min": min(disc) if disc else None,
            "disc_err_estimate_n": est, "disc_subset": len(disc),
            "fp32_within_0p1_disc": (worst <= 0.1 * est) if disc else None}


def accuracy_report(which):
    """Per-workload end-of-run accuracy (one JSON line per workload): the
    configured run on the GPU in FP64 and, for FP32 workloads, in FP32 with
    the same number of CFL steps; the relative l1 difference of the two, the
    difference of the FP64 run from the same run on half as many cells per
    axis (restricted), mass drift and bounds."""
    from paper_2510_11527_amd import af
    from paper_2510_11527_amd import workloads as W
    out = []

    def fourier_half(spec, U):
        return coarse_fourier(spec, U)

    def half_of(name, spec):
        d = spec["dim"]
        n = spec["n"][0] // 2
        if name == "c2":
            return W.config2(n=n)
        if name == "c3":
            return W.config3(n=n, precision=64)
        return None

    for name in which:
        t0 = time.perf_counter()
        if name == "c2":
            spec, U = W.config2()
        elif name == "c3":
            spec, U = W.config3(precision=64)
        elif name == "c5":
            spec, U = W.config5()
        else:
            raise SystemExit("accuracy report: unknown workload " + name)
        s64 = dict(spec, precision=64)
        c64 = af.Context(s64)
        c64.set_state(0, U)
        m0 = c64.norms(0)["mass"]
        if spec.get("t_end"):
            run_to(c64, spec["t_end"])
        else:
            c64.step(spec["steps"])
        V64, t64 = c64.get_state(0)
        n64 = c64.norms(0)
        steps = n64["steps"]
        c64.close()
        rec = {"workload": name, "t": t64, "steps": steps, "mass_drift_rel": (n64["mass"] - m0) / abs(m0),
               "min": min(n64["min_avg"], n64["min_pv"]), "max": max(n64["max_avg"], n64["max_pv"]),
               "bounds": [spec["umin"], spec["umax"]]}
        if name in ("c3", "c5"):
            s32 = dict(spec, precision=32)
            U32 = W.round_to(U, 32)
            c32 = af.Context(s32)
            c32.set_state(0, U32)
            if spec.get("t_end"):
                run_to(c32, spec["t_end"])
            else:
                c32.step(spec["steps"])
            V32, t32 = c32.get_state(0)
            c32.close()
            rec["fp32_vs_fp64_rel_l1"] = rel_l1(V32, V64)
            rec["fp32_t"] = t32
        # discretisation: the same run on half as many cells per axis, to the same time
        if name == "c5":
            sc, Uc = coarse_fourier(spec, U)
        else:
            sc, Uc = half_of(name, spec)
        sc = dict(sc, precision=64, umin=spec["umin"], umax=spec["umax"])
        cc = af.Context(sc)
        cc.set_state(0, Uc)
        run_to(cc, t64, chunk=200)
        Vc, _ = cc.get_state(0)
        cc.close()
        rec["n_vs_half_n_rel_l1"] = rel_l1(restrict(spec, V64), Vc)
        rec["seconds"] = time.perf_counter() - t0
        log("accuracy %s: %s" % (name, rec))
        out.append(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--variant", type=int, default=None, help="tile variant (default: autotuned)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile variant")
    ap.add_argument("--autotune-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--integrator", default="ssprk3", choices=["ssprk3", "ssprk54", "euler"],
                    help="euler: one forward-Euler stage plus a plain state copy per step (profiling reference)")
    ap.add_argument("--accuracy-report", default=None,
                    help="comma-separated workloads (c2,c3,c5): end-of-run accuracy report instead of the benchmark")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library drives one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    from paper_2510_11527_amd import af
    if not os.path.exists(af.LIB_PATH):
        from paper_2510_11527_amd import build as B
        B.build(verbose=False)

    if args.accuracy_report:
        for rec in accuracy_report(args.accuracy_report.split(",")):
            print(json.dumps(rec), flush=True)
        return

    t0 = time.perf_counter()
    wname, items = workload(args.workload)
    log("workload %s: %d instances generated in %.1f s" % (wname, len(items), time.perf_counter() - t0))
    prec = items[0][0]["precision"]
    ctx = make_ctx(items, variant=args.variant, integrator=args.integrator)
    work = ctx.work()
    if args.warmup > 0:
        ctx.step(args.warmup)
    log("warmup done")
    tuned = None
    if args.variant is None and not args.no_autotune:
        # untimed: every built tile variant on the warmed-up state, which the
        # tuner restores afterwards
        chosen, ms = ctx.autotune(args.autotune_steps)
        tuned = {ctx.variant_name(v): round(float(m), 5) for v, m in enumerate(ms) if m > 0}
        log("autotune: %s (stage ms %s)" % (ctx.variant_name(chosen), tuned))
    variant_name = ctx.variant_name(ctx.variant())
    # timed region: K steps in one graph launch; inputs already in HBM
    ctx.step(1)
    ctx.step(args.steps)  # builds the graph for K steps (and runs them)
    t1 = time.perf_counter()
    ctx.step(args.steps)
    t2 = time.perf_counter()
    el = t2 - t1
    per_step = STAGES[args.integrator]
    stages = per_step * args.steps
    value = work["dofs"] * stages / el
    log("timed %d steps in %.4f s" % (args.steps, el))

    roof = None
    if not args.no_kernel_timing:
        # stage-kernel durations from HIP events around every stage launch on
        # the context stream, over K more steps of the same workload
        ms, nl = ctx.step_timed(args.steps)
        achieved = work["bytes_per_stage"] / (ms * 1e-3) / 1e9
        copy_gbs = af.copy_rate(1 << 30, 20)
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "attainable_copy": copy_gbs,
                "frac_of_attainable": achieved / copy_gbs,
                "traffic": measured_traffic(wname, variant_name),
                "valu_busy_pct": measured_valu_busy(wname, variant_name),
                "kernel": "stage kernel %s (%s)" % (variant_name, "fp32" if prec == 32 else "fp64"),
                "mean_launch_ms": ms, "launches": nl,
                "algorithmic_bytes_per_launch": work["bytes_per_stage"]}
        log("stage kernel mean %.4f ms over %d launches -> %.1f GB/s (copy kernel %.1f GB/s)" % (
            ms, nl, achieved, copy_gbs))

    line = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == 32 else "f64", "data": "synthetic",
            "config": {"workload": wname, "instances": len(items), "cells": work["cells"], "dofs": work["dofs"],
                       "integrator": args.integrator, "limiter": bool(items[0][0]["limiter"]),
                       "si": bool(items[0][0]["si"]), "cfl": items[0][0]["cfl"], "tile": variant_name,
                       "tile_choice": "autotuned" if tuned else ("given" if args.variant is not None else "default"),
                       "graph": "one hipGraph launch of %d steps" % args.steps},
            "cell_updates_per_s": work["cells"] * stages / el,
            "step_hbm_frac": work["bytes_per_stage"] * stages / el / 1e9 / HBM_PEAK_GBS}
    if roof:
        line["roofline"] = roof
    if tuned:
        line["autotune_stage_ms"] = tuned
    if not args.no_fp64_plain and prec == 32:
        ctxs = []
        try:
            ctxs, line["fp64_plain"] = fp64_plain(items, args.steps, args.integrator)
            line["fp32_batched_over_fp64_plain"] = value / line["fp64_plain"]["value"]
            log("fp64 plain: %.3e cell-DoF updates/s per stage (%d instances, %.3f s)" % (
                line["fp64_plain"]["value"], len(items), line["fp64_plain"]["seconds"]))
        except Exception as e:  # reported, not fatal
            line["fp64_plain"] = {"error": str(e)}
        if ctxs and args.workload == "c4" and args.integrator == "ssprk3":
            try:
                line["accuracy"] = c4_accuracy(items, ctxs, items[0][0]["steps"], ctx)
                log("accuracy: %s" % line["accuracy"])
            except Exception as e:  # reported, not fatal
                line["accuracy"] = {"error": str(e)}
        for c in ctxs:
            c.close()
    ctx.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(items, 12_000_000 if items[0][0]["dim"] == 2 else 2_000_000,
                                              args.integrator)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
