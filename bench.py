"""Throughput benchmark of the GLM-MHD block hot path on one MI355X.

Default workload: 3D 256^3 periodic random-mode state held as 4096 blocks of
16^3 (+2 ghost layers), FP64, SSPRK(3,3), CFL 0.8.  One "step" is one full
SSPRK step: CFL reduction, then per stage a ghost fill and a stage update.

Prints ONE JSON line (rank 0) with Mcell-updates/s, the roofline of the
dominant kernel (its launches timed with HIP events on the library's stream
inside the timed region) and the CPU oracle timed on a bounded sample of the
same workload.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s + HBM GB/s (FP64 vs FP32/batched); p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 VALU instruction
# per 4 cycles per SIMD (16 lanes; FP64 add/mul/fma at full rate on gfx950)
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4.0
# Counter figures of the fused stage (rocprofv3 --pmc, per launch shape),
# committed under profiles/ as a JSON block, with the hash of the kernel
# sources they were taken from; a source change makes them unusable (null).
COUNTER_PROFILE = "profiles/stage_fused_counters_by_shape_random_modes_256.md"
KERNEL_SOURCES = ("paper_2303_03026_amd/csrc/fused.hip", "paper_2303_03026_amd/csrc/device_mhd.h",
                  "paper_2303_03026_amd/csrc/kernels.h")


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# The same for the fused stage with three ghost layers ('wenozp5' + HLLC on
# random modes 256^3): VALU wave-instructions per launch.
COUNTER_PROFILE5 = "profiles/stage_fused5_wave_states_random_modes_256.md"
KERNEL_SOURCES5 = tuple("paper_2303_03026_amd/csrc/" + f for f in (
    "fused5_stage.h", "fused5.hip", "fused5_hllc.hip", "fused5_hlld.hip", "device_mhd.h", "kernels.h"))


def kernel_hash5():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES5:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stage5_counters(precision, workload, n, limiter, flux):
    """(None, VALU wave-instructions per launch, the mean over one step's
    three stages) of the five-cell stage from the committed profile, or None
    when it does not match the kernel sources, the scheme or the grid."""
    if workload != "random_modes" or n != 256 or limiter != LIMITERS.index("wenozp5") or flux != 2:
        return None
    try:
        with open(os.path.join(ROOT, COUNTER_PROFILE5)) as f:
            prof = json.loads(f.read().split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if prof.get("kernel_sources_sha16") != kernel_hash5():
        return None
    rec = prof.get("valu_insts", {}).get(precision)
    if rec is None:
        return None
    return None, (rec["w1"] + 2 * rec["w_lt1"]) / 3.0


def stage_counters(precision, tune, workload, n):
    """Counter figures per stage launch of the fused stage for this launch
    shape, from the committed profile, as (fetch + write HBM bytes, VALU
    wave-instructions), each the mean over one step's three stages; None
    when no profile matches the current kernel sources and shape."""
    if workload != "random_modes" or n != 256 or tune is None:
        return None
    path = os.path.join(ROOT, COUNTER_PROFILE)
    try:
        with open(path) as f:
            text = f.read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        prof = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if prof.get("kernel_sources_sha16") != kernel_hash():
        return None
    rec = prof.get("shapes", {}).get(precision, {}).get("%d,%d,%d" % tuple(tune))
    if rec is None:
        return None
    fc, wc = prof["calibration"]["fetch"], prof["calibration"]["write"]
    # launches per step: one with w == 1, two with w < 1
    per = [(r["fetch_kib"] * fc + r["write_kib"] * wc) * 1024.0 for r in (rec["w1"], rec["w_lt1"])]
    valu = [r["valu_insts"] for r in (rec["w1"], rec["w_lt1"])]
    return (per[0] + 2 * per[1]) / 3.0, (valu[0] + 2 * valu[1]) / 3.0


# Algorithmic HBM bytes per cell for one stage launch: read the input state,
# write the output state, and read the base state when the stage weight is
# not 1; one state is 72 B per cell in FP64 and 40 B in FP32-mixed.


LIMITERS = ("vanleer", "koren", "cada3", "weno5", "wenoz5", "mp5", "wenozp5")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", choices=["plain", "fused"], default="fused")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", choices=["f64", "mixed"], default="f64",
                    help="f64: all FP64; mixed: FP32 storage and face arithmetic, FP64 energy and CFL")
    ap.add_argument("--workload", choices=["random_modes", "current_sheet", "shock_cloud", "kelvin_helmholtz",
                                           "alfven_shock"],
                    default="random_modes",
                    help="kelvin_helmholtz: the paper's 2D shear layer, 128 x 64 base with the interface band "
                         "refined to --levels levels (use with --limiter wenozp5 --flux hllc for its run); "
                         "alfven_shock: the paper's 2D MHD shock-cloud test, 128^2 base with the cloud and the "
                         "shock refined to --levels levels (use with --limiter koren and --flux hll/hllc/hlld)")
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--limiter", choices=list(LIMITERS), default="vanleer",
                    help="weno5 / wenoz5 / mp5 / wenozp5 run on 3 ghost layers (FP64 on both paths, FP32-mixed on the fused path)")
    ap.add_argument("--flux", choices=["hll", "hlld", "hllc"], default="hll")
    ap.add_argument("--regrid", action="store_true",
                    help="also time one regrid (coarsen the top level, refine every eighth block below)")
    ap.add_argument("--lohner", action="store_true",
                    help="also time the Loehner refinement indicator of the density (amrvac_lohner)")
    ap.add_argument("--adapt-every", type=int, default=0,
                    help="also run an adaptive segment of --steps steps that regrids every N steps from the "
                         "device Loehner indicator of the density (refine above 0.1, coarsen below 0.025, up to "
                         "--levels levels; the AMR workloads)")
    ap.add_argument("--tune", default="auto",
                    help="fused-stage launch shape: 'auto' (autotuner, before the warmup), 'default', or z,r,x")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other forms (plain FP64, FP32-mixed, current sheet, shock cloud, served)")
    ap.add_argument("--form-steps", type=int, default=20, help="timed steps of each other form")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="jobs of the served form (0: none)")
    ap.add_argument("--no-graph-pass", action="store_true")
    ap.add_argument("--sweep-shapes", action="store_true",
                    help="profiling helper: run one w=1 and one w<1 fused stage per launch shape, in the "
                         "autotuner's order, print the order and exit")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (calibrates HBM counters)")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, small):
    """The oracle (unchanged) on the host cores: one SSPRK(3,3) step of the
    full grid on all cores, reported as Mcell-updates/s; beside it, one
    thread on a smaller grid of the same construction (the per-cell work of
    a block does not depend on the grid size)."""
    from oracle import oracle
    cores = oracle.default_threads()
    sim = oracle.OracleSim(w, nthreads=cores)
    t0 = time.perf_counter()
    sim.steps(1)
    t1 = time.perf_counter()
    sim.close()
    one = oracle.OracleSim(small, nthreads=1)
    s0 = time.perf_counter()
    one.steps(2)
    s1 = time.perf_counter()
    one.close()
    return {"value": w.interior_cells / (t1 - t0) / 1e6, "unit": "Mcell-updates/s", "cores": cores,
            "kind": "oracle", "seconds": t1 - t0,
            "sample": "1 of the %d SSPRK(3,3) steps on the full %s grid (%d cells), OpenMP over blocks"
                      % (w.nsteps, w.name, w.interior_cells),
            "single_thread": {"value": 2 * small.interior_cells / (s1 - s0) / 1e6, "seconds": s1 - s0,
                              "sample": "2 SSPRK(3,3) steps of %s (%d cells), 1 thread"
                                        % (small.name, small.interior_cells)},
            "cpu_model": cpu_model()}


def make_workload(name, n=256, levels=6):
    from paper_2303_03026_amd import inputs
    if name == "random_modes":
        return inputs.random_modes(n, 3, seed=1)
    if name == "current_sheet":
        return inputs.current_sheet(n=n if n != 256 else 192)
    if name == "kelvin_helmholtz":
        return inputs.kelvin_helmholtz(max_level=levels)
    if name == "alfven_shock":
        return inputs.alfven_shock_cloud(max_level=levels)
    return inputs.shock_cloud_amr()


def roofline(avg_ms, bytes_per_launch, counters, kernel):
    """Roofline of the stage kernel over its live average launch time.  With
    the committed counter profile for these kernel sources and this launch
    shape, the bound is the VALU issue rate ("alu": VALU wave-instructions
    per launch from the profile over the launch time, against the 614.4 G/s
    issue peak), which is what limits the stage; the HBM view (algorithmic
    bytes per launch against 8 TB/s, and the profile's counter traffic) is
    kept beside it.  Without a matching profile only the HBM view exists."""
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic, valu = (None, None) if counters is None else counters
    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": bytes_per_launch,
           "traffic_frac": None if traffic is None else traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if valu is None:
        return dict(hbm, kernel=kernel, avg_launch_ms=avg_ms, valu=None)
    rate = valu / (avg_ms * 1e-3)
    return {"bound": "alu", "kernel": kernel, "achieved": rate, "peak": VALU_PEAK_WAVE_INSTS,
            "unit": "VALU wave-instructions/s", "frac": rate / VALU_PEAK_WAVE_INSTS, "traffic": traffic,
            "avg_launch_ms": avg_ms, "valu_wave_insts_per_launch": valu, "hbm": hbm}


def time_grid(w, path, mixed, steps, warmup, tune_mode="auto", graph_pass=False, keep=False, label=None):
    """Time `steps` SSPRK(3,3) steps of workload w (inputs in HBM before the
    timed region): per step the CFL reduction, then per stage a ghost fill
    and the stage, the last stage folding the next step's CFL rate in where
    it can.  Every stage launch is bracketed by HIP events on the library's
    stream.  Returns the form's record (and the simulation with keep)."""
    import torch
    from paper_2303_03026_amd import amrvac
    pth = amrvac.PATH_FUSED if path == "fused" else amrvac.PATH_PLAIN
    sim = amrvac.Simulation(w, path=pth, precision=amrvac.FP32_MIXED if mixed else amrvac.FP64)
    state_bytes = 40.0 if mixed else 72.0
    stream = sim.stream
    fused2 = pth == amrvac.PATH_FUSED and w.ng == 2
    tune_times = {}
    if fused2 and tune_mode != "default":
        if tune_mode == "auto":
            print("bench: autotuning the fused stage (%s)" % (label or w.name), file=sys.stderr, flush=True)
            _, tune_times = sim.autotune(in_slot=0, out_slot=1, reps=3)
        else:
            sim.set_tune(*[int(v) for v in tune_mode.split(",")])
    tune = sim.get_tune() if fused2 else None
    weights = [(0, 0, 1, 1.0), (1, 0, 2, 0.25), (2, 0, 0, 2.0 / 3.0)]

    def step(events=None):
        sim.cfl(0)
        for s, (i, b, o, wt) in enumerate(weights):
            sim.fill(i)
            if events is not None:
                events[s][0].record(stream)
            sim.stage(i, b, o, wt, cfl=(s == len(weights) - 1))
            if events is not None:
                events[s][1].record(stream)

    for _ in range(warmup):
        step()
    sim.sync_flags()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(3)]
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flags, nfix, last_dt, rc = sim.sync_flags(raise_on_error=False)
    if rc != 0:
        print("bench: non-physical state flagged (flags=%d)" % flags, file=sys.stderr)
        sys.exit(3)
    cells = w.interior_cells
    stage_ms = [[evs[k][s][0].elapsed_time(evs[k][s][1]) for k in range(steps)] for s in range(3)]
    avg_ms = sum(sum(x) for x in stage_ms) / (3 * steps)
    # per cell: stage 1 reads in and writes out; stages 2 and 3 also read base
    bytes_per_launch = cells * state_bytes * (2 + 3 + 3) / 3.0
    if fused2 and w.limiter == 0 and w.flux == 0:
        counters = stage_counters("mixed" if mixed else "f64", tune, w.workload_name, w.n_linear)
    elif pth == amrvac.PATH_FUSED and w.ng == 3:
        counters = stage5_counters("mixed" if mixed else "f64", w.workload_name, w.n_linear, w.limiter, w.flux)
    else:
        counters = None
    rec = {"workload": label or w.name, "path": path, "precision": "fp32-mixed" if mixed else "fp64",
           "blocks": int(w.nblocks), "cells": cells, "steps": steps, "warmup": warmup,
           "ms_per_step": (t1 - t0) * 1e3 / steps, "mcell_updates_per_s": cells * steps / (t1 - t0) / 1e6,
           "stage_ms": [sum(x) / steps for x in stage_ms],
           "roofline": roofline(avg_ms, bytes_per_launch, counters, "stage (%s path)" % path),
           "tune": None if tune is None else {"zseg": tune[0], "rotate": tune[1], "xcd": tune[2]},
           "autotune_ms_per_launch": {"%d,%d,%d" % k: round(v, 4) for k, v in tune_times.items()}}
    if graph_pass:
        sim.advance(2, graph=True)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        sim.advance(steps, graph=True)
        torch.cuda.synchronize()
        rec["graph_ms_per_step"] = (time.perf_counter() - g0) * 1e3 / steps
        sim.sync_flags()
    if keep:
        return rec, sim
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return rec


def served(njobs, load=0.8, budget_gb=32.0):
    """A short served stream of the serving mix (2D 32^2..256^2 and 3D
    32^3..128^3 random-mode jobs, 20..500 steps, half FP32-mixed): all jobs
    at once (the saturated rate), then Poisson arrivals at `load` times that
    rate; latency is completion minus arrival."""
    from paper_2303_03026_amd import inputs, serve
    jobs = inputs.serving_jobs(njobs, seed=4, rate=1.0)
    print("bench: serving %d jobs" % njobs, file=sys.stderr, flush=True)
    eng = serve.ServingEngine(budget_bytes=budget_gb * 1e9)
    sat = eng.run([dict(j, arrival=0.0) for j in jobs], log_every=5.0)
    rate_sat = len(jobs) / sat["wall_s"]
    res = eng.run(jobs, time_scale=1.0 / (load * rate_sat), log_every=5.0)
    eng.close()
    for r in (sat, res):
        r.pop("results", None)
    return {"workload": "serving mix, %d jobs (seed 4), %d GB pools" % (njobs, budget_gb),
            "saturated": {"wall_s": sat["wall_s"], "mcell_updates_per_s": sat["mcell_updates_per_s"],
                          "latency_p50_s": sat["latency_p50_s"], "latency_p99_s": sat["latency_p99_s"]},
            "load": load,
            "mcell_updates_per_s": res["mcell_updates_per_s"], "wall_s": res["wall_s"],
            "latency_p50_s": res["latency_p50_s"], "latency_p99_s": res["latency_p99_s"],
            "latency_max_s": res["latency_max_s"], "queue_p99_s": res["queue_p99_s"]}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU decomposition is a design note, not code)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2303_03026_amd import amrvac

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        bcopy = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        bcopy.copy_(a)
        torch.cuda.synchronize()
        print("bench: calibration copy of %d bytes done" % a.numel(), file=sys.stderr, flush=True)
        del a, bcopy
    print("bench: generating the %s input" % args.workload, file=sys.stderr, flush=True)
    w = make_workload(args.workload, args.n, args.levels)
    w.workload_name, w.n_linear = args.workload, args.n
    w.limiter = LIMITERS.index(args.limiter)
    w.flux = {"hll": 0, "hlld": 1, "hllc": 2}[args.flux]
    mixed = args.precision == "mixed"
    w.ng = 2
    if w.limiter >= 3:  # the five-cell stencils: 3 ghost layers
        w.ng = 3
    if mixed:
        args.path = "fused"
    if args.sweep_shapes:
        sim = amrvac.Simulation(w, path=amrvac.PATH_FUSED, precision=amrvac.FP32_MIXED if mixed else amrvac.FP64)
        order = amrvac.tune_candidates(3)
        sim.cfl(0)
        for shape in order:
            sim.set_tune(*shape)
            sim.fill(0)
            sim.stage(0, 0, 1, 1.0)
            sim.fill(1)
            sim.stage(1, 0, 2, 0.25)
        sim.sync_flags()
        sim.close()
        print(json.dumps({"sweep_shapes": order, "launches_per_shape": ["w=1", "w<1"]}), flush=True)
        return

    K = args.steps
    print("bench: headline form, %d warmup + %d timed steps (path=%s)" % (args.warmup, K, args.path),
          file=sys.stderr, flush=True)
    head, sim = time_grid(w, args.path, mixed, K, args.warmup, args.tune, graph_pass=not args.no_graph_pass,
                          keep=True, label=args.workload)
    workload_desc = ("%s: %dD, %d leaf blocks of 16^%d + %d ghost layers on %d level(s), %s GLM-MHD state, "
                     "SSPRK(3,3), CFL 0.8, %s, %s limiter, %s flux"
                     % (w.name, w.ndim, w.nblocks, w.ndim, w.ng, w.max_level, args.workload,
                        "FP32-mixed" if mixed else "FP64", args.limiter, args.flux.upper()))
    regrid = None
    if args.regrid:
        # one regrid of the current state: coarsen every top-level sibling
        # set, refine every eighth block of the level below (2:1 restored)
        top = int(w.level.max())
        flags = np.where(w.level == top, -1, np.where((w.level == top - 1) & (np.arange(w.nblocks) % 8 == 0), 1, 0))
        lv, ij = sim.regrid_plan(flags)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            new = sim.regrid(lv, ij)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - r0) * 1e3)
            new.close()
        regrid = {"ms": min(times), "blocks_in": int(w.nblocks), "blocks_out": int(len(lv)),
                  "cells_out": int(len(lv)) * w.nx ** w.ndim,
                  "what": "amrvac_regrid wall time (new context, tables, ghost fill of the old slot, "
                          "transfer kernel, stream sync), best of 3"}
    adaptive = None
    if args.adapt_every > 0:
        # an adaptive run: steps, and every N steps indicator -> plan -> regrid
        # (the new context keeps the launch shape); wall time of everything
        cur = sim
        cell_updates, regrids, t_ind, t_regrid = 0, 0, 0.0, 0.0
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        for k in range(K):
            cur.advance(1, nstages=3)
            cell_updates += int(len(cur.level)) * w.nx ** w.ndim
            if (k + 1) % args.adapt_every == 0 and k + 1 < K:
                torch.cuda.synchronize()  # (the steps so far are not charged to the regrid)
                r0 = time.perf_counter()
                flags = cur.lohner_flags(refine=0.1, coarsen_ratio=0.25, weights=[1.0] + [0.0] * 8)
                r1 = time.perf_counter()
                # (2D workloads may refine up to --levels; 3D ones keep their
                # deepest level, as eight children per refinement fill HBM fast)
                cap = max(args.levels, int(w.level.max())) if w.ndim == 2 else int(w.level.max())
                lv, ij = cur.regrid_plan(flags, max_level=cap)
                new = cur.regrid(lv, ij)
                if cur is not sim:
                    cur.close()
                cur = new
                t_ind += r1 - r0
                t_regrid += time.perf_counter() - r1
                regrids += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - a0
        adaptive = {"steps": K, "regrid_every": args.adapt_every, "regrids": regrids, "wall_s": wall,
                    "ms_per_step": wall * 1e3 / K, "mcell_updates_per_s": cell_updates / wall / 1e6,
                    "indicator_s": t_ind, "plan_and_regrid_s": t_regrid,
                    "blocks_start": int(w.nblocks), "blocks_end": int(len(cur.level)),
                    "what": "advance, then every N steps Loehner flags (device) -> plan (host) -> regrid (device); "
                            "cell updates counted on the grid of each step"}
        if cur is not sim:
            cur.close()
    lohner = None
    if args.lohner:
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            ind = sim.lohner(weights=[1.0] + [0.0] * 8, wavefilter=0.01)
            times.append((time.perf_counter() - r0) * 1e3)
        lohner = {"ms": min(times), "blocks": int(w.nblocks), "refine_above_0.2": int((ind > 0.2).sum()),
                  "what": "amrvac_lohner on the density, wall time (ghost fill, indicator kernel, copy of one "
                          "double per block to the host, stream sync), best of 5"}
    sim.close()
    del sim
    torch.cuda.empty_cache()

    # the other forms of the same path on the same GPU, each with its own
    # roofline (default run only: the benchmark's own workload, FP64 fused)
    forms = None
    default_run = (args.workload == "random_modes" and args.n == 256 and args.path == "fused" and not mixed
                   and args.limiter == "vanleer" and args.flux == "hll")
    if default_run and not args.no_forms:
        fk = max(5, min(K, args.form_steps))
        forms = {}
        print("bench: forms, %d timed steps each" % fk, file=sys.stderr, flush=True)
        forms["plain_fp64_random_modes_256"] = time_grid(w, "plain", False, max(3, fk // 4), 1,
                                                          label="random_modes_256")
        forms["fused_mixed_random_modes_256"] = time_grid(w, "fused", True, fk, args.warmup,
                                                          label="random_modes_256")
        for name in ("current_sheet", "shock_cloud"):
            wf = make_workload(name)
            wf.workload_name, wf.n_linear = name, 192 if name == "current_sheet" else 128
            label = "current_sheet_192" if name == "current_sheet" else "shock_cloud_amr_3levels"
            forms["fused_fp64_" + label] = time_grid(wf, "fused", False, fk, args.warmup, label=label)
            if name == "current_sheet":
                forms["fused_mixed_" + label] = time_grid(wf, "fused", True, fk, args.warmup, label=label)
        # the fifth-order reconstruction on the same grid (three ghost layers)
        w5 = dataclasses.replace(w, limiter=LIMITERS.index("wenozp5"), flux=2, ng=3)
        w5.workload_name, w5.n_linear = "random_modes", 256
        label = "random_modes_256_wenozp5_hllc"
        forms["fused_fp64_" + label] = time_grid(w5, "fused", False, fk, args.warmup, label=label)
        forms["fused_mixed_" + label] = time_grid(w5, "fused", True, fk, args.warmup, label=label)
        del w5
        if args.serve_jobs > 0:
            forms["served_mix"] = served(args.serve_jobs)

    out = {
        "metric": METRIC,
        "value": head["mcell_updates_per_s"],
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": workload_desc,
                   "path": args.path, "cells": head["cells"], "stage_weights": [1.0, 0.25, 2.0 / 3.0],
                   "tune": head["tune"]},
        "autotune_ms_per_launch": head["autotune_ms_per_launch"],
        "algorithmic_hbm_gbs_per_step": head["cells"] * 8 * (40.0 if mixed else 72.0)
        / (head["ms_per_step"] * 1e-3) / 1e9,
        "graph_ms_per_step": head.get("graph_ms_per_step"),
        "regrid": regrid,
        "lohner": lohner,
        "adaptive": adaptive,
        "stage_ms": head["stage_ms"],
        "roofline": head["roofline"],
        "forms": forms,
    }
    if not args.no_cpu_baseline:
        from paper_2303_03026_amd import inputs
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        wc = make_workload(args.workload, args.n, args.levels)
        if args.workload == "random_modes":
            small = inputs.random_modes(64, 3, seed=1)
        elif args.workload == "current_sheet":
            small = inputs.current_sheet(n=48)
        elif args.workload == "kelvin_helmholtz":
            small = inputs.kelvin_helmholtz(max_level=3)
        elif args.workload == "alfven_shock":
            small = inputs.alfven_shock_cloud(max_level=3)
        else:
            small = inputs.shock_cloud_amr(base_n=32)
        wc.limiter, wc.flux, wc.ng = LIMITERS.index(args.limiter), {"hll": 0, "hlld": 1, "hllc": 2}[args.flux], \
            (3 if LIMITERS.index(args.limiter) >= 3 else 2)
        small.limiter, small.flux, small.ng = wc.limiter, wc.flux, wc.ng
        out["cpu_baseline"] = cpu_baseline(wc, small)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
