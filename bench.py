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
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s + HBM GB/s (FP64 vs FP32/batched); p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
# HBM bytes per stage launch measured with rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch; FETCH scaled by 2.0 and WRITE by 1.0, the
# factors a plain 1 GiB device copy gives), on the random-mode 256^3 grid,
# per launch shape (zseg, rotate, xcd): (w == 1, w < 1) pairs of (fetch KiB,
# write KiB), from `bench.py --sweep-shapes --calib-copy` under
# `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE`.  They describe the
# kernel sources whose hash is the key; after any change to those sources the
# figure is reported as null.
KERNEL_SOURCES = ("paper_2303_03026_amd/csrc/fused.hip", "paper_2303_03026_amd/csrc/device_mhd.h",
                  "paper_2303_03026_amd/csrc/kernels.h", "paper_2303_03026_amd/csrc/runtime.cpp")
MEASURED_TRAFFIC = {
    ("85fbb682025e7cf6", "f64"): {
        (1, 0, 0): ((2853971, 1180213), (3635124, 1180186)),
        (1, 0, 1): ((2711750, 1180135), (3556114, 1180210)),
        (1, 1, 0): ((2860358, 1179945), (3646867, 1180327)),
        (1, 1, 1): ((2697082, 1180012), (3551265, 1180446)),
        (2, 0, 0): ((3065565, 1179902), (3855293, 1180110)),
        (2, 0, 1): ((2943412, 1179929), (3803694, 1180104)),
        (2, 1, 0): ((3083797, 1179876), (3860799, 1180154)),
        (2, 1, 1): ((2930331, 1179949), (3782540, 1180241)),
        (4, 0, 0): ((3509365, 1179740), (4303084, 1179806)),
        (4, 0, 1): ((3175818, 1179747), (4059770, 1179807)),
        (4, 1, 0): ((3516348, 1179749), (4305320, 1179841)),
        (4, 1, 1): ((3151064, 1179784), (4069100, 1179847)),
    },
    ("85fbb682025e7cf6", "mixed"): {
        (1, 0, 0): ((1711248, 819487), (2175041, 819515)),
        (1, 0, 1): ((1570383, 819447), (2071591, 819548)),
        (1, 1, 0): ((1706729, 819438), (2170357, 819709)),
        (1, 1, 1): ((1570718, 819457), (2076652, 819708)),
        (2, 0, 0): ((1824812, 819363), (2300065, 819474)),
        (2, 0, 1): ((1702641, 819348), (2214107, 819452)),
        (2, 1, 0): ((1829813, 819384), (2308121, 819582)),
        (2, 1, 1): ((1707661, 819384), (2216199, 819553)),
        (4, 0, 0): ((2095719, 819257), (2557707, 819358)),
        (4, 0, 1): ((1824226, 819233), (2366593, 819338)),
        (4, 1, 0): ((2099225, 819257), (2563594, 819378)),
        (4, 1, 1): ((1822572, 819235), (2365448, 819349)),
    },
}
FETCH_CAL, WRITE_CAL = 2.0, 1.0


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision, tune, workload, n):
    """Counter bytes per stage launch (mean over one step's three stages),
    or None when no measurement matches the current kernel and shape."""
    if workload != "random_modes" or n != 256 or tune is None:
        return None
    m = MEASURED_TRAFFIC.get((kernel_hash(), precision), {}).get(tuple(tune))
    if m is None:
        return None
    per = [(f * FETCH_CAL + w * WRITE_CAL) * 1024.0 for f, w in m]
    return (per[0] + 2 * per[1]) / 3.0
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
                    help="weno5 / wenoz5 / mp5 / wenozp5 need 3 ghost layers: FP64 plain path only")
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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(the multi-GPU decomposition is a design note, not code)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2303_03026_amd import amrvac, inputs

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        bcopy = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        bcopy.copy_(a)
        torch.cuda.synchronize()
        print("bench: calibration copy of %d bytes done" % a.numel(), file=sys.stderr, flush=True)
        del a, bcopy
    print("bench: generating %d^3 %s input" % (args.n, args.workload), file=sys.stderr, flush=True)
    if args.workload == "random_modes":
        w = inputs.random_modes(args.n, 3, seed=1)
    elif args.workload == "current_sheet":
        w = inputs.current_sheet(n=args.n)
    elif args.workload == "kelvin_helmholtz":
        w = inputs.kelvin_helmholtz(max_level=args.levels)
    elif args.workload == "alfven_shock":
        w = inputs.alfven_shock_cloud(max_level=args.levels)
    else:
        w = inputs.shock_cloud_amr()
    w.limiter = LIMITERS.index(args.limiter)
    w.flux = {"hll": 0, "hlld": 1, "hllc": 2}[args.flux]
    mixed = args.precision == "mixed"
    w.ng = 2
    if w.limiter >= 3:  # the five-cell stencils: 3 ghost layers, FP64 (fused in 2D only)
        if mixed:
            sys.exit("bench: the fifth-order reconstructions run in FP64 only")
        w.ng = 3
        if w.ndim == 3:
            args.path = "plain"
    if mixed:
        args.path = "fused"
    path = amrvac.PATH_FUSED if args.path == "fused" else amrvac.PATH_PLAIN
    sim = amrvac.Simulation(w, path=path, precision=amrvac.FP32_MIXED if mixed else amrvac.FP64)
    state_bytes = 40.0 if mixed else 72.0
    stream = sim.stream
    if args.sweep_shapes:
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
    tune_times = {}
    if path == amrvac.PATH_FUSED and w.ng == 2 and args.tune != "default":
        if args.tune == "auto":
            print("bench: autotuning the fused stage", file=sys.stderr, flush=True)
            _, tune_times = sim.autotune(in_slot=0, out_slot=1, reps=3)
        else:
            sim.set_tune(*[int(v) for v in args.tune.split(",")])
    tune = sim.get_tune() if path == amrvac.PATH_FUSED and w.ng == 2 else None
    weights = [(0, 0, 1, 1.0), (1, 0, 2, 0.25), (2, 0, 0, 2.0 / 3.0)]

    def step(events=None):
        # the last stage folds the next step's CFL rate in (fused path), so
        # cfl() is then only the final reduction
        sim.cfl(0)
        for s, (i, b, o, wt) in enumerate(weights):
            sim.fill(i)
            if events is not None:
                events[s][0].record(stream)
            sim.stage(i, b, o, wt, cfl=(s == len(weights) - 1))
            if events is not None:
                events[s][1].record(stream)

    print("bench: warmup %d steps (path=%s)" % (args.warmup, args.path), file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    sim.sync_flags()

    K = args.steps
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(3)]
           for _ in range(K)]
    print("bench: timing %d steps" % K, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flags, nfix, last_dt, rc = sim.sync_flags(raise_on_error=False)
    if rc != 0:
        print("bench: non-physical state flagged (flags=%d)" % flags, file=sys.stderr)
        sys.exit(3)
    ms_per_step = (t1 - t0) * 1e3 / K
    cells = w.interior_cells
    value = cells * K / (t1 - t0) / 1e6

    # dominant kernel: the stage update (per-launch average over the timed region)
    stage_ms = [[evs[k][s][0].elapsed_time(evs[k][s][1]) for k in range(K)] for s in range(3)]
    avg_ms = sum(sum(x) for x in stage_ms) / (3 * K)
    # per cell: stage 1 reads in, writes out; stages 2 and 3 also read base
    bytes_per_launch = cells * state_bytes * (2 + 3 + 3) / 3.0
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9

    traffic = (measured_traffic(args.precision, tune, args.workload, args.n)
               if args.path == "fused" and args.limiter == "vanleer" and args.flux == "hll" else None)

    graph_ms = None
    if not args.no_graph_pass:
        sim.advance(2, graph=True)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        sim.advance(K, graph=True)
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - g0) * 1e3 / K
        sim.sync_flags()
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

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %dD, %d leaf blocks of 16^%d + %d ghost layers on %d level(s), %s GLM-MHD "
                               "state, SSPRK(3,3), CFL 0.8, %s, %s limiter, %s flux"
                               % (w.name, w.ndim, w.nblocks, w.ndim, w.ng, w.max_level, args.workload, "FP32-mixed" if mixed else "FP64",
                                  args.limiter, args.flux.upper()),
                   "path": args.path, "cells": cells, "stage_weights": [1.0, 0.25, 2.0 / 3.0],
                   "tune": None if tune is None else {"zseg": tune[0], "rotate": tune[1], "xcd": tune[2]}},
        "autotune_ms_per_launch": {"%d,%d,%d" % k: round(v, 4) for k, v in tune_times.items()},
        "algorithmic_hbm_gbs_per_step": cells * 8 * state_bytes / (ms_per_step * 1e-3) / 1e9,
        "graph_ms_per_step": graph_ms,
        "regrid": regrid,
        "lohner": lohner,
        "adaptive": adaptive,
        "stage_ms": [sum(x) / K for x in stage_ms],
        "roofline": {"bound": "hbm", "kernel": "stage (%s path)" % args.path, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
                     # the counter traffic of this launch shape over the live launch time
                     "traffic_gbs": None if traffic is None else traffic / (avg_ms * 1e-3) / 1e9,
                     "traffic_frac": None if traffic is None else traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
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
        small.limiter, small.flux, small.ng = w.limiter, w.flux, w.ng
        out["cpu_baseline"] = cpu_baseline(w, small)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
