"""Continuous-batching server for independent GLM-MHD simulations.

Jobs (a grid, an initial state, a step count and a precision) arrive over
time.  The engine keeps one batch context per (dimension, precision) class,
each with a block pool carved from a fixed HBM budget; a job is admitted when
its class's pool has a contiguous free run for its blocks, stays resident on
the device, and is advanced
together with every other resident job of its class by one SSPRK step per
round.  The four classes run on their own streams, so their rounds overlap
on the device.  A job leaves as soon as its last step is done; the places it
frees are reused by the next admission.

Jobs that arrive together are queued largest (cells x steps) first, so that
a burst does not end with one long job running alone.  Initial states are
built on worker threads in queue order; admission never waits for one (a
job whose state is not ready yet is passed over until it is).  Admission
within a class is first come, first served with backfill: when the oldest
waiting job does not fit, later jobs of the class that do fit (among the
next `backfill_window` whose initial states are ready) are admitted ahead
of it, until the oldest has waited `max_head_wait_s`; from then on nothing
passes it, so every job is admitted within that wait plus the time for one
run of its size to free up.

Reported per run: per-job latency (completion minus arrival; p50, p99, max),
queueing delay, and the aggregate Mcell-updates/s of all jobs.
"""
from __future__ import annotations

import collections
import concurrent.futures
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import amrvac, inputs


def block_bytes(ndim: int, mixed: bool) -> int:
    pn = 16 + 4
    return pn ** ndim * (40 if mixed else 72)


class ServingEngine:
    """budget_bytes of HBM is split over the four job classes by the given
    shares; each class pool holds capacity = share * budget / (3 * block
    bytes) blocks (three state slots per block for SSPRK(3,3))."""

    CLASSES = [(2, False), (2, True), (3, False), (3, True)]

    def __init__(self, budget_bytes: float = 32e9, shares=(0.05, 0.05, 0.6, 0.3), max_jobs: int = 1024,
                 device: str = "cuda", prefetch_workers: int = 8, autotune: bool = True,
                 max_head_wait_s: float = 0.25, backfill_window: int = 32):
        import torch
        self.torch = torch
        self.max_head_wait_s = max_head_wait_s
        self.backfill_window = backfill_window
        self.device = device
        self.pools: Dict[tuple, amrvac.Batch] = {}
        self.capacity = {}
        for cls, share in zip(self.CLASSES, shares):
            ndim, mixed = cls
            cap = int(share * budget_bytes / (3 * block_bytes(ndim, mixed)))
            shape = inputs.random_modes(32, ndim, seed=0)
            self.pools[cls] = amrvac.Batch(shape, max(cap, 1), max_jobs, nstages=3,
                                           precision=amrvac.FP32_MIXED if mixed else amrvac.FP64, device=device)
            self.capacity[cls] = max(cap, 1)
            if autotune:
                self.pools[cls].set_tune(*self.tune_for(ndim, mixed))
        self.pool_exec = concurrent.futures.ThreadPoolExecutor(max_workers=prefetch_workers)

    def tune_for(self, ndim: int, mixed: bool):
        """Launch shape of a class's pool: the autotuner's choice on a
        representative resident set (a 128^3 grid in 3D, 512^2 in 2D, about
        the block count of a few dozen typical jobs)."""
        w = inputs.random_modes(128 if ndim == 3 else 512, ndim, seed=0)
        sim = amrvac.Simulation(w, path=amrvac.PATH_FUSED, precision=amrvac.FP32_MIXED if mixed else amrvac.FP64,
                                device=self.device)
        shape, _ = sim.autotune(reps=3)
        sim.close()
        return shape

    def close(self):
        for b in self.pools.values():
            b.close()
        self.pool_exec.shutdown(wait=False)

    @staticmethod
    def job_class(job) -> tuple:
        return (job["ndim"], bool(job["mixed"]))

    def run(self, jobs: List[dict], time_scale: float = 1.0, keep_results: Optional[set] = None,
            log_every: float = 10.0) -> dict:
        """Serve ``jobs`` (dicts from inputs.serving_jobs; arrival in seconds,
        multiplied by time_scale).  Returns latency/throughput statistics and
        the final states of the job ids in keep_results."""
        torch = self.torch
        # arrival order; among jobs that arrive together, the largest
        # (cells x steps) first, so that a burst does not end on a long job
        # left running alone
        order = sorted(range(len(jobs)),
                       key=lambda i: (jobs[i]["arrival"], -(jobs[i]["n"] ** jobs[i]["ndim"]) * jobs[i]["steps"]))
        futures = {}
        ahead = 64

        def prepare(job):
            # generate the job's initial state and pin it (worker thread), so
            # that admission queues its upload without a host wait
            w = inputs.serving_job_workload(job)
            w.prim = torch.from_numpy(np.ascontiguousarray(w.prim, dtype=np.float64)).pin_memory()
            return w

        for i in order[:ahead]:
            futures[i] = self.pool_exec.submit(prepare, jobs[i])
        next_prefetch = ahead
        queues = {cls: [] for cls in self.CLASSES}
        resident = {cls: {} for cls in self.CLASSES}  # job id in pool -> job index
        # steps left per resident job, kept here in step with the pool (every
        # round advances each resident job with steps left by one step)
        left = {cls: {} for cls in self.CLASSES}
        arrived = 0
        results = {}
        rec = {}
        cell_steps = 0.0
        t0 = time.perf_counter()
        last_log = t0
        pending_events = {cls: collections.deque() for cls in self.CLASSES}
        finishing = collections.deque()  # (event after a job's last step, job index)
        while (arrived < len(order) or finishing or any(queues[c] for c in self.CLASSES)
               or any(resident[c] for c in self.CLASSES)):
            now = time.perf_counter() - t0
            # arrivals
            while arrived < len(order) and jobs[order[arrived]]["arrival"] * time_scale <= now:
                i = order[arrived]
                queues[self.job_class(jobs[i])].append(i)
                rec[i] = {"arrival": jobs[i]["arrival"] * time_scale}
                arrived += 1
                if next_prefetch < len(order):
                    j = order[next_prefetch]
                    futures[j] = self.pool_exec.submit(prepare, jobs[j])
                    next_prefetch += 1
            # admissions: oldest first within each class, with backfill
            # while the oldest waiting job has waited less than the bound
            for cls in self.CLASSES:
                q = queues[cls]
                pool = self.pools[cls]
                k = 0
                while k < len(q) and k < self.backfill_window:
                    i = q[k]
                    if not futures[i].done():
                        # initial state still being built: never wait for it
                        # here (the device would idle); it is admitted once
                        # ready, in queue order among the ready ones
                        k += 1
                        continue
                    w = futures[i].result()
                    jid = pool.add_job(w)
                    if jid is None:
                        # no room: later ready jobs that fit pass it only
                        # while the oldest waiting job has waited less than
                        # the bound
                        head_wait = time.perf_counter() - t0 - rec[q[0]]["arrival"]
                        if head_wait >= self.max_head_wait_s:
                            break
                        k += 1
                        continue
                    del q[k]
                    resident[cls][jid] = i
                    left[cls][jid] = int(w.nsteps)
                    rec[i]["admitted"] = time.perf_counter() - t0
                    rec[i]["cells"] = w.interior_cells
                    del futures[i]
            # one round per class with resident unfinished jobs
            stepped = False
            for cls in self.CLASSES:
                pool = self.pools[cls]
                active = [jid for jid, n in left[cls].items() if n > 0]
                if not active:
                    continue
                pool.step()
                stepped = True
                for jid in active:
                    left[cls][jid] -= 1
                    cell_steps += rec[resident[cls][jid]]["cells"]
                ev = torch.cuda.Event()
                ev.record(pool.stream)
                pending_events[cls].append(ev)
                # bound the host's run-ahead to two rounds per class
                while len(pending_events[cls]) > 2:
                    pending_events[cls].popleft().synchronize()
            # completions: the job leaves the pool at once (a job placed in
            # its blocks is written behind its last step on the stream); its
            # completion time is taken when an event after that step fires
            for cls in self.CLASSES:
                pool = self.pools[cls]
                for jid in [j for j, n in left[cls].items() if n == 0]:
                    del left[cls][jid]
                    i = resident[cls].pop(jid)
                    if keep_results is not None and jobs[i]["id"] in keep_results:
                        results[jobs[i]["id"]] = pool.get_job(jid)
                    ev = torch.cuda.Event()
                    ev.record(pool.stream)
                    finishing.append((ev, i))
                    pool.remove_job(jid)
            now = time.perf_counter() - t0
            for _ in range(len(finishing)):
                ev, i = finishing.popleft()
                if ev.query():
                    rec[i]["done"] = now
                else:
                    finishing.append((ev, i))
            if not stepped:
                nxt = jobs[order[arrived]]["arrival"] * time_scale if arrived < len(order) else None
                if nxt is not None and not any(queues[c] for c in self.CLASSES):
                    time.sleep(max(0.0, min(0.01, nxt - (time.perf_counter() - t0))))
                elif finishing:
                    time.sleep(0.0002)
            if time.perf_counter() - last_log > log_every:
                last_log = time.perf_counter()
                ndone = sum(1 for r in rec.values() if "done" in r)
                print("serve: %d/%d done, %d resident, %.1f s" % (
                    ndone, len(jobs), sum(len(resident[c]) for c in self.CLASSES), last_log - t0), flush=True)
        for pool in self.pools.values():
            fl, nfix, rc = pool.sync_flags(raise_on_error=False)
            if rc != 0:
                raise RuntimeError("serving: non-physical state flagged (flags %d)" % fl)
        t_end = time.perf_counter() - t0
        lat = np.array([r["done"] - r["arrival"] for r in rec.values()])
        wait = np.array([r["admitted"] - r["arrival"] for r in rec.values()])
        return {
            "jobs": len(jobs),
            "wall_s": t_end,
            "mcell_updates_per_s": cell_steps / t_end / 1e6,
            "cell_steps": cell_steps,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_max_s": float(lat.max()),
            "queue_p50_s": float(np.percentile(wait, 50)),
            "queue_p99_s": float(np.percentile(wait, 99)),
            "results": results,
        }


def total_cell_steps(jobs: List[dict]) -> float:
    return float(sum((j["n"] ** j["ndim"]) * j["steps"] for j in jobs))


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serve a seeded stream of independent GLM-MHD jobs")
    ap.add_argument("--jobs", type=int, default=2000)
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of the saturated rate")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape in every pool")
    args = ap.parse_args(argv)
    jobs = inputs.serving_jobs(args.jobs, seed=args.seed, rate=1.0)
    eng = ServingEngine(budget_bytes=args.budget_gb * 1e9, autotune=not args.no_autotune)
    shapes = {"%dd_%s" % (c[0], "mixed" if c[1] else "f64"): eng.pools[c].get_tune() for c in eng.CLASSES}
    # saturated throughput: every job arrives at once
    sat = eng.run([dict(j, arrival=0.0) for j in jobs])
    rate_sat = len(jobs) / sat["wall_s"]
    # Poisson arrivals at load * saturated job rate (arrival times are drawn at rate 1)
    res = eng.run(jobs, time_scale=1.0 / (args.load * rate_sat))
    eng.close()
    for r in (sat, res):
        r.pop("results", None)
    print(json.dumps({"saturated": sat, "load": args.load, "served": res, "pool_launch_shapes": shapes}))


if __name__ == "__main__":
    main()
