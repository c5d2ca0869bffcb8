#!/usr/bin/env python3
"""Benchmark of the super-droplet coalescence step on one MI355X.

Default workload: the large domain -- 1024 x 1024 cells, Poisson(128) super-droplets
per cell (~134M SDs, injected empty and single-SD cells), bimodal lognormal radii,
geometric kernel, dt = 0.5 s -- with its state resident in HBM.  A step is one
coalescence step of every cell (sdm_coalesce_step: live count, shuffle, pairing,
collision update, all in one kernel launch for this cell-size range).

Prints ONE JSON line: pair tests/s over the timed steps, the roofline of the
dominant kernel (algorithmic bytes per launch / mean launch duration from HIP events
on the launch stream), and the FP64 CPU oracle timed on a bounded sample (all cores
the process may use, and one thread).  The same line carries the other workloads'
figures: us/step of the Golovin box and of the 2D domain, the batched ensemble
against per-instance plain launches, and the served stream's p50/p99 latency
against sequential plain launches (--headline-only skips them).

Other workloads (--workload): domain2d, box, ensemble (batched vs per-instance plain
launches), served (continuous batching vs sequential plain launches), transport
(particle transport with a re-sort by cell, then coalescence, every step).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coalescence pair tests/s + achieved HBM GB/s; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes: read xi and r of every SD (16 B), offset (4 B) and volume (8 B)
# of every cell, write both members of a colliding pair (2 x 16 B; most collisions
# change only xi_j and r_k, so this is the generous count)
BYTES_PER_SD = 16
BYTES_PER_CELL = 12
BYTES_PER_COLLISION = 32
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_wave_groups_large_domain.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "sq_k_wave_groups_large_domain.txt")
KERNEL_SOURCES = ["paper_1310_1905_amd/csrc/step_kernels.hpp",
                  "paper_1310_1905_amd/csrc/device_math.hpp"]


LAUNCH_FIELDS = ("group_slots", "groups_per_wave", "waves_per_block", "xcd_remap",
                 "block_slots", "block_split")


def launch_fields(text: str) -> dict:
    """--launch value (comma-separated, in LAUNCH_FIELDS order, a prefix of them) as keywords."""
    vals = [int(v) for v in text.split(",")]
    if not 1 <= len(vals) <= len(LAUNCH_FIELDS):
        raise SystemExit(f"--launch takes 1 to {len(LAUNCH_FIELDS)} values")
    return dict(zip(LAUNCH_FIELDS, vals))


def kernel_source_hash() -> str:
    """Hash of the step-kernel sources with // comments and blank lines removed, so
    that a profile stays matched to the code it measured across comment edits."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            lines = (re.sub(r"//.*$", "", x).rstrip() for x in f.read().splitlines())
        h.update("\n".join(x for x in lines if x).encode())
    return h.hexdigest()[:16]


def _profile_value(path: str, key: str):
    """A value from a committed rocprofv3 summary, if the summary was taken on the
    current kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals[key].split()[0])
    except (KeyError, ValueError, IndexError):
        return None


def measured_traffic():
    """HBM bytes per launch of the dominant kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE,
    calibrated with a copy kernel)."""
    return _profile_value(TRAFFIC_FILE, "hbm_bytes_per_launch")


def measured_valu_busy():
    """Fraction of the SIMDs' issue cycles the dominant kernel fills with VALU
    instructions (rocprofv3 SQ_INSTS_VALU, 4 cycles per wave64 instruction)."""
    return _profile_value(SQ_FILE, "valu_issue_busy_frac")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores() -> int:
    """Cores this process may run on: its CPU affinity, capped by OMP_NUM_THREADS
    when the host sets it (the share of the machine granted to the job)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _oracle_rate(pop, n_cells_sample: int, steps: int, threads: int):
    import oracle
    ncs = min(n_cells_sample, pop.n_cells)
    n_sd = int(np.count_nonzero(pop.cell < ncs))
    st = oracle.SlotState(pop.cell[:n_sd], pop.xi[:n_sd], pop.r[:n_sd], pop.dV[:ncs])
    kind = oracle.GEOMETRIC if pop.kernel == "geometric" else oracle.GOLOVIN
    t0 = time.perf_counter()
    for t in range(steps):
        if threads == 1:
            st.step(pop.dt, kind, pop.seed, t)
        else:
            st.step_parallel(pop.dt, kind, pop.seed, t, threads=threads)
    el = time.perf_counter() - t0
    return float(st.stats[0]) / el, ncs, n_sd, el


def cpu_baseline(pop, n_cells_sample: int, steps: int, single_cells: int):
    """The FP64 oracle as it stands, on all cores this process may use (threads
    over independent cell ranges; bit-identical to one thread), and on one thread
    over a smaller sample of the same domain."""
    cores = _host_cores()
    rate, ncs, n_sd, el = _oracle_rate(pop, n_cells_sample, steps, cores)
    rate1, ncs1, n_sd1, el1 = _oracle_rate(pop, single_cells, 1, 1)
    return {"value": rate, "unit": "pair tests/s", "cores": cores, "kind": "oracle",
            "sample": f"first {ncs} of {pop.n_cells} cells ({n_sd} SDs), {steps} steps, "
                      f"{el:.1f} s wall on {cores} threads",
            "single_thread_value": rate1,
            "single_thread_sample": f"first {ncs1} cells ({n_sd1} SDs), 1 step, {el1:.1f} s",
            "cpu_model": _cpu_model(), "host_cpus_visible": os.cpu_count()}


def calibration_copy(gib: float) -> int:
    """Three plain device copies of `gib` GiB, for scaling the HBM byte counters of a
    profile run; returns the bytes of one copy."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    return 8 * n


def bench_large(args):
    import torch

    from paper_1310_1905_amd import sdm, synth
    log("generating the 1024x1024-cell population")
    pop = synth.large_domain(seed=synth.SEEDS[0], nx=args.nx, ny=args.nx)
    log(f"{pop.n_sd} SDs in {pop.n_cells} cells; initialising")
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    ctx = sdm.Context(pop.cell, pop.xi, pop.r, pop.dV, stream=stream)
    if args.launch:
        ctx.set_launch_config(**launch_fields(args.launch))
    elif args.autotune:
        best = ctx.autotune(pop.dt, pop.kernel, seed=pop.seed ^ 0x5A5A, reps=8)
        log(f"autotuned launch config {best.as_dict()}")
    cfg = ctx.launch_config().as_dict()
    plan = ctx.plan()
    for t in range(args.warmup):
        ctx.step(pop.dt, pop.kernel, pop.seed, t)
    torch.cuda.synchronize()
    p0, c0 = ctx.stats()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        ctx.step(pop.dt, pop.kernel, pop.seed, args.warmup + i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p1, c1 = ctx.stats()
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    pairs = p1 - p0
    colls = c1 - c0
    log(f"{args.steps} steps in {wall * 1e3:.2f} ms; mean launch {launch_ms * 1e3:.1f} us; "
        f"{pairs} pair tests, {colls} collisions")
    alg_bytes = (BYTES_PER_SD * pop.n_sd + BYTES_PER_CELL * pop.n_cells
                 + BYTES_PER_COLLISION * colls / args.steps)
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": pairs / wall, "unit": "pair tests/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "large_domain_1024x1024_poisson128_geometric_dt0.5",
                   "n_sd": pop.n_sd, "n_cells": pop.n_cells, "parallelism": "single_gpu",
                   "groups": plan[0], "wave_cells": plan[1], "block_cells": plan[2],
                   "grid_cells": plan[3],
                   "launch": cfg},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_wave_groups", "algorithmic_bytes_per_launch": alg_bytes,
                     "mean_launch_ms": launch_ms,
                     "valu_issue_busy_frac": measured_valu_busy()},
    }
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    if args.calib_copy_gib > 0:
        out["calibration_copy_bytes"] = calibration_copy(args.calib_copy_gib)
    if args.cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(pop, args.cpu_cells, args.cpu_steps, args.cpu_cells_1t)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large",
                    choices=["large", "domain2d", "box", "ensemble", "served", "transport",
                             "extras"])
    ap.add_argument("--nx", type=int, default=1024, help="cells per side (large domain)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--cpu-cells", type=int, default=1 << 20)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--cpu-cells-1t", type=int, default=1 << 17,
                    help="cells of the single-thread oracle sample")
    ap.add_argument("--headline-only", dest="others", action="store_false",
                    help="skip the box, 2D-domain, ensemble and served figures of the "
                         "default run")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0)
    ap.add_argument("--instances", type=int, default=4096, help="ensemble size")
    ap.add_argument("--requests", type=int, default=200, help="served stream length")
    ap.add_argument("--served-requests", type=int, default=200,
                    help="served stream length of the headline run's served figures")
    ap.add_argument("--max-run", type=int, default=3600, help="longest served run (steps)")
    ap.add_argument("--served-loads", default="0.7",
                    help="served workload: arrival rates as fractions of the saturated rate, "
                         "comma-separated (the first one's figures are the line's)")
    ap.add_argument("--no-served-sequential", dest="served_sequential", action="store_false",
                    help="served workload: skip the one-at-a-time baseline")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="served HBM budget")
    ap.add_argument("--launch", default="",
                    help="fixed launch config group_slots,groups_per_wave,waves_per_block,"
                         "xcd_remap[,block_slots[,block_split]] for the large domain, the box "
                         "and the 2D domain (skips their autotuner)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is supported: the coalescence step would "
                                   "shard by cell ranges with no exchange, but no multi-GPU "
                                   "path is provided", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "large":
        out = bench_large(args)
        if args.others:
            from paper_1310_1905_amd import bench_workloads
            out.update(bench_workloads.secondary(args))
    else:
        from paper_1310_1905_amd import bench_workloads
        out = bench_workloads.run(args)
        if args.calib_copy_gib > 0:
            out["calibration_copy_bytes"] = calibration_copy(args.calib_copy_gib)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
