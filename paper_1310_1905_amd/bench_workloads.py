"""Secondary benchmark workloads of bench.py (one JSON line each):

  domain2d -- 75 x 75 cells x 64 SDs, geometric kernel, dt = 1 s (latency-bound: us/step)
  box      -- one cell of 2^13 SDs, Golovin kernel, dt = 1 s (latency-bound: us/step)
  ensemble -- 4096 independent single-cell boxes (N_sd log-uniform 2^8..2^16), one
              graph-replayed batch step vs per-instance plain launches
  served   -- Poisson request stream served by continuous batching vs one request at a
              time with plain launches; p50/p99 latency
  extras   -- the large domain: step time under the release rules with recycling, and the
              per-cell moment, concentration and P_ij-probe kernels (HIP events)
  transport -- the large domain (1024 x 1024 cells of 20 m) with particle transport:
              single-eddy flow + sedimentation, re-sort by cell, then coalescence, every
              step; or the 2D domain with --nx 75
"""
from __future__ import annotations

import sys
import time

import numpy as np
import torch

from . import sdm, serve, synth

METRIC = "coalescence pair tests/s + achieved HBM GB/s; served p50/p99 latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _line(args, value, ms_per_step, workload, extra=None, unit="pair tests/s"):
    out = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": workload, "parallelism": "single_gpu"}}
    if extra:
        out["config"].update(extra)
    return out


def _single(args, pop, workload):
    stream = torch.cuda.Stream()
    ctx = sdm.Context(pop.cell, pop.xi, pop.r, pop.dV, stream=stream)
    if getattr(args, "launch", ""):
        fields = ("group_slots", "groups_per_wave", "waves_per_block", "xcd_remap",
                  "block_slots", "block_split")
        ctx.set_launch_config(**dict(zip(fields, (int(v) for v in args.launch.split(",")))))
    elif getattr(args, "autotune", True):
        ctx.autotune(pop.dt, pop.kernel, seed=pop.seed ^ 0x5A5A, reps=5)
    for t in range(args.warmup):
        ctx.step(pop.dt, pop.kernel, pop.seed, t)
    torch.cuda.synchronize()
    p0, _ = ctx.stats()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.step(pop.dt, pop.kernel, pop.seed, args.warmup + i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p1, _ = ctx.stats()
    cfg = ctx.launch_config().as_dict()
    ctx.close()
    return _line(args, (p1 - p0) / wall, wall * 1e3 / args.steps, workload,
                 {"n_sd": pop.n_sd, "n_cells": pop.n_cells, "us_per_step": wall * 1e6 / args.steps,
                  "launch": cfg})


def run_ensemble(args):
    pops = synth.ensemble(seed=synth.SEEDS[0], n_instances=args.instances)
    n_sd = sum(p.n_sd for p in pops)
    log(f"ensemble: {len(pops)} instances, {n_sd} SDs")
    b = sdm.Batch(n_sd, len(pops), len(pops))
    handles = [b.add(p.cell, p.xi, p.r, p.dV, p.kernel, p.dt, p.seed) for p in pops]
    if getattr(args, "launch", ""):
        fields = ("group_slots", "groups_per_wave", "waves_per_block", "xcd_remap", "block_slots")
        b.set_launch_config(**dict(zip(fields, (int(v) for v in args.launch.split(",")[:5]))))
        launch = b.launch_config().as_dict()
    else:
        launch = b.autotune(reps=3).as_dict() if getattr(args, "autotune", True) else None
    log(f"ensemble: batch launch config {b.launch_config().as_dict()}")
    for _ in range(args.warmup):
        b.step(use_graph=True)
    torch.cuda.synchronize()
    pt0 = sum(b.get(h, with_state=False)[2].pair_tests for h in handles)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.step(use_graph=True)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    pt1 = sum(b.get(h, with_state=False)[2].pair_tests for h in handles)
    batched = (pt1 - pt0) / wall_b
    # plain launches: one context per instance, one launch per instance and step
    plain_steps = max(2, args.steps // 20)
    stream = torch.cuda.Stream()
    ctxs = [sdm.Context(p.cell, p.xi, p.r, p.dV, stream=stream) for p in pops]
    for c, p in zip(ctxs, pops):
        c.step(p.dt, p.kernel, p.seed, 0)
    torch.cuda.synchronize()
    q0 = sum(c.stats()[0] for c in ctxs)
    t0 = time.perf_counter()
    for t in range(plain_steps):
        for c, p in zip(ctxs, pops):
            c.step(p.dt, p.kernel, p.seed, 1 + t)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t0
    q1 = sum(c.stats()[0] for c in ctxs)
    plain = (q1 - q0) / wall_p
    # equal accuracy: the same instance is bit-identical in both modes
    same = True
    for k in range(0, len(pops), max(1, len(pops) // 16)):
        ref = sdm.Context(pops[k].cell, pops[k].xi, pops[k].r, pops[k].dV, stream=stream)
        for t in range(args.warmup + args.steps):
            ref.step(pops[k].dt, pops[k].kernel, pops[k].seed, t)
        xa, ra = ref.state_numpy()
        xb, rb, _ = b.get(handles[k])
        same &= bool(np.array_equal(xa, xb.cpu().numpy().view(np.uint64)) and
                     np.array_equal(ra.view(np.uint64), rb.cpu().numpy().view(np.uint64)))
        ref.close()
    return _line(args, batched, wall_b * 1e3 / args.steps, "ensemble_4096_boxes_batched_graph",
                 {"n_sd": n_sd, "instances": len(pops), "launch": launch,
                  "plain_launch_pair_tests_per_s": plain,
                  "plain_ms_per_step": wall_p * 1e3 / plain_steps,
                  "speedup_vs_plain": batched / plain, "bit_identical_to_plain": same})


SERVED_MAX_REQUESTS = 200   # the stream length that has run cleanly


def _check_served_length(n: int):
    if n > SERVED_MAX_REQUESTS:
        raise ValueError(
            f"served streams of more than {SERVED_MAX_REQUESTS} requests are refused: one run "
            "of 2000 requests aborted with a corrupted host heap, whose cause is not found")


def run_served(args):
    """The served stream: its saturated rate (every request arriving at once), then
    Poisson arrivals at each load of --served-loads times that rate (0.7 by
    default), and the same requests one at a time at the first load unless
    --no-served-sequential.  The figures of the first load are the line's."""
    _check_served_length(args.requests)
    reqs = synth.request_stream(seed=synth.SEEDS[0], n_requests=args.requests, rate=1.0,
                                steps_hi=args.max_run)
    total_steps_sd = sum(q.pop.n_sd * q.pop.steps for q in reqs)
    log(f"served: {len(reqs)} requests, {total_steps_sd:.3g} SD-steps")
    # saturated throughput: everything arrives at once
    eng = serve.Engine(budget_bytes=int(args.budget_gib * (1 << 30)))
    t0 = time.perf_counter()
    res_sat = eng.run(reqs, time_scale=0.0)
    sat_wall = time.perf_counter() - t0
    eng.close()
    sat_rate = len(reqs) / sat_wall
    loads = [float(x) for x in str(getattr(args, "served_loads", "0.7")).split(",")]
    per_load = []
    for rho in loads:
        # Poisson arrivals at rho times the saturated request rate
        scale = 1.0 / (rho * sat_rate)
        eng = serve.Engine(budget_bytes=int(args.budget_gib * (1 << 30)))
        t0 = time.perf_counter()
        res = eng.run(reqs, time_scale=scale)
        wall = time.perf_counter() - t0
        eng.close()
        per_load.append({"load_vs_saturation": rho, "arrival_rate_per_s": 1.0 / scale,
                         "latency": serve.latency_summary(res),
                         "pair_tests_per_s": sum(r.pair_tests for r in res) / wall})
        log(f"served at {rho} of saturation: p50 {per_load[-1]['latency']['p50_s']:.3f} s, "
            f"p99 {per_load[-1]['latency']['p99_s']:.3f} s")
    first = per_load[0]
    extra = {"requests": len(reqs), "arrival_rate_per_s": first["arrival_rate_per_s"],
             "load_vs_saturation": first["load_vs_saturation"],
             "largest_request_sds": max(q.pop.n_sd for q in reqs),
             "saturated_requests_per_s": sat_rate,
             "latency": first["latency"],
             "saturated_pair_tests_per_s": sum(r.pair_tests for r in res_sat) / sat_wall}
    if len(per_load) > 1:
        extra["loads"] = per_load
    if getattr(args, "served_sequential", True):
        scale = 1.0 / (first["load_vs_saturation"] * sat_rate)
        t0 = time.perf_counter()
        seq = serve.run_sequential(reqs, time_scale=scale)
        wall_seq = time.perf_counter() - t0
        seq_rate = sum(r.pair_tests for r in seq) / wall_seq
        extra.update({"sequential_latency": serve.latency_summary(seq),
                      "sequential_pair_tests_per_s": seq_rate,
                      "speedup_vs_sequential": first["pair_tests_per_s"] / seq_rate})
    return _line(args, first["pair_tests_per_s"], None,
                 "served_poisson_stream_continuous_batching", extra)
def run_transport(args):
    """Transport + coalescence per step; the two parts timed separately with HIP events."""
    nx = args.nx
    d = 20.0
    pop = synth.large_domain(seed=synth.SEEDS[0], nx=nx, ny=nx) if nx > 75 else \
        synth.domain_2d(seed=synth.SEEDS[0], nx=nx, ny=nx)
    x, z = synth.positions_in_cells(pop, nx, nx, d, d, seed=5)
    stream = torch.cuda.Stream()
    ctx = sdm.Context(pop.cell, pop.xi, pop.r, pop.dV, stream=stream)
    ctx.attach_transport(x, z, nx, nx, d, d)
    cx, cz = synth.eddy_courant(nx, nx, d, d, pop.dt, w_max=2.0)
    cx_t = torch.as_tensor(cx, device="cuda")
    cz_t = torch.as_tensor(cz, device="cuda")
    ctx.set_launch_config(group_slots=256, groups_per_wave=8, waves_per_block=1)
    for t in range(args.warmup):
        ctx.transport(cx_t, cz_t, pop.dt, sediment=True)
        ctx.step(pop.dt, pop.kernel, pop.seed, t)
    torch.cuda.synchronize()
    p0, _ = ctx.stats()
    tr = []
    co = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        stream.synchronize()   # the previous coalescence step is not part of the transport time
        a = time.perf_counter()
        ctx.transport(cx_t, cz_t, pop.dt, sediment=True)   # synchronises (re-plan)
        b = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.step(pop.dt, pop.kernel, pop.seed, args.warmup + i)
        e1.record(stream)
        tr.append(b - a)
        co.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p1, _ = ctx.stats()
    co_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in co]))
    return _line(args, (p1 - p0) / wall, wall * 1e3 / args.steps,
                 f"transport_{nx}x{nx}_eddy_sedimentation_geometric",
                 {"n_sd": pop.n_sd, "n_cells": pop.n_cells,
                  "transport_ms_per_step": 1e3 * float(np.mean(tr)),
                  "coalescence_ms_per_step": co_ms})


def _timed(stream, fn, reps):
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))


def run_extras(args):
    """Costs of the rows beyond the plain step, on the large domain."""
    pop = synth.large_domain(seed=synth.SEEDS[0], nx=args.nx, ny=args.nx)
    stream = torch.cuda.Stream()
    ctx = sdm.Context(pop.cell, pop.xi, pop.r, pop.dV, stream=stream)
    ctx.set_launch_config(group_slots=256, groups_per_wave=8, waves_per_block=1)
    reps = max(3, args.steps)
    step = [0]

    def one_step():
        ctx.step(pop.dt, pop.kernel, pop.seed, step[0])
        step[0] += 1

    for _ in range(args.warmup):
        one_step()
    plain_ms = _timed(stream, one_step, reps)
    ctx.set_rules(sdm.RULE_RELEASE | sdm.RULE_RECYCLE)
    for _ in range(args.warmup):
        one_step()
    rules_ms = _timed(stream, one_step, reps)
    recycled = ctx.recycled()
    ctx.set_rules(0)
    n_sd, n_cells = pop.n_sd, pop.n_cells
    out_m = torch.empty(n_cells, dtype=torch.float64, device="cuda")
    out_c = torch.empty(n_cells, dtype=torch.int32, device="cuda")
    L = sdm.lib()
    torch.cuda.synchronize()
    mom_ms = _timed(stream, lambda: L.sdm_diag_moments(ctx._ctx, 3, 0.0, float("inf"), None,
                                                      out_m.data_ptr()), reps)
    conc_ms = _timed(stream, lambda: L.sdm_diag_sd_conc(ctx._ctx, out_c.data_ptr()), reps)
    probe_ms = _timed(stream, lambda: L.sdm_probe_probability(ctx._ctx, pop.dt, 1, pop.seed, 0,
                                                             None, None), reps)
    mom_bytes = 16 * n_sd + 12 * n_cells + 8 * n_cells
    conc_bytes = 8 * n_sd + 4 * n_cells + 4 * n_cells
    return _line(args, n_sd / (mom_ms * 1e-3), plain_ms, "extras_large_domain_1024x1024",
                 {"n_sd": n_sd, "n_cells": n_cells, "plain_step_ms": plain_ms,
                  "release_rules_recycling_step_ms": rules_ms, "recycled_slots": recycled,
                  "moments_ms": mom_ms, "moments_GBps": mom_bytes / (mom_ms * 1e-3) / 1e9,
                  "sd_conc_ms": conc_ms, "sd_conc_GBps": conc_bytes / (conc_ms * 1e-3) / 1e9,
                  "probe_ms": probe_ms},
                 unit="SDs/s (moment kernel)")


def secondary(args):
    """The figures of the other workloads for the headline line, each on its own
    small budget of steps: us/step of the box and the 2D domain, the batched
    ensemble against per-instance plain launches, the served stream's latency."""
    import argparse
    out = {}

    def sub(**kw):
        d = dict(vars(args))
        d.update(kw)
        return argparse.Namespace(**d)

    log("box: 8192 SDs, Golovin")
    box = _single(sub(steps=400, warmup=20), synth.box_golovin(seed=synth.SEEDS[0]),
                  "box_8192_golovin")
    out["box_us_per_step"] = box["config"]["us_per_step"]
    log("2D domain: 75 x 75 x 64 SDs, geometric")
    d2 = _single(sub(steps=400, warmup=20), synth.domain_2d(seed=synth.SEEDS[0]),
                 "domain_2d_75x75x64_geometric")
    out["domain2d_us_per_step"] = d2["config"]["us_per_step"]
    out["box_launch"] = box["config"]["launch"]
    out["domain2d_launch"] = d2["config"]["launch"]
    log("ensemble: 4096 boxes")
    ens = run_ensemble(sub(steps=30, warmup=3))
    c = ens["config"]
    out["ensemble"] = {"workload": c["workload"], "instances": c["instances"], "n_sd": c["n_sd"],
                       "launch": c["launch"], "ms_per_batch_step": ens["ms_per_step"],
                       "pair_tests_per_s": ens["value"],
                       "plain_ms_per_step": c["plain_ms_per_step"],
                       "plain_pair_tests_per_s": c["plain_launch_pair_tests_per_s"],
                       "speedup_vs_plain": c["speedup_vs_plain"],
                       "bit_identical_to_plain": c["bit_identical_to_plain"]}
    torch.cuda.empty_cache()
    log(f"served: {args.served_requests} requests")
    srv = run_served(sub(requests=args.served_requests, served_loads="0.7",
                         served_sequential=True))
    c = srv["config"]
    out["served"] = {"workload": c["workload"], "requests": c["requests"],
                     "largest_request_sds": c["largest_request_sds"],
                     "arrival_rate_per_s": c["arrival_rate_per_s"],
                     "load_vs_saturation": c["load_vs_saturation"],
                     "p50_s": c["latency"]["p50_s"], "p99_s": c["latency"]["p99_s"],
                     "pair_tests_per_s": srv["value"],
                     "sequential_p50_s": c["sequential_latency"]["p50_s"],
                     "sequential_p99_s": c["sequential_latency"]["p99_s"],
                     "sequential_pair_tests_per_s": c["sequential_pair_tests_per_s"],
                     "speedup_vs_sequential": c["speedup_vs_sequential"],
                     "saturated_pair_tests_per_s": c["saturated_pair_tests_per_s"]}
    return out


def run(args):
    if args.workload == "served":
        _check_served_length(args.requests)   # before any GPU work
    torch.cuda.set_device(0)
    if args.workload == "domain2d":
        return _single(args, synth.domain_2d(seed=synth.SEEDS[0]), "domain_2d_75x75x64_geometric")
    if args.workload == "box":
        return _single(args, synth.box_golovin(seed=synth.SEEDS[0]), "box_8192_golovin")
    if args.workload == "ensemble":
        return run_ensemble(args)
    if args.workload == "served":
        return run_served(args)
    if args.workload == "transport":
        return run_transport(args)
    if args.workload == "extras":
        return run_extras(args)
    raise ValueError(args.workload)
