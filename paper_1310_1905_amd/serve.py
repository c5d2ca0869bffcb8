"""Continuous-batching request loop over the batch ABI (sdm_batch_*).

Requests (coalescence runs of different sizes and lengths) arrive over time.  The
engine keeps every admitted request's super-droplet state resident in HBM inside one
batch, admits waiting requests in arrival order whenever their SDs, cells and an
instance slot fit in the batch's capacity (the HBM budget), advances every admitted
request by one step per iteration in a single (graph-replayed) launch sequence, and
retires a request as soon as it has done its run length.  Work of requests that
arrived at different times therefore overlaps on the device.

Because the random numbers are keyed by each request's own (seed, step, cell,
slot), a request's result is bit-identical alone and in any mix.

The comparison baseline, ``run_sequential``, serves the same requests one at a time
in arrival order, each with plain per-step launches on its own context.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import sdm


@dataclass
class Result:
    index: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    pair_tests: int
    xi: np.ndarray | None = None
    r: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def budget_capacity(budget_bytes: int, max_instances: int, cells_per_sd: float = 0.01):
    """Largest (max_sd, max_cells) whose batch workspace fits in budget_bytes."""
    lo, hi = 1, 1 << 31
    L = sdm.lib()
    while lo < hi:
        mid = (lo + hi + 1) // 2
        cells = max(1024, int(mid * cells_per_sd))
        if L.sdm_batch_workspace_bytes(mid, cells, max_instances) <= budget_bytes:
            lo = mid
        else:
            hi = mid - 1
    return lo, max(1024, int(lo * cells_per_sd))


class Engine:
    """use_graph: replay a captured graph of the batch step.  Off by default: the
    step is GPU-bound (a replay and an eager step of a served batch take the same
    time), while the set of requests changes every few iterations, and each change
    would capture and instantiate the graph again."""

    def __init__(self, budget_bytes: int, max_instances: int = 1024, keep_state: bool = False,
                 use_graph: bool = False):
        max_sd, max_cells = budget_capacity(budget_bytes, max_instances)
        self.batch = sdm.Batch(max_sd, max_cells, max_instances)
        self.capacity = (max_sd, max_cells, max_instances)
        self.keep_state = keep_state
        self.use_graph = use_graph
        self.iterations = 0

    def run(self, requests, time_scale: float = 1.0, log=None):
        """Serve ``requests`` (objects with .arrival and .pop) in wall-clock time;
        arrival times are multiplied by time_scale.  Returns the list of Results."""
        order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        pending = list(order)
        waiting = []
        live = {}             # handle -> (index, admitted_at, steps_left)
        results = []
        max_sd, max_cells, _ = self.capacity
        for i in order:
            p = requests[i].pop
            if p.n_sd > max_sd or p.n_cells > max_cells:
                raise ValueError(f"request {i} can never fit in the batch capacity")
        t0 = time.perf_counter()
        while pending or waiting or live:
            now = time.perf_counter() - t0
            while pending and requests[pending[0]].arrival * time_scale <= now:
                waiting.append(pending.pop(0))
            # admission in arrival order, while capacity allows
            while waiting:
                i = waiting[0]
                p = requests[i].pop
                try:
                    h = self.batch.add(p.cell, p.xi, p.r, p.dV, p.kernel, p.dt, p.seed)
                except sdm.SdmError as e:
                    if e.status == -5:     # capacity: wait for retirements
                        break
                    raise
                waiting.pop(0)
                live[h] = (i, time.perf_counter() - t0, p.steps)
            if not live:
                if pending:
                    wait = requests[pending[0]].arrival * time_scale - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            # one step of every admitted request; retire the finished ones
            self.batch.step(use_graph=self.use_graph)
            self.iterations += 1
            finished = []
            for h, (i, adm, left) in live.items():
                left -= 1
                live[h] = (i, adm, left)
                if left == 0:
                    finished.append(h)
            for h in finished:
                i, adm, _ = live.pop(h)
                _, _, cnt = self.batch.get(h, with_state=False)
                xi, r = self.batch.remove(h, with_state=self.keep_state)
                done = time.perf_counter() - t0
                res = Result(i, requests[i].arrival * time_scale, adm, done, cnt.steps_done,
                             cnt.pair_tests)
                if self.keep_state:
                    res.xi = xi.cpu().numpy().view(np.uint64)
                    res.r = r.cpu().numpy()
                results.append(res)
                if log:
                    log(f"request {i} done: latency {res.latency:.3f} s")
        return results

    def close(self):
        self.batch.close()


def run_sequential(requests, time_scale: float = 1.0, keep_state: bool = False):
    """The same requests one at a time in arrival order, plain per-step launches."""
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
    stream = torch.cuda.Stream()
    results = []
    t0 = time.perf_counter()
    for i in order:
        q = requests[i]
        now = time.perf_counter() - t0
        if q.arrival * time_scale > now:
            time.sleep(q.arrival * time_scale - now)
        adm = time.perf_counter() - t0
        p = q.pop
        ctx = sdm.Context(p.cell, p.xi, p.r, p.dV, stream=stream)
        for t in range(p.steps):
            ctx.step(p.dt, p.kernel, p.seed, t)
        pairs, _ = ctx.stats()
        res = Result(i, q.arrival * time_scale, adm, 0.0, p.steps, pairs)
        if keep_state:
            res.xi, res.r = ctx.state_numpy()
        else:
            torch.cuda.synchronize()
        res.finished = time.perf_counter() - t0
        ctx.close()
        results.append(res)
    return results


def latency_summary(results):
    lat = np.array([r.latency for r in results])
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "n": int(lat.size)}
