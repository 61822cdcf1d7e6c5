"""Serving form: a request loop for coarsening jobs over resident compressed
graphs, with continuous batching.

A request names a resident graph and a seed; its job is the multilevel loop of
``coarsen`` (cluster, contract, repeat; Sections I and II-A of the paper).
The server keeps the compressed graphs on the device and works in steps. At
every step it admits the requests that have arrived, as long as a slot is free
and the job's device-memory estimate fits in what the budget has left; then it
runs one coarsening level for every active job at once: the current graphs of
all active jobs go through one batched clustering (one launch sequence for the
whole mix, grouped by representation: the resident graphs are compressed and
unweighted, the coarse levels plain and weighted), then every job contracts its own graph. Jobs that reach
their stop rule leave and free their slot and memory; requests that arrived
meanwhile join at the next step. A job's result does not depend on the mix:
the batched clustering gives every graph exactly the labels of a run alone,
and each job's seeds, caps and stop rule are its own.

Optionally, jobs are split by size into two such loops, each on its own host
thread and stream (big graphs, and the rest), so small jobs do not wait for
the levels of big ones and both share the device.

The sequential baseline runs the same requests one at a time in arrival order
(``coarsen`` per request). Both report throughput and latency percentiles of
completion time minus arrival time under the same arrival trace.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

from . import (Graph, coarsen, coarsen_params, lp_batch_cluster, lp_contract, memory_info)


def job_bytes(g: Graph) -> int:
    """Device-memory estimate of one coarsening job on g: clustering scratch
    (about 120 bytes per vertex), contraction records and the coarse graph
    (about 24 bytes per directed edge), with a factor 2 margin."""
    return 2 * (120 * g.n + 24 * g.two_m)


@dataclass
class Request:
    rid: int
    arrival: float   # seconds after the start of the run
    graph: int       # index into the resident pool
    seed: int


@dataclass
class Result:
    rid: int
    arrival: float
    start: float
    done: float
    levels: list = field(default_factory=list)  # per level: (n, two_m) of the clustered graph
    final_n: int = 0
    labels: list = field(default_factory=list)  # per level labels (kept when requested)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Job:
    req: Request
    cur: Graph
    owned: bool          # cur is a coarse level owned by the job
    n_target: int
    cap: int
    level: int
    est: int
    result: Result


def requests(trace) -> list[Request]:
    """Requests from (arrival, graph, seed) tuples."""
    return [Request(i, float(t), int(gi), int(sd)) for i, (t, gi, sd) in enumerate(trace)]


def _wait_until(t0: float, t: float) -> None:
    while True:
        d = t - (time.perf_counter() - t0)
        if d <= 0:
            return
        time.sleep(min(d, 0.002))


def run_sequential(pool: list[Graph], reqs: list[Request], rounds: int = 5, keep_labels: bool = False):
    """FIFO, one job at a time."""
    import torch

    out = []
    t0 = time.perf_counter()
    for r in sorted(reqs, key=lambda q: q.arrival):
        _wait_until(t0, r.arrival)
        start = time.perf_counter() - t0
        levels, final, _, _ = coarsen(pool[r.graph], seed=r.seed, rounds=rounds)
        torch.cuda.synchronize()
        res = Result(r.rid, r.arrival, start, time.perf_counter() - t0,
                     [(lv[0].n, lv[0].two_m) for lv in levels], final.n,
                     [lv[1].clone() for lv in levels] if keep_labels else [])
        for lv in levels[1:]:
            lv[0].free()
        if final is not pool[r.graph]:
            final.free()
        out.append(res)
    return out


class Server:
    """Continuous-batching server over a resident pool of graphs.

    With ``split_edges > 0`` jobs are split by size into two lanes: jobs on
    graphs with at least ``split_edges`` directed edges, and the rest. Each
    lane is its own continuous-batching loop on its own host thread and
    stream, so a step of small jobs never waits for the level of a big one,
    and the two lanes' kernels share the device; this lowers the median
    latency but costs throughput, so the default is one lane. The slot limit
    holds per lane; the memory budget is shared by the lanes.

    Admission charges every job its estimate (job_bytes) against the budget
    left after the resident graphs, and compares with the larger of the
    admitted jobs' estimates and the device memory the library actually holds
    (blocks in use, blocks its cache keeps for reuse, and blocks from a
    caller's allocator). Only a job that arrives while no job is active in
    any lane may exceed the budget on its own."""

    def __init__(self, pool: list[Graph], budget_bytes: int = 200 * 10**9, max_active: int = 64,
                 rounds: int = 5, max_levels: int = 32, keep_labels: bool = False, split_edges: int = 0):
        self.pool = pool
        self.budget = budget_bytes - sum(g.nbytes + 8 * (g.n + 1) for g in pool)
        self.max_active = max_active
        self.rounds = rounds
        self.max_levels = max_levels
        self.keep_labels = keep_labels
        self.split_edges = split_edges
        self.peak_active = 0
        self.steps = 0
        self._mu = threading.Lock()
        self._used = 0
        self._active = 0
        self.peak_used = 0  # largest sum of admitted estimates

    def run(self, reqs: list[Request]) -> list[Result]:
        if self.split_edges > 0:
            big = [r for r in reqs if self.pool[r.graph].two_m >= self.split_edges]
            lanes = [[r for r in reqs if self.pool[r.graph].two_m < self.split_edges], big]
        else:
            lanes = [list(reqs)]
        lanes = [ln for ln in lanes if ln]
        results: list[Result] = []
        errors: list[BaseException] = []
        t0 = time.perf_counter()

        def lane(rs):
            try:
                self._lane(rs, t0, results)
            except BaseException as e:  # re-raised by run()
                errors.append(e)

        threads = [threading.Thread(target=lane, args=(rs,)) for rs in lanes[1:]]
        for t in threads:
            t.start()
        if lanes:
            lane(lanes[0])
        for t in threads:
            t.join()
        if errors:
            raise errors[0]
        return sorted(results, key=lambda r: r.rid)

    def _admit(self, est: int) -> bool:
        with self._mu:
            if self._active > 0:
                m = memory_info()
                held = max(self._used, m["live"] + m["cached"] + m["external"])
                if held + est > self.budget:
                    return False
            self._used += est
            self._active += 1
            self.peak_active = max(self.peak_active, self._active)
            self.peak_used = max(self.peak_used, self._used)
            return True

    def _release(self, est: int) -> None:
        with self._mu:
            self._used -= est
            self._active -= 1

    def _lane(self, reqs: list[Request], t0: float, results: list) -> None:
        import torch

        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            pending = deque(sorted(reqs, key=lambda q: q.arrival))
            active: list[_Job] = []
            while pending or active:
                now = time.perf_counter() - t0
                # admission: arrived, a free slot, and the memory estimate fits
                while pending and pending[0].arrival <= now and len(active) < self.max_active:
                    r = pending[0]
                    g = self.pool[r.graph]
                    est = job_bytes(g)
                    if not self._admit(est):
                        break
                    pending.popleft()
                    n_target, cap = coarsen_params(g.n, g.total_vwgt)
                    active.append(_Job(r, g, False, n_target, cap, 0, est, Result(r.rid, r.arrival, now, 0.0)))
                if not active:
                    _wait_until(t0, pending[0].arrival)
                    continue
                with self._mu:
                    self.steps += 1
                # jobs already at their target leave without another level
                still = []
                for j in active:
                    if j.cur.n <= j.n_target or j.level >= self.max_levels:
                        self._finish(j, t0, results, stream)
                    else:
                        still.append(j)
                active = still
                if not active:
                    continue
                # one level for every active job: batched clustering per representation
                labels = {}
                kinds = sorted({(j.cur.compressed, j.cur.weighted) for j in active})
                for kind in kinds:
                    grp = [j for j in active if (j.cur.compressed, j.cur.weighted) == kind]
                    outs = lp_batch_cluster([j.cur for j in grp], [j.cap for j in grp], self.rounds,
                                            [j.req.seed + j.level for j in grp])
                    for j, lab in zip(grp, outs):
                        labels[id(j)] = lab
                still = []
                for j in active:
                    lab = labels[id(j)]
                    nxt, _ = lp_contract(j.cur, lab, want_map=False)
                    j.result.levels.append((j.cur.n, j.cur.two_m))
                    if self.keep_labels:
                        j.result.labels.append(lab.clone())
                    prev_n = j.cur.n
                    if j.owned:
                        j.cur.free()  # made on this stream: released in its order
                    j.cur, j.owned = nxt, True
                    j.level += 1
                    if 100 * j.cur.n > 95 * prev_n or j.cur.n <= j.n_target or j.level >= self.max_levels:
                        self._finish(j, t0, results, stream)
                    else:
                        still.append(j)
                active = still

    def _finish(self, j: _Job, t0: float, results: list, stream) -> None:
        stream.synchronize()
        j.result.final_n = j.cur.n
        j.result.done = time.perf_counter() - t0
        if j.owned:
            j.cur.free()
        self._release(j.est)
        with self._mu:
            results.append(j.result)


def summarize(results: list[Result]) -> dict:
    lat = sorted(r.latency for r in results)
    if not lat:
        return {}
    span = max(r.done for r in results) - min(r.arrival for r in results)

    def pct(p):
        k = min(len(lat) - 1, max(0, math.ceil(p / 100 * len(lat)) - 1))
        return lat[k]

    return {"requests": len(results), "throughput_per_s": len(results) / span if span > 0 else None,
            "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "mean_ms": 1e3 * sum(lat) / len(lat)}
