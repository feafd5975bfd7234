"""Serving: continuous batching of protein queries against a resident database.

The database is dealt into ``nchunks`` interleaved chunks (the length-sorted
groups of 128 subjects go round-robin, so every chunk has the same length
mix).  A request is complete once it has scored every chunk.  The scheduler
runs iterations: one launch in which every active request scores its next
chunk.  Requests that arrive while others are on the GPU are admitted at the
next iteration boundary, as soon as a slot is free and the memory budget
(one score vector of n int32 per active request) allows, so their work
overlaps on the device with the requests already in flight.  When a request
has covered all chunks its top-k is taken and it retires, freeing its slot.
Under the oldest-first policy with no cap on active requests, every active
request runs in every iteration, so all of them score the same chunk (the
iteration count mod ``nchunks``); on a database tuned for query pairs
(``db.tune(lane_pack=2)``) they then share lanes two queries at a time.

``batch_run`` is dynamic batching: whenever the GPU is free, every waiting
request (up to ``max_batch``) is searched against the whole database in one
batched launch sequence, two queries per lane (query pairs), so a burst of
arrivals costs less GPU time than the same requests one by one.

``fifo_run`` is the plain baseline on the same arrival trace: one search per
request, in arrival order, each alone on the GPU.

Timing is wall-clock; latency = completion (top-k on the host) - arrival.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    query: np.ndarray
    arrival: float
    start_chunk: int = 0
    done_chunks: int = 0
    slot: object = None
    admitted: float = 0.0
    finished: float = 0.0


@dataclass
class ServeReport:
    latencies: np.ndarray
    results: dict                      # rid -> (top scores, top indices)
    iterations: int
    max_active: int
    makespan: float
    cells: int
    admitted_order: list = field(default_factory=list)
    busy: float = 0.0                  # seconds spent in iterations (launch to completion)

    def summary(self) -> dict:
        lat = self.latencies
        return {"requests": int(lat.size), "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                "iterations": self.iterations, "max_active": self.max_active,
                "makespan_s": self.makespan, "gcups": self.cells / self.makespan / 1e9 if self.makespan > 0 else 0.0,
                "busy_gcups": self.cells / self.busy / 1e9 if self.busy > 0 else 0.0}


class GpuEngine:
    """Engine on the HIP library: score vectors are torch tensors."""

    def __init__(self, db, subst, gap_open=10, gap_extend=2, k=10, stream=None):
        import torch
        import paper_2309_09609_amd as sw
        self.sw, self.torch = sw, torch
        self.db, self.subst, self.go, self.ge, self.k, self.stream = db, db.matrix(subst), gap_open, gap_extend, k, stream
        self.slot_bytes = 4 * max(db.n, 1)

    def new_slot(self):
        return self.torch.empty(max(self.db.n, 1), dtype=self.torch.int32, device=self.db.device)

    def step(self, reqs, chunks, nchunks):
        qs = [r.query for r in reqs]
        qo = np.zeros(len(qs) + 1, dtype=np.int64)
        qo[1:] = np.cumsum([q.size for q in qs])
        self.sw.sw_search_multi(np.concatenate(qs) if qs else np.zeros(0, np.int8), qo, chunks, nchunks,
                                self.db.handle, self.subst, self.go, self.ge, [r.slot for r in reqs], self.stream)

    def topk(self, req):
        return self.sw.topk(req.slot[: self.db.n], self.k, self.stream)

    def sync(self):
        self.torch.cuda.synchronize()

    def fetch(self, handle):
        ts, ti = handle
        return ts.cpu().numpy(), ti.cpu().numpy()


class Server:
    """Continuous-batching scheduler (see the module docstring)."""

    def __init__(self, engine, nchunks=8, mem_budget=2 << 30, max_slots=512, max_active=None, policy="fifo"):
        self.engine = engine
        self.nchunks = int(nchunks)
        self.max_slots = int(max(1, min(max_slots, mem_budget // max(engine.slot_bytes, 1))))
        # at most max_active admitted requests share one iteration; the others keep their slot and wait
        self.max_active = int(max_active) if max_active else self.max_slots
        # "fifo": oldest admitted first; "srpt": least remaining work (query length x chunks left) first,
        # so a short query that arrives can overtake long ones at the next chunk boundary
        if policy not in ("fifo", "srpt"):
            raise ValueError("policy must be 'fifo' or 'srpt'")
        self.policy = policy
        self.free = []                   # recycled score vectors
        self.allocated = 0

    def _slot(self):
        if self.free:
            return self.free.pop()
        self.allocated += 1
        return self.engine.new_slot()

    def run(self, queries, arrivals, clock=time.perf_counter, sleep=time.sleep, cells_per_query=None,
            progress=None) -> ServeReport:
        order = np.argsort(np.asarray(arrivals, dtype=np.float64), kind="stable")
        reqs = [Request(int(i), queries[int(i)], float(arrivals[int(i)])) for i in order]
        nxt = 0
        waiting = collections.deque()
        active = []
        results, admitted_order = {}, []
        iterations, max_active, it_counter = 0, 0, 0
        busy = 0.0
        t0 = clock()
        first_arrival = reqs[0].arrival if reqs else 0.0
        while len(results) < len(reqs):
            now = clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            while waiting and len(active) < self.max_slots:
                r = waiting.popleft()
                r.slot = self._slot()
                r.start_chunk = it_counter % self.nchunks
                r.admitted = now
                active.append(r)
                admitted_order.append(r.rid)
            if not active:
                if nxt < len(reqs):
                    sleep(max(0.0, reqs[nxt].arrival - (clock() - t0)))
                continue
            if self.policy == "srpt":
                running = sorted(active, key=lambda r: (r.query.size * (self.nchunks - r.done_chunks), r.arrival))
                running = running[: self.max_active]
            else:
                running = active[: self.max_active]
            t_it = clock()
            max_active = max(max_active, len(running))
            chunks = [(r.start_chunk + r.done_chunks) % self.nchunks for r in running]
            self.engine.step(running, chunks, self.nchunks)
            it_counter += 1
            iterations += 1
            finished = []
            for r in running:
                r.done_chunks += 1
                if r.done_chunks == self.nchunks:
                    finished.append((r, self.engine.topk(r)))
            self.engine.sync()
            busy += clock() - t_it
            now = clock() - t0
            for r, h in finished:
                results[r.rid] = self.engine.fetch(h)
                r.finished = now
                self.free.append(r.slot)
                r.slot = None
                if progress:
                    progress(len(results), len(reqs))
            active = [r for r in active if r.done_chunks < self.nchunks]
        lat = np.array([r.finished - r.arrival for r in sorted(reqs, key=lambda r: r.rid)])
        makespan = (max(r.finished for r in reqs) - first_arrival) if reqs else 0.0
        cells = int(sum(cells_per_query(r.query) for r in reqs)) if cells_per_query else 0
        return ServeReport(lat, results, iterations, max_active, makespan, cells, admitted_order, busy)


def fifo_run(db, queries, arrivals, subst, gap_open=10, gap_extend=2, k=10, clock=time.perf_counter,
             sleep=time.sleep, cells_per_query=None, progress=None) -> ServeReport:
    """Plain baseline: requests served one at a time in arrival order (sw_search + sw_topk)."""
    import torch
    import paper_2309_09609_amd as sw
    order = np.argsort(np.asarray(arrivals, dtype=np.float64), kind="stable")
    out = torch.empty(max(db.n, 1), dtype=torch.int32, device=db.device)
    lat = np.zeros(len(queries))
    results = {}
    busy = 0.0
    t0 = clock()
    last = 0.0
    for i in order:
        i = int(i)
        wait = arrivals[i] - (clock() - t0)
        if wait > 0:
            sleep(wait)
        t_it = clock()
        db.search(queries[i], subst, gap_open, gap_extend, out=out)
        ts, ti = sw.topk(out[: db.n], k)
        torch.cuda.synchronize()
        busy += clock() - t_it
        results[i] = (ts.cpu().numpy(), ti.cpu().numpy())
        last = clock() - t0
        lat[i] = last - arrivals[i]
        if progress:
            progress(len(results), len(queries))
    first = float(np.min(arrivals)) if len(arrivals) else 0.0
    cells = int(sum(cells_per_query(q) for q in queries)) if cells_per_query else 0
    return ServeReport(lat, results, len(queries), 1, last - first, cells, [int(i) for i in order], busy)


def batch_run(db, queries, arrivals, subst, gap_open=10, gap_extend=2, k=10, max_batch=16, clock=time.perf_counter,
              sleep=time.sleep, cells_per_query=None, progress=None) -> ServeReport:
    """Dynamic batching (see the module docstring).  ``db`` should be tuned for
    query pairs (``db.tune(lane_pack=2)``); results are identical either way."""
    import torch
    order = [int(i) for i in np.argsort(np.asarray(arrivals, dtype=np.float64), kind="stable")]
    lat = np.zeros(len(queries))
    results = {}
    busy, iterations, biggest = 0.0, 0, 0
    t0 = clock()
    nxt, last = 0, 0.0
    while nxt < len(order):
        now = clock() - t0
        if arrivals[order[nxt]] > now:
            sleep(max(0.0, arrivals[order[nxt]] - now))
            continue
        batch = []
        while nxt < len(order) and len(batch) < max_batch and arrivals[order[nxt]] <= clock() - t0:
            batch.append(order[nxt])
            nxt += 1
        t_it = clock()
        _, ts, ti = db.search_batch([queries[i] for i in batch], subst, gap_open, gap_extend, k=k, keep_scores=False)
        torch.cuda.synchronize()
        busy += clock() - t_it
        iterations += 1
        biggest = max(biggest, len(batch))
        ts, ti = ts.cpu().numpy(), ti.cpu().numpy()
        last = clock() - t0
        for r, i in enumerate(batch):
            results[i] = (ts[r], ti[r])
            lat[i] = last - arrivals[i]
        if progress:
            progress(len(results), len(queries))
    first = float(np.min(arrivals)) if len(arrivals) else 0.0
    cells = int(sum(cells_per_query(q) for q in queries)) if cells_per_query else 0
    return ServeReport(lat, results, iterations, biggest, last - first, cells, order, busy)
