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

``paired_run`` is first-come first-served with length-matched pairs: the
oldest waiting request is launched together with the waiting request of the
most similar length when the shorter is at least ``ratio`` of the longer, so
the two share lanes as a query pair (two 16-bit queries against one subject
per lane); otherwise it runs alone.  A pair of lengths m and r*m costs about
2m rows at the query-pair rate instead of (1 + r) m rows at the plain rate,
so pairing only pays for r near 1.  Launches are queued on the stream ahead
of the GPU (up to ``depth`` units in flight, the next one issued shortly
before the running one is expected to finish), so the GPU does not wait for
the host between requests; completion is seen through events, and the top-k
lists come back through pinned host memory.  With ``ratio`` above 1 it is
plain FIFO with the launches pipelined.

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
    paired: int = 0                    # units that carried two requests (paired_run)

    def summary(self) -> dict:
        lat = self.latencies
        return {"requests": int(lat.size), "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                "iterations": self.iterations, "max_active": self.max_active,
                "makespan_s": self.makespan, "gcups": self.cells / self.makespan / 1e9 if self.makespan > 0 else 0.0,
                "busy_gcups": self.cells / self.busy / 1e9 if self.busy > 0 else 0.0, "paired_units": self.paired}


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


class PairEngine:
    """Units of one or two queries through ``sw_search_batch_ws`` on a torch
    workspace (top-k only), results copied to pinned host memory, completion
    marked by an event; ``depth`` sets of output buffers."""

    def __init__(self, db, subst, gap_open=10, gap_extend=2, k=10, depth=2, stream=None):
        import torch
        import paper_2309_09609_amd as sw
        self.sw, self.torch, self.db = sw, torch, db
        self.subst, self.go, self.ge, self.k = db.matrix(subst), gap_open, gap_extend, k
        self.stream = stream if stream is not None else torch.cuda.current_stream(db.device)
        self.ws = None
        dev = db.device
        self.ts_d = [torch.empty((2, k), dtype=torch.int32, device=dev) for _ in range(depth)]
        self.ti_d = [torch.empty((2, k), dtype=torch.int64, device=dev) for _ in range(depth)]
        self.ts_h = [torch.empty((2, k), dtype=torch.int32, pin_memory=True) for _ in range(depth)]
        self.ti_h = [torch.empty((2, k), dtype=torch.int64, pin_memory=True) for _ in range(depth)]
        self.events = [torch.cuda.Event() for _ in range(depth)]

    def launch(self, slot, queries):
        qs = [np.ascontiguousarray(q, dtype=np.int8) for q in queries]
        qo = np.zeros(len(qs) + 1, dtype=np.int64)
        qo[1:] = np.cumsum([q.size for q in qs])
        need = self.sw.sw_batch_workspace_bytes(self.db.handle, qo, self.k, True)
        if self.ws is None or self.ws.numel() < need:
            self.ws = None                              # freed in stream order (same stream)
            with self.torch.cuda.stream(self.stream):
                self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.db.device)
        nq = len(qs)
        self.sw.sw_search_batch_ws(np.concatenate(qs), qo, self.db.handle, self.subst, self.go, self.ge, self.k,
                                   None, self.ts_d[slot], self.ti_d[slot], self.ws, self.stream)
        with self.torch.cuda.stream(self.stream):
            self.ts_h[slot][:nq].copy_(self.ts_d[slot][:nq], non_blocking=True)
            self.ti_h[slot][:nq].copy_(self.ti_d[slot][:nq], non_blocking=True)
        self.events[slot].record(self.stream)
        return slot, nq

    def done(self, handle):
        return self.events[handle[0]].query()

    def fetch(self, handle):
        slot, nq = handle
        self.events[slot].synchronize()
        ts, ti = self.ts_h[slot].numpy(), self.ti_h[slot].numpy()
        return [(ts[i].copy(), ti[i].copy()) for i in range(nq)]


class PairedFifo:
    """First-come first-served with length-matched pairs, launches pipelined
    (see the module docstring).

    ``ratio``: the shorter query of a pair is at least this fraction of the
    longer; ``window``: how many waiting requests behind the oldest are
    considered as its partner; ``depth``: units in flight; ``lead``: seconds
    before the running units' estimated end at which the next unit is issued
    (the estimate uses the padded rows of a unit, max length x queries, at the
    rate the retired units ran)."""

    def __init__(self, engine, ratio=0.85, depth=2, window=64, lead=0.02, poll=0.0005):
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.engine, self.ratio, self.depth, self.window = engine, float(ratio), int(depth), int(window)
        self.lead, self.poll = float(lead), float(poll)

    def _partner(self, waiting, lens):
        head = lens[waiting[0]]
        best, best_r = None, self.ratio
        for j in range(1, min(len(waiting), self.window + 1)):
            m = lens[waiting[j]]
            r = min(head, m) / max(head, m, 1)
            if r > best_r or (best is None and r >= best_r):
                best, best_r = j, r
        return best

    def run(self, queries, arrivals, clock=time.perf_counter, sleep=time.sleep, cells_per_query=None,
            progress=None) -> ServeReport:
        arrivals = np.asarray(arrivals, dtype=np.float64)
        order = [int(i) for i in np.argsort(arrivals, kind="stable")]
        lens = [int(np.asarray(q).size) for q in queries]
        n = len(order)
        lat = np.zeros(n)
        results, launch_order = {}, []
        waiting = []
        inflight = collections.deque()       # [handle, rids, rows, launched at, estimated end]
        rate = None                          # padded rows per second of the retired units
        busy, units, paired, biggest = 0.0, 0, 0, 0
        last_done = 0.0
        nxt = 0
        t0 = clock()
        while len(results) < n:
            now = clock() - t0
            while nxt < n and arrivals[order[nxt]] <= now:
                waiting.append(order[nxt])
                nxt += 1
            # issue the next unit: nothing in flight, or the last one is expected to end within `lead`
            while waiting and len(inflight) < self.depth and (
                    not inflight or (rate is not None and inflight[-1][4] - now <= self.lead)):
                j = self._partner(waiting, lens)
                rids = [waiting[0]] + ([waiting[j]] if j is not None else [])
                for r in sorted(([j] if j is not None else []) + [0], reverse=True):
                    waiting.pop(r)
                rows = max(lens[r] for r in rids) * len(rids)
                slot = units % self.depth
                h = self.engine.launch(slot, [queries[r] for r in rids])
                start = max(now, inflight[-1][4]) if inflight else now
                est_end = start + (rows / rate if rate else 0.0)
                inflight.append([h, rids, rows, now, est_end])
                launch_order.extend(rids)
                units += 1
                paired += len(rids) == 2
                biggest = max(biggest, len(rids))
            if inflight and self.engine.done(inflight[0][0]):
                h, rids, rows, launched, _ = inflight.popleft()
                out = self.engine.fetch(h)
                done = clock() - t0
                service = max(done - max(launched, last_done), 1e-9)
                busy += service
                last_done = done
                r_unit = rows / service
                rate = r_unit if rate is None else 0.7 * rate + 0.3 * r_unit
                for rid, res in zip(rids, out):
                    results[rid] = res
                    lat[rid] = done - arrivals[rid]
                # re-estimate the units still in flight from this completion
                t = done
                for u in inflight:
                    t = max(t, u[3]) + u[2] / rate
                    u[4] = t
                if progress:
                    progress(len(results), n)
                continue
            if not inflight and not waiting:
                if nxt < n:
                    sleep(max(0.0, arrivals[order[nxt]] - (clock() - t0)))
                continue
            sleep(self.poll)
        first = float(arrivals.min()) if n else 0.0
        cells = int(sum(cells_per_query(q) for q in queries)) if cells_per_query else 0
        makespan = float(max(lat[i] + arrivals[i] for i in range(n)) - first) if n else 0.0
        return ServeReport(lat, results, units, biggest, makespan, cells, launch_order, busy, paired)


def paired_run(db, queries, arrivals, subst, gap_open=10, gap_extend=2, k=10, ratio=0.85, depth=2, window=64,
               lead=0.02, clock=time.perf_counter, sleep=time.sleep, cells_per_query=None,
               progress=None) -> ServeReport:
    """Length-paired FIFO with pipelined launches on ``db`` (see the module
    docstring); ``db`` should be tuned for query pairs with at least two lanes
    per subject (``db.tune(lane_pack=2, force_lanes=2)``); results are the
    same either way."""
    eng = PairEngine(db, subst, gap_open, gap_extend, k, depth)
    return PairedFifo(eng, ratio, depth, window, lead).run(queries, arrivals, clock, sleep, cells_per_query, progress)
