"""Host logic of the continuous-batching scheduler, on the CPU with a fake
engine and a simulated clock (no GPU)."""
import numpy as np
import pytest

from paper_2309_09609_amd.serve import Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeEngine:
    """Records which chunk each request scores at each step; a step costs time
    proportional to the number of requests in it."""

    def __init__(self, clock, slot_bytes=100, step_cost=0.01):
        self.clock, self.slot_bytes, self.step_cost = clock, slot_bytes, step_cost
        self.log = []          # (step, rid, chunk)
        self.steps = 0
        self.sizes = []

    def new_slot(self):
        return object()

    def step(self, reqs, chunks, nchunks):
        assert len(set(id(r.slot) for r in reqs)) == len(reqs), "two active requests share a slot"
        for r, c in zip(reqs, chunks):
            self.log.append((self.steps, r.rid, c))
        self.sizes.append(len(reqs))
        self.steps += 1
        self.clock.t += self.step_cost * len(reqs)

    def topk(self, r):
        return r.rid

    def sync(self):
        pass

    def fetch(self, h):
        return ("top", h)


def run(nreq, nchunks, budget, arrivals):
    clock = FakeClock()
    eng = FakeEngine(clock)
    srv = Server(eng, nchunks=nchunks, mem_budget=budget)
    qs = [np.zeros(10 + i, np.int8) for i in range(nreq)]
    rep = srv.run(qs, arrivals, clock=clock, sleep=clock.sleep, cells_per_query=lambda q: q.size)
    return eng, srv, rep


@pytest.mark.parametrize("nchunks", [1, 3, 8])
def test_every_request_scores_every_chunk_once(nchunks):
    arr = np.linspace(0, 0.3, 25)
    eng, srv, rep = run(25, nchunks, 10 ** 6, arr)
    seen = {}
    for _, rid, c in eng.log:
        seen.setdefault(rid, []).append(c)
    assert sorted(seen) == list(range(25))
    for rid, cs in seen.items():
        assert sorted(cs) == list(range(nchunks)), rid
    assert set(rep.results) == set(range(25))
    assert all(rep.results[r] == ("top", r) for r in range(25))
    assert (rep.latencies > 0).all()


def test_admission_is_bounded_by_memory():
    arr = np.zeros(20)                        # everything arrives at once
    eng, srv, rep = run(20, 4, budget=350, arrivals=arr)   # 350 // 100 = 3 slots
    assert srv.max_slots == 3
    assert max(eng.sizes) <= 3 and rep.max_active == 3
    assert srv.allocated == 3                 # slots are recycled, never more than the budget
    assert set(rep.results) == set(range(20))
    assert rep.admitted_order == list(range(20))


def test_late_arrivals_join_requests_in_flight():
    """Continuous batching: a request arriving while others are mid-way joins the
    next iteration instead of waiting for them to finish."""
    arr = np.array([0.0, 0.0, 0.015, 0.035])
    eng, srv, rep = run(4, 8, 10 ** 6, arr)
    first_step = {}
    last_step = {}
    for s, rid, _ in eng.log:
        first_step.setdefault(rid, s)
        last_step[rid] = s
    assert first_step[2] > first_step[0] and first_step[2] < last_step[0]
    assert first_step[3] < last_step[0]
    assert max(eng.sizes) >= 3


def test_idle_server_waits_for_arrivals():
    arr = np.array([1.0, 5.0])
    eng, srv, rep = run(2, 2, 10 ** 6, arr)
    assert eng.steps == 4 and max(eng.sizes) == 1
    assert rep.latencies.max() < 0.1


def test_srpt_one_at_a_time_lets_short_requests_overtake():
    """max_active=1 with least-remaining-work order: preemptive shortest-first at
    chunk boundaries; every request still scores every chunk exactly once."""
    clock = FakeClock()
    eng = FakeEngine(clock)
    srv = Server(eng, nchunks=4, mem_budget=10 ** 6, max_active=1, policy="srpt")
    qs = [np.zeros(1000, np.int8), np.zeros(10, np.int8), np.zeros(400, np.int8)]   # 400 x 4 < 1000 x 2 left
    arr = np.array([0.0, 0.015, 0.015])      # the long one is one chunk in when the others arrive
    rep = srv.run(qs, arr, clock=clock, sleep=clock.sleep, cells_per_query=lambda q: q.size)
    assert max(eng.sizes) == 1 and rep.max_active == 1
    order = [rid for _, rid, _ in eng.log]
    assert order[:2] == [0, 0]                # the long request ran alone until the others arrived
    assert order[2:6] == [1, 1, 1, 1]         # then the shortest runs to completion
    assert order[6:10] == [2, 2, 2, 2] and order[10:] == [0, 0]
    seen = {}
    for _, rid, c in eng.log:
        seen.setdefault(rid, []).append(c)
    assert all(sorted(cs) == [0, 1, 2, 3] for cs in seen.values())
    assert rep.latencies[1] < rep.latencies[2] < rep.latencies[0]


# ------------------------------------------------------------------ length-paired FIFO (paired_run)
class FakeGpu:
    """A serial device: a unit starts when it is launched or when the previous one ends, whichever is
    later, and lasts its padded rows x ``row_cost`` (x ``pair_speedup`` for two queries)."""

    def __init__(self, clock, row_cost=1e-4, pair_speedup=0.9):
        self.clock, self.row_cost, self.pair_speedup = clock, row_cost, pair_speedup
        self.units = []                # [rids-as-lengths, start, end]
        self.end = 0.0
        self.inflight = 0
        self.max_inflight = 0
        self.slots = set()

    def launch(self, slot, queries):
        assert slot not in self.slots, "an output slot reused while in flight"
        self.slots.add(slot)
        now = self.clock()
        rows = max(q.size for q in queries) * len(queries)
        cost = rows * self.row_cost * (self.pair_speedup if len(queries) == 2 else 1.0)
        start = max(now, self.end)
        self.end = start + cost
        self.units.append(([q.size for q in queries], start, self.end))
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)
        return (slot, len(self.units) - 1, [int(q[0]) for q in queries])

    def done(self, h):
        return self.clock() >= self.units[h[1]][2]

    def fetch(self, h):
        assert self.done(h)
        self.slots.discard(h[0])
        self.inflight -= 1
        return [("top", tag) for tag in h[2]]


def paired(lengths, arrivals, ratio=0.85, depth=2, window=64):
    from paper_2309_09609_amd.serve import PairedFifo
    clock = FakeClock()
    gpu = FakeGpu(clock)
    qs = [np.full(int(m), i, np.int16) for i, m in enumerate(lengths)]   # first element tags the request
    rep = PairedFifo(gpu, ratio=ratio, depth=depth, window=window).run(
        qs, np.asarray(arrivals, float), clock=clock, sleep=clock.sleep, cells_per_query=lambda q: q.size)
    return gpu, rep


def test_paired_every_request_once_and_results_routed():
    rng = np.random.default_rng(5)
    lens = rng.integers(50, 2000, 60)
    arr = np.sort(rng.uniform(0, 3.0, 60))
    gpu, rep = paired(lens, arr)
    assert set(rep.results) == set(range(60))
    assert all(rep.results[r] == ("top", r) for r in range(60))
    assert sorted(rep.admitted_order) == list(range(60))
    assert (rep.latencies > 0).all()
    assert gpu.max_inflight <= 2 and gpu.inflight == 0


def test_paired_heads_in_arrival_order_and_pairs_within_ratio():
    rng = np.random.default_rng(6)
    lens = rng.integers(50, 2000, 80)
    arr = np.sort(rng.uniform(0, 2.0, 80))
    gpu, rep = paired(lens, arr, ratio=0.8)
    heads, i = [], 0
    for sizes, _, _ in gpu.units:
        heads.append(rep.admitted_order[i])
        if len(sizes) == 2:
            assert min(sizes) / max(sizes) >= 0.8
        i += len(sizes)
    order_rank = {int(r): k for k, r in enumerate(np.argsort(arr, kind="stable"))}
    assert [order_rank[h] for h in heads] == sorted(order_rank[h] for h in heads)
    assert rep.paired > 0


def test_paired_picks_the_closest_length():
    # everything waiting at once: 100 pairs with 95 (not 90), 300 with 290, 1000 runs alone
    gpu, rep = paired([100, 300, 95, 290, 1000, 90], np.zeros(6), ratio=0.85, depth=1)
    assert [sorted(u[0]) for u in gpu.units] == [[95, 100], [290, 300], [1000], [90]]
    assert rep.paired == 2


def test_paired_ratio_above_one_is_plain_fifo():
    rng = np.random.default_rng(7)
    lens = rng.integers(50, 2000, 40)
    arr = np.sort(rng.uniform(0, 1.0, 40))
    gpu, rep = paired(lens, arr, ratio=1.01)
    assert rep.paired == 0 and all(len(u[0]) == 1 for u in gpu.units)
    assert rep.admitted_order == [int(i) for i in np.argsort(arr, kind="stable")]


def test_paired_pipelining_keeps_the_device_busy():
    """With a backlog the next unit is queued before the running one ends: no idle gaps on the device
    after the first completion (depth 2), where one unit at a time leaves a poll interval per unit."""
    lens = np.full(30, 500)
    lens[::2] = 700                                  # no pairs at ratio 0.99
    arr = np.zeros(30)

    def idle(gpu):
        return sum(max(0.0, b[1] - a[2]) for a, b in zip(gpu.units[1:], gpu.units[2:]))
    g2, _ = paired(lens, arr, ratio=0.99, depth=2)
    g1, _ = paired(lens, arr, ratio=0.99, depth=1)
    assert g2.max_inflight == 2 and g1.max_inflight == 1
    assert idle(g2) < 1e-9 < idle(g1)
