"""Seeded random cases through every entry point, against the oracle (tolerance
0): random alphabet sizes, int8 matrices (not necessarily symmetric, down to
-128), gap penalties, database and query lengths, tuning knobs and modes."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

CASES = range(10)


def _case(seed):
    rng = np.random.default_rng(9000 + seed)
    A = int(rng.choice([4, 20, 24]))
    lo = int(rng.choice([-128, -20, -4, 0]))
    hi = int(rng.choice([1, 5, 11, 60, 127]))
    sm = rng.integers(lo, hi + 1, size=(A, A)).astype(np.int8)
    if rng.random() < 0.5:
        sm = np.triu(sm) + np.triu(sm, 1).T                  # symmetric
    go = int(rng.choice([0, 1, 5, 10, 25, 200]))
    ge = int(rng.choice([0, 1, 2, 7, 30]))
    n = int(rng.integers(1, 300))
    lens = np.exp(rng.uniform(0, np.log(2500), n)).astype(np.int64)
    lens[rng.random(n) < 0.05] = 0
    res = rng.integers(0, A, int(lens.sum())).astype(np.int8)
    offs = np.zeros(n + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    queries = [rng.integers(0, A, int(m)).astype(np.int8) for m in rng.integers(1, 1200, 3)]
    # plant a stretch of a subject in the first query so some scores are large
    k = int(np.argmax(lens))
    if lens[k] > 20 and queries[0].size > 20:
        w = int(min(lens[k], queries[0].size) // 2)
        queries[0][:w] = res[offs[k]:offs[k] + w]
    knobs = dict(force_lanes=int(rng.choice([0, 1, 2, 8, 64])), rows_per_lane=int(rng.choice([0, 4, 8, 16])),
                 lane_pack=int(rng.choice([1, 2])))
    return A, sm, go, ge, res, offs, queries, knobs


@pytest.mark.parametrize("seed", CASES)
def test_random_case(gpu, seed):
    import torch
    A, sm, go, ge, res, offs, queries, knobs = _case(seed)
    ctx = f"seed {seed}: A={A} go/ge={go}/{ge} n={offs.size - 1} knobs={knobs}"
    D = gpu.Database(res, offs, alphabet=A, **knobs)
    want = [oracle.scores(q, res, offs, sm, go, ge) for q in queries]
    # one query at a time, local
    for q, w in zip(queries, want):
        got = D.search(q, sm, go, ge)
        torch.cuda.synchronize()
        assert (got.cpu().numpy().astype(np.int64) == w).all(), ctx
        ts, ti = gpu.topk(got, 7)
        ws, wi = oracle.topk(w, 7)
        assert (ts.cpu().numpy() == ws).all() and (ti.cpu().numpy() == wi).all(), ctx
    # all queries in one batched launch sequence
    scores, ts, ti = D.search_batch(queries, sm, go, ge, k=5)
    torch.cuda.synchronize()
    for r, w in enumerate(want):
        assert (scores[r].cpu().numpy().astype(np.int64) == w).all(), ctx + f" batch row {r}"
        ws, wi = oracle.topk(w, 5)
        assert (ts[r].cpu().numpy() == ws).all() and (ti[r].cpu().numpy() == wi).all(), ctx
    # end-to-end modes
    for mode in ("global", "semiglobal"):
        got = D.search(queries[1], sm, go, ge, mode=mode)
        torch.cuda.synchronize()
        w = oracle.scores(queries[1], res, offs, sm, go, ge, mode=mode)
        assert (got.cpu().numpy().astype(np.int64) == w).all(), ctx + " " + mode
    # alignments of the first query's top hits, against the oracle's choice
    top = [int(i) for i in oracle.topk(want[0], 3)[1] if i >= 0]
    for a, k in zip(D.align(queries[0], top, sm, go, ge), top):
        b = oracle.align(queries[0], res[offs[k]:offs[k + 1]], sm, go, ge)
        assert a["score"] == want[0][k] and all(a[key] == b[key] for key in ("score", "q_begin", "q_end", "s_begin", "s_end", "ops")), ctx
    D.close()
