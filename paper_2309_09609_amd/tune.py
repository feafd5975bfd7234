"""Autotuner for the batched search.

Tries lane packing (two subjects or two queries in the 16-bit halves of a
lane) and tiling and work-splitting choices of the sweep (rows per lane, the
size of a work unit relative to a persistent wave's share, a minimum number of
cooperating lanes per subject) on a sample of the caller's batch, keeps
only candidates whose scores are bit-identical to the first candidate's, and
picks the fastest.  Results are cached in a JSON file keyed by the GPU
architecture and a bucket of the workload shape, so later runs skip the search.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

# lane_pack 1: the two 16-bit halves of a lane hold two subjects; 2: two queries
DEFAULT_CANDIDATES = [
    dict(rows_per_lane=16, unit_share=250, force_lanes=0, lane_pack=1),
    dict(rows_per_lane=16, unit_share=250, force_lanes=2, lane_pack=1),
    dict(rows_per_lane=16, unit_share=100, force_lanes=2, lane_pack=1),
    dict(rows_per_lane=8, unit_share=250, force_lanes=0, lane_pack=1),
    dict(rows_per_lane=16, unit_share=250, force_lanes=0, lane_pack=2),
    dict(rows_per_lane=16, unit_share=250, force_lanes=2, lane_pack=2),
    dict(rows_per_lane=16, unit_share=100, force_lanes=2, lane_pack=2),
    dict(rows_per_lane=8, unit_share=250, force_lanes=2, lane_pack=2),
]


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "swsearch", "tune.json")


def shape_key(arch: str, n_subjects: int, qlens) -> str:
    """Bucket: arch, log2 of the subject count, batch size and mean query length."""
    q = np.asarray(qlens, dtype=np.float64)
    return f"{arch}|n2^{int(np.log2(max(n_subjects, 1)))}|nq2^{int(np.log2(max(q.size, 1)))}|m2^{int(np.log2(max(q.mean() if q.size else 1, 1)))}"


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _sample(queries, k: int, seed: int = 0):
    """Up to k queries spread over the length range of the batch, taken as k/2
    neighbours in length order, so that pairing queries by length in the sample
    looks like pairing them in the whole batch."""
    if len(queries) <= k:
        return list(queries)
    order = np.argsort([q.size for q in queries], kind="stable")
    anchors = np.linspace(0, len(order) - 2, max(k // 2, 1)).round().astype(int)
    pick = sorted(set(int(i) for a in anchors for i in (a, a + 1)))
    return [queries[order[i]] for i in pick]


def tune(db, queries, subst, gap_open=10, gap_extend=2, candidates=None, sample=8, repeats=2,
         cache_path: str | None = None, use_cache=True, verbose=False) -> dict:
    """Pick the fastest parity-passing knobs for ``db.search_batch`` on this
    batch shape, apply them to ``db`` and return
    ``{"knobs": ..., "gcups": ..., "trials": [...], "cached": bool}``."""
    import torch
    candidates = list(candidates or DEFAULT_CANDIDATES)
    cache_path = cache_path or default_cache_path()
    key = shape_key(_arch(), db.n, [q.size for q in queries])
    cache = {}
    if use_cache and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            db.tune(**cache[key]["knobs"])
            return dict(cache[key], cached=True)
    qs = _sample(queries, sample)
    cells = sum(int(q.size) for q in qs) * int(db.offsets[-1] - db.offsets[0])
    ref = None
    trials = []
    for c in candidates:
        db.tune(**c)
        scores, _, _ = db.search_batch(qs, subst, gap_open, gap_extend, k=0)   # warm-up, captures the graph
        torch.cuda.synchronize()
        got = scores.cpu().numpy()
        if ref is None:
            ref = got
        ok = bool(np.array_equal(got, ref))
        best = float("inf")
        for _ in range(repeats):
            t = time.perf_counter()
            db.search_batch(qs, subst, gap_open, gap_extend, k=0)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        trials.append(dict(knobs=c, parity=ok, seconds=best, gcups=cells / best / 1e9))
        if verbose:
            print(f"tune {c}: parity={ok} {cells / best / 1e9:.0f} GCUPS", flush=True)
    eligible = [t for t in trials if t["parity"]]
    win = max(eligible, key=lambda t: t["gcups"])
    db.tune(**win["knobs"])
    out = dict(knobs=win["knobs"], gcups=win["gcups"], trials=trials, key=key)
    if use_cache:
        cache[key] = dict(knobs=win["knobs"], gcups=win["gcups"], key=key)
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return dict(out, cached=False)
