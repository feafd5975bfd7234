"""Autotuner for the batched search.

Tries lane packing (two subjects or two queries in the 16-bit halves of a
lane) and tiling and work-splitting choices of the sweep (rows per lane, the
size of a work unit relative to a persistent wave's share, a minimum number of
cooperating lanes per subject) on a sample of the caller's batch and picks the
fastest candidate that passes the parity gate:

* every candidate's scores of a sample of subjects (the longest, the
  shortest and some in between) must equal the scores the library's
  alignment kernel computes for the same pairs -- a separate kernel that
  fills Eq. 1-3 in 32-bit cells, independent of every 16-bit tiling tried;
* when the caller passes ``verify`` (for instance a check against a CPU
  reference), every candidate must pass it as well.

No candidate passing is an error.  The winner is cached in memory per process
and, when ``cache_path`` is given, in a JSON file keyed by the GPU
architecture, the workload's shape, the substitution matrix and the gap
penalties.
"""
from __future__ import annotations

import hashlib
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

_memory_cache: dict = {}


def shape_key(arch: str, n_subjects: int, qlens, subst=None, gap_open=None, gap_extend=None) -> str:
    """Bucket: arch, log2 of the subject count, batch size and mean query length, plus a hash of the
    substitution matrix and the gap penalties (knobs are reused only for the same scoring setup)."""
    q = np.asarray(qlens, dtype=np.float64)
    key = (f"{arch}|n2^{int(np.log2(max(n_subjects, 1)))}|nq2^{int(np.log2(max(q.size, 1)))}"
           f"|m2^{int(np.log2(max(q.mean() if q.size else 1, 1)))}")
    if subst is not None:
        sm = np.ascontiguousarray(np.asarray(subst, dtype=np.int8))
        key += f"|sm{hashlib.sha1(sm.tobytes()).hexdigest()[:12]}x{sm.size}|g{gap_open}/{gap_extend}"
    return key


def _arch() -> str:
    try:
        import torch
        if torch.cuda.is_available():
            p = torch.cuda.get_device_properties(torch.cuda.current_device())
            return getattr(p, "gcnArchName", p.name).split(":")[0]
    except ImportError:
        pass
    return "cpu"


def _sync():
    import torch
    if torch.cuda.is_available():
        torch.cuda.synchronize()


def _numpy(x) -> np.ndarray:
    return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)


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


def sample_subjects(offsets, count: int = 48, seed: int = 0) -> np.ndarray:
    """Subjects whose scores gate a candidate: the longest (cooperating lanes, many
    passes), the shortest (padding, empty subjects) and random ones in between."""
    lens = np.diff(np.asarray(offsets, dtype=np.int64))
    n = lens.size
    if n <= count:
        return np.arange(n, dtype=np.int64)
    order = np.argsort(-lens, kind="stable")
    k = max(count // 4, 1)
    rng = np.random.default_rng(seed)
    mid = rng.choice(order[k:n - k], size=count - 2 * k, replace=False)
    return np.unique(np.concatenate([order[:k], order[n - k:], mid])).astype(np.int64)


def reference_scores(db, qs, subst, gap_open, gap_extend, idx) -> np.ndarray:
    """[len(qs), len(idx)] scores from the library's 32-bit alignment kernel."""
    al = db.align_batch(qs, [idx] * len(qs), subst, gap_open, gap_extend)
    return np.array([[a["score"] for a in row] for row in al], dtype=np.int64).reshape(len(qs), len(idx))


def tune(db, queries, subst, gap_open=10, gap_extend=2, candidates=None, sample=8, repeats=2,
         cache_path: str | None = None, use_cache=True, verify=None, subjects=48, verbose=False) -> dict:
    """Pick the fastest parity-passing knobs for ``db.search_batch`` on this
    batch shape, apply them to ``db`` and return
    ``{"knobs", "gcups", "trials", "key", "cached", "gate"}``.

    ``verify(query_index, scores_row) -> bool``, if given, is called for every
    sampled query of every candidate with that query's full score row."""
    candidates = list(candidates or DEFAULT_CANDIDATES)
    key = shape_key(_arch(), db.n, [q.size for q in queries], subst, gap_open, gap_extend)
    cache = {}
    if use_cache:
        if cache_path and os.path.exists(cache_path):
            try:
                cache = json.load(open(cache_path))
            except (OSError, ValueError):
                cache = {}
        hit = cache.get(key) or _memory_cache.get(key)
        if hit:
            db.tune(**hit["knobs"])
            return dict(hit, cached=True)
    qs = _sample(queries, sample)
    idx = sample_subjects(db.offsets, subjects)
    ref = reference_scores(db, qs, subst, gap_open, gap_extend, idx) if idx.size and qs else None
    cells = sum(int(q.size) for q in qs) * int(db.offsets[-1] - db.offsets[0])
    trials = []
    for c in candidates:
        db.tune(**c)
        scores, _, _ = db.search_batch(qs, subst, gap_open, gap_extend, k=0)   # warm-up: runs directly
        _sync()
        db.search_batch(qs, subst, gap_open, gap_extend, k=0)                  # the repeat captures the graph
        got = _numpy(scores)
        ok = ref is None or bool(np.array_equal(got[:, idx].astype(np.int64), ref))
        if ok and verify is not None:
            ok = all(bool(verify(i, got[i])) for i in range(len(qs)))
        best = float("inf")
        for _ in range(repeats):
            t = time.perf_counter()
            db.search_batch(qs, subst, gap_open, gap_extend, k=0)
            _sync()
            best = min(best, time.perf_counter() - t)
        trials.append(dict(knobs=c, parity=ok, seconds=best, gcups=cells / best / 1e9))
        if verbose:
            print(f"tune {c}: parity={ok} {cells / best / 1e9:.0f} GCUPS", flush=True)
    eligible = [t for t in trials if t["parity"]]
    if not eligible:
        db.tune()
        raise RuntimeError(f"autotuner: no candidate passed the parity gate ({len(trials)} tried)")
    win = max(eligible, key=lambda t: t["gcups"])
    db.tune(**win["knobs"])
    gate = {"subjects": int(idx.size), "queries": len(qs), "reference": "32-bit alignment kernel",
            "verify": verify is not None}
    entry = dict(knobs=win["knobs"], gcups=win["gcups"], key=key, gate=gate)
    if use_cache:
        _memory_cache[key] = entry
        if cache_path:
            cache[key] = entry
            d = os.path.dirname(cache_path)
            if d:
                os.makedirs(d, exist_ok=True)
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, cache_path)
    return dict(entry, trials=trials, cached=False)
