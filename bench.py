#!/usr/bin/env python3
"""Benchmark: Smith-Waterman/Gotoh protein database search on one MI355X.

One step = the whole hot path over one batch of synthetic input: the 20
queries (144..5,478 residues) of the paper-scale workload, each searched in
the plain form (one query per launch sequence, on one stream) against the
570,000-subject synthetic database that is already packed in HBM.  GCUPS
counts true cells only: sum over queries of m x (total database residues).

Prints one JSON line.  ``--form batched`` times the batched form instead (all
queries of the step in one sw_search_batch call); ``--workload`` picks another
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS on 1 MI355X (plain vs batched), % int-VALU peak; p50/p99 query latency"
# Algorithmic lane operations per cell of the 16-bit sweep, in the minimal form
# of Eq. 1-3 (H - Go shared by E and F, no move): hd = Hdiag + SM;
# H = max(hd, E, F) (one three-input maximum); hgo = H - Go; E - Ge; F - Ge;
# E' = max(E - Ge, hgo, floor); F' = max(F - Ge, hgo) -- 7 operations -- plus
# S = max(S, H), which a three-input maximum folds in for two cells at a
# time: 7.5.
CELL_OPS = 7.5
MODE_CELL_OPS = 8.0


# Oracle threads at most: a GPU host's CPU share for one GPU (the box runs other GPUs' work too).
HOST_THREAD_CAP = 16


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, HOST_THREAD_CAP))


def host_report() -> dict:
    """What the host offers (nproc, the CPUs this process may use, the CPU model) and the thread cap."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model, "thread_cap": HOST_THREAD_CAP,
            "threads_used": host_cores(),
            "cap_reason": "the oracle uses at most one GPU's share of the host (16 threads)"}


def workload(name: str):
    from inputs import synth
    if name == "sp570k":
        db = synth.sp570k()
        return synth.workload2_queries(), db, "20 queries 144..5,478 vs 570,000 subjects (2.07e8 residues), BLOSUM62 10/2"
    if name == "small2k":
        qs, db = synth.workload1()
        return qs, db, "1 query of 144 vs 2,000 subjects, BLOSUM62 10/2"
    if name == "long10k":
        qs, db = synth.workload4()
        return qs, db, "64 queries 500..5,000 vs 10,000 subjects 3,000..35,000, BLOSUM62 10/2"
    if name == "serve10M":
        db = synth.workload5_db()
        return [], db, "10,000,000 subjects (log-normal median 250, max 35,000), Poisson query arrivals"
    if name == "batch256":
        db = synth.sp570k()
        return synth.workload3_queries(db), db, "256 queries 50..5,000 vs 570,000 subjects, BLOSUM62 10/2, top-10"
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(args):
    """HBM bytes per launch of the plain 16-bit sweep from the committed PMC
    summary, if it was taken on the kernel source as it is now (else None)."""
    import hashlib
    if args.form != "plain" or args.workload != "sp570k" or args.mode != "local":
        return None
    path = os.path.join(ROOT, "profiles", "traffic_k_sweep_i16_sp570k_plain.json")
    try:
        d = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2309_09609_amd", "csrc", "sw_kernels.hip"), "rb").read()
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return d.get("hbm_bytes_per_launch_avg")


def cpu_baseline(queries, db, sm, seconds: float, mode: str = "local"):
    """The oracle, as it stands, on the host cores: the queries in order, each
    against consecutive blocks of subjects, until about ``seconds`` of work."""
    import oracle
    threads = host_cores()
    lengths = db.lengths
    block = 4000

    def run(nthreads, limit, blk):
        cells, t0, parts = 0, time.perf_counter(), []
        for qi, q in enumerate(queries):
            done = 0
            while done < db.n and time.perf_counter() - t0 < limit:
                idx = np.arange(done, min(db.n, done + blk), dtype=np.int64)
                oracle.scores(q, db.residues, db.offsets, sm, 10, 2, idx=idx, threads=nthreads, mode=mode)
                cells += int(q.size) * int(lengths[idx].sum())
                done += idx.size
            if done:
                parts.append((qi, int(q.size), done))
            if done < db.n:
                break
        return cells, time.perf_counter() - t0, parts

    cells, dt, parts = run(threads, seconds, block)
    # the same oracle on one thread, over a quarter of the time
    cells1, dt1, _ = run(1, seconds / 4, block // 8)
    desc = ", ".join(f"query {qi} (m={m}) vs {done} subjects" for qi, m, done in parts)
    full = sum(int(q.size) for q in queries) * int(lengths.sum())     # one step of the workload
    gcups = cells / dt / 1e9
    return {"value": round(gcups, 4), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"{desc}: {cells:.3e} cells in {dt:.1f} s",
            "single_thread_gcups": round(cells1 / dt1 / 1e9, 4),
            "extrapolated_step_s": round(full / (gcups * 1e9), 1), "host": host_report()}


SERVE_POLICIES = ("plain", "paired", "pipelined", "served", "dynamic", "dynamic-q2", "srpt")


def served_policies(args):
    """(policies in order, headline policy) of the served form; SystemExit for a list without plain FIFO
    and at least one other known policy."""
    pols = [p for p in args.policies.split(",") if p]
    if "plain" not in pols or len(set(pols)) < 2 or not set(pols) <= set(SERVE_POLICIES):
        raise SystemExit(f"--policies: plain and at least one of {[p for p in SERVE_POLICIES if p != 'plain']}")
    return pols, args.headline if args.headline in pols else [p for p in pols if p != "plain"][0]


def serve_bench(args, sw, D, db, sm, total_res, perfmodel):
    """Served form: the serving policies against plain FIFO on one Poisson trace."""
    import torch
    from inputs import synth
    from paper_2309_09609_amd.serve import GpuEngine, Server, batch_run, fifo_run, paired_run
    warm = args.serve_warmup
    qs = synth.workload5_queries(warm + args.requests + 5)
    cells = lambda q: int(q.size) * total_res  # noqa: E731
    # plain service rate from a few searches
    out = torch.empty(db.n, dtype=torch.int32, device="cuda")
    D.search(qs[0], sm, 10, 2, out=out)
    torch.cuda.synchronize()
    t = time.perf_counter()
    probe = qs[-5:]
    for q in probe:
        D.search(q, sm, 10, 2, out=out)
        sw.topk(out, 10)
    torch.cuda.synchronize()
    service = (time.perf_counter() - t) / len(probe) * float(np.mean([q.size for q in qs[: warm + args.requests]])) \
        / float(np.mean([q.size for q in probe]))
    rate = args.load / service
    print(f"# plain service time {service * 1e3:.1f} ms -> arrival rate {rate:.2f}/s", file=sys.stderr, flush=True)
    trace = qs[: warm + args.requests]
    arrivals = synth.poisson_arrivals(rate, len(trace))
    pols, headline = served_policies(args)

    def progress(name):
        step = max(1, args.requests // 5)

        def cb(done, total):
            if done % step == 0 or done == total:
                print(f"# {name}: {done}/{total} requests done", file=sys.stderr, flush=True)
        return cb

    def run_policy(pol, tr, arr, **kw):
        """One policy on a trace; the knobs it runs with are applied first and reset afterwards."""
        if pol == "plain":
            return fifo_run(D, tr, arr, sm, **kw)
        if pol in ("paired", "pipelined"):
            if pol == "paired":
                D.tune(lane_pack=2, force_lanes=2)
            ratio = args.pair_ratio if pol == "paired" else 2.0        # above 1: never pairs
            r = paired_run(D, tr, arr, sm, ratio=ratio, depth=2, **kw)
        elif pol == "served":
            D.tune(lane_pack=args.lane_pack)
            r = Server(GpuEngine(D, sm, 10, 2, k=10), nchunks=args.chunks, mem_budget=2 << 30).run(tr, arr, **kw)
        elif pol in ("dynamic", "dynamic-q2"):
            D.tune(lane_pack=2 if pol == "dynamic-q2" else 1)
            r = batch_run(D, tr, arr, sm, **kw)
        else:   # srpt: one request at a time, least remaining work first at every chunk boundary
            r = Server(GpuEngine(D, sm, 10, 2, k=10), nchunks=args.chunks, mem_budget=2 << 30, max_active=1,
                       policy="srpt").run(tr, arr, **kw)
        D.tune()
        return r

    reps = {}
    for pol in pols:
        run_policy(pol, trace[:warm], arrivals[:warm] - arrivals[0])
        reps[pol] = run_policy(pol, trace[warm:], arrivals[warm:] - arrivals[warm], cells_per_query=cells,
                               progress=progress(pol))
        print(f"# {pol}: {reps[pol].summary()}", file=sys.stderr, flush=True)
    fifo_rep = reps["plain"]
    fifo, served = fifo_rep.summary(), reps[headline].summary()
    # every policy must return the same top-10 for every request
    same = all(np.array_equal(fifo_rep.results[i][0], o.results[i][0]) and
               np.array_equal(fifo_rep.results[i][1], o.results[i][1]) for o in reps.values() for i in fifo_rep.results)
    forms = {"paired": "served (length-paired FIFO, query pairs, pipelined launches)",
             "pipelined": "served (FIFO, pipelined launches)", "served": "served (continuous batching)",
             "dynamic": "served (dynamic batching)", "dynamic-q2": "served (dynamic batching, query pairs)",
             "srpt": "served (least remaining work first, chunk preemption)"}
    res = {
        "metric": METRIC, "value": round(served["gcups"], 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.requests,
        "warmup": warm, "ms_per_step": round(served["makespan_s"] / args.requests * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int16x2 saturating + int32 recompute", "data": "synthetic",
        "config": {"workload": "serve10M", "form": forms[headline], "subjects": db.n,
                   "residues": total_res, "requests": args.requests, "arrival_rate_per_s": round(rate, 3),
                   "load_vs_plain": args.load, "pair_ratio": args.pair_ratio, "chunks": args.chunks,
                   "matrix": "BLOSUM62", "gap_open": 10, "gap_extend": 2},
        "latency": {"served_policy": headline, "served_p50_s": round(served["p50_s"], 4),
                    "served_p99_s": round(served["p99_s"], 4),
                    "plain_p50_s": round(fifo["p50_s"], 4), "plain_p99_s": round(fifo["p99_s"], 4),
                    "p99_gain": round(fifo["p99_s"] / served["p99_s"], 3) if served["p99_s"] > 0 else None},
        "extra": {"policies": {k: v.summary() for k, v in reps.items()}, "same_top10_all_policies": same,
                  "plain_service_ms": round(service * 1e3, 2),
                  "pct_int32_cell_peak": round(100 * served["gcups"] / perfmodel.mi355x_peak_gcups(), 2)},
    }
    D.close()
    print(json.dumps(res), flush=True)


def topk_timing(sw, scores, k: int, reps: int = 20):
    """The top-k of one search's score vector, timed apart from the search:
    mean over ``reps`` calls, and the rate at which it reads the scores (4 bytes
    each, once per call for the first launch) against 8 TB/s of HBM."""
    import torch
    sw.topk(scores, k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sw.topk(scores, k)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = scores.numel() * 4 / (ms * 1e-3) / 1e9
    return {"k": k, "n": int(scores.numel()), "ms": round(ms, 4), "scores_read_gb_per_s": round(gbs, 1),
            "frac_of_hbm": round(gbs / 8000.0, 4)}


ALIGN_CELL_OPS = 9


def align_bench(args, sw, D, queries, db, sm, total_res, perfmodel):
    """Alignment form: search each query, then align the top 10 of every query
    in one sw_align_batch call per step; one sw_align call per query is timed
    beside it."""
    import torch
    out = torch.empty(db.n, dtype=torch.int32, device="cuda")
    tops = []
    for q in queries:
        D.search(q, sm, 10, 2, out=out)
        ts, ti = sw.topk(out[: db.n], 10)
        tops.append(ti.cpu().numpy())
    lens = np.diff(db.offsets)
    cells = sum(int(q.size) * int(lens[t].sum()) for q, t in zip(queries, tops))
    for i in range(args.warmup):
        D.align_batch(queries, tops, sm, 10, 2)
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        al = D.align_batch(queries, tops, sm, 10, 2)
        print(f"# step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    for q, t in zip(queries, tops):
        one = D.align(q, t, sm, 10, 2)
    el1 = time.perf_counter() - t1
    same = all(D.align(q, t, sm, 10, 2) == a for q, t, a in zip(queries[:3], tops[:3], al[:3]))
    n_al = len(queries) * 10
    # The fill sweeps Eq. 1-3 in int32 lanes: 9 operations per cell (diagonal add, three-input maximum
    # and the floor for H, H - Go shared by E and F, two extension subtractions, two maxima, the running
    # maximum); the direction byte it also records is not counted.  Pairs with both sides below 2,048
    # residues fill on one workgroup each, longer ones as tiles over the GPU (one anti-diagonal of tiles
    # per launch); a call lasts about as long as its longest pair's wavefront, so the whole-chip fraction
    # is small by construction.
    call_s = el / args.steps
    longest = max(int(q.size) * int(lens[k]) for q, t in zip(queries, tops) for k in t)
    tiled = sum(1 for q, t in zip(queries, tops) for k in t if q.size >= 2048 and lens[k] >= 2048)
    peak_chip = perfmodel.int_valu_lane_ops_per_s()
    achieved = ALIGN_CELL_OPS * cells / call_s
    roof = {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": round(peak_chip / 1e12, 3),
            "unit": "TOP/s (int32 lane-ops)", "frac": round(achieved / peak_chip, 4), "traffic": None,
            "kernel": "k_align_fill, k_align_tile, k_align_trace (one call)", "ops_per_cell": ALIGN_CELL_OPS,
            "longest_pair": {"cells": longest, "gcups": round(longest / call_s / 1e9, 3)},
            "tiled_pairs": tiled}
    res = {
        "metric": "GCUPS of the traceback (top-10 alignments per query)", "value": round(cells * args.steps / el / 1e9, 2),
        "unit": "GCUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "form": "align (one sw_align_batch call per step)",
                   "queries": len(queries), "alignments_per_query": 10, "subjects": db.n, "residues": total_res,
                   "matrix": "BLOSUM62", "gap_open": 10, "gap_extend": 2},
        "extra": {"alignments_per_s": round(n_al * args.steps / el, 1), "cells_per_step": cells,
                  "one_call_per_query": {"gcups": round(cells / el1 / 1e9, 2), "ms": round(el1 * 1e3, 3)},
                  "batch_equals_per_query": same,
                  "last_alignment": {k: al[-1][-1][k] for k in ("score", "q_begin", "q_end", "s_begin", "s_end")}},
        "roofline": roof,
    }
    D.close()
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_align_baseline(queries, tops, db, sm, args.cpu_seconds)
    print(json.dumps(res), flush=True)


def cpu_align_baseline(queries, tops, db, sm, seconds: float):
    """The oracle's alignment, as it stands, on the host cores (one pair per
    thread; the C call runs outside the interpreter lock): the same pairs in
    query order until about ``seconds`` of work."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    threads = host_cores()
    pairs = [(q, int(k)) for q, t in zip(queries, tops) for k in t]
    cells, done, t0 = 0, 0, time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        while done < len(pairs) and time.perf_counter() - t0 < seconds:
            batch = pairs[done:done + threads]
            subj = [db.residues[db.offsets[k]:db.offsets[k + 1]] for _, k in batch]
            list(pool.map(lambda a: oracle.align(a[0], a[1], sm, 10, 2), [(q, d) for (q, _), d in zip(batch, subj)]))
            cells += sum(int(q.size) * int(d.size) for (q, _), d in zip(batch, subj))
            done += len(batch)
    dt = time.perf_counter() - t0
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"the first {done} of the {len(pairs)} (query, subject) pairs in query order: "
                      f"{cells:.3e} cells in {dt:.1f} s", "host": host_report()}


PAIR_CELL_OPS = 8


def pair_bench(args, perfmodel):
    """One long pair spread over the GPU (sw_pair): two sequences of --pair-len residues with a
    mutated shared stretch, the tiles of one anti-diagonal per launch."""
    import torch
    import paper_2309_09609_amd as sw
    from inputs import blosum62, synth
    sm = blosum62()
    L = args.pair_len
    rng = synth.rng_for(6, 1)
    q = synth.background_residues(rng, L)
    d = synth.background_residues(rng, L)
    hom = synth.mutate(rng, q[L // 4: L // 4 + L // 2], 0.3, 0.02)[: L // 2]
    d[L // 5: L // 5 + hom.size] = hom
    ws = torch.empty(sw.sw_pair_workspace_bytes(L, L), dtype=torch.uint8, device="cuda")
    score = torch.empty(1, dtype=torch.int32, device="cuda")
    for i in range(args.warmup):
        sw.sw_pair(q, d, sm, 10, 2, d_score=score, d_ws=ws)
        torch.cuda.synchronize()
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        sw.sw_pair(q, d, sm, 10, 2, d_score=score, d_ws=ws)
    e1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    cells = L * L
    peak = perfmodel.int_valu_lane_ops_per_s()
    achieved = PAIR_CELL_OPS * cells / (ms * 1e-3)
    launches = (L + 255) // 256 + (L + 255) // 256 - 1
    res = {
        "metric": "GCUPS of one long pair spread over the GPU", "value": round(cells * args.steps / el / 1e9, 2),
        "unit": "GCUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"pair{L // 1000}k", "form": "pair (sw_pair)", "query_len": L, "subject_len": L,
                   "matrix": "BLOSUM62", "gap_open": 10, "gap_extend": 2},
        # 8 int32 lane-operations per cell (diagonal add, three-input maximum for H, H - Go, two extension
        # subtractions, two three-input maxima with the floor, the running maximum); one wave per tile and
        # at most one tile per 256 x 256 block of an anti-diagonal in flight, so the whole-GPU fraction is
        # bounded by the pair's own wavefront parallelism
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": round(peak / 1e12, 3),
                     "unit": "TOP/s (int32 lane-ops)", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "k_pair_tile", "launches_per_step": launches,
                     "avg_launch_ms": round(ms / launches, 4), "ops_per_cell": PAIR_CELL_OPS},
        "extra": {"score": int(score.item()), "event_ms_per_step": round(ms, 3)},
    }
    if args.pair_align and L <= 50_000:
        # the alignment of the same pair (traceback): the tiled fill against one workgroup for the pair
        offs = np.array([0, L], np.int64)
        D = sw.Database(d, offs)
        times, alns = {}, {}
        for mode, name in ((2, "tiled"), (1, "one_workgroup"), (2, "tiled")):
            D.tune(align_tiles=mode)
            t = time.perf_counter()
            alns[name] = D.align(q, [0], sm, 10, 2)[0]
            times[name] = time.perf_counter() - t        # the second tiled call is the one kept (warm)
            print(f"# align {name}: {times[name] * 1e3:.1f} ms", file=sys.stderr, flush=True)
        D.close()
        res["extra"]["align"] = {"tiled_ms": round(times["tiled"] * 1e3, 2),
                                 "one_workgroup_ms": round(times["one_workgroup"] * 1e3, 2),
                                 "tiled_gcups": round(cells / times["tiled"] / 1e9, 2),
                                 "speedup": round(times["one_workgroup"] / times["tiled"], 2),
                                 "same_alignment": alns["tiled"] == alns["one_workgroup"],
                                 "score_equals_sw_pair": alns["tiled"]["score"] == int(score.item()),
                                 "ops": len(alns["tiled"]["ops"])}
    if not args.no_cpu_baseline:
        import oracle
        n = min(L, 20_000)
        t = time.perf_counter()
        want = oracle.pair(q[:n], d[:n], sm, 10, 2)
        dt = time.perf_counter() - t
        res["cpu_baseline"] = {"value": round(n * n / dt / 1e9, 4), "unit": "GCUPS", "cores": 1, "kind": "oracle",
                               "sample": f"the first {n} x {n} residues of the pair ({n * n:.2e} cells, one thread: "
                                         f"one pair is one serial recurrence in the oracle) in {dt:.1f} s",
                               "score": int(want), "host": host_report()}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sp570k", choices=["sp570k", "small2k", "long10k", "batch256", "serve10M"])
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "served", "align", "pair"])
    ap.add_argument("--pair-len", type=int, default=100_000, help="pair form: residues of each sequence")
    ap.add_argument("--pair-align", action="store_true",
                    help="pair form: also align the pair (traceback), tiled fill vs one workgroup (up to 50,000)")
    ap.add_argument("--requests", type=int, default=200, help="served form: measured requests")
    ap.add_argument("--load", type=float, default=0.8, help="served form: arrival rate / plain service rate")
    ap.add_argument("--chunks", type=int, default=8, help="served form: database chunks per request cycle")
    ap.add_argument("--lane-pack", type=int, default=1, choices=[1, 2],
                    help="served form: 2 = requests that share an iteration share lanes two queries at a time")
    ap.add_argument("--policies", default="plain,paired,pipelined",
                    help="served form: comma list, run in this order on the same trace: plain (FIFO, one search "
                         "per request; required), paired (FIFO with length-matched query pairs, pipelined "
                         "launches), pipelined (FIFO, pipelined launches, no pairs), served (continuous batching "
                         "over database chunks), dynamic (batches of waiting requests, subject pairs per lane), "
                         "dynamic-q2 (the same with query pairs per lane), srpt (one request at a time, least "
                         "remaining work first at every chunk boundary)")
    ap.add_argument("--headline", default="paired", help="served form: the policy whose figures the line reports")
    ap.add_argument("--serve-warmup", type=int, default=10, help="served form: warm-up requests before the trace")
    ap.add_argument("--pair-ratio", type=float, default=0.85,
                    help="served form, paired policy: the shorter query of a pair is at least this share of the longer")
    ap.add_argument("--knobs", default="", help="batched form: JSON tuning knobs instead of autotuning")
    ap.add_argument("--mode", default="local", choices=["local", "global", "semiglobal"],
                    help="plain form: alignment mode (global and semi-global run in biased 16-bit cells, exact)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched-compare", action="store_true",
                    help="plain form: skip timing the batched form on the same queries")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}))
        return
    if args.form == "served":
        served_policies(args)                  # a bad list fails before the 10M-subject workload is built
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(a search would shard the database across GPUs).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2309_09609_amd as sw
    from inputs import blosum62
    from paper_2309_09609_amd import perfmodel

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.form == "pair":
        return pair_bench(args, perfmodel)
    sm = blosum62()
    t = time.perf_counter()
    queries, db, desc = workload(args.workload)
    print(f"# workload {args.workload}: {desc}; generated in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    t = time.perf_counter()
    D = sw.Database(db.residues, db.offsets)
    torch.cuda.synchronize()
    pack_s = time.perf_counter() - t          # host-to-device copy, sort, interleave (once per database)
    print(f"# packed in {pack_s:.1f} s", file=sys.stderr, flush=True)
    total_res = int(db.offsets[-1] - db.offsets[0])
    if args.form == "served":
        return serve_bench(args, sw, D, db, sm, total_res, perfmodel)
    if args.form == "align":
        return align_bench(args, sw, D, queries, db, sm, total_res, perfmodel)
    qlens = [int(q.size) for q in queries]
    cells_step = sum(qlens) * total_res
    out = torch.empty(db.n, dtype=torch.int32, device="cuda")

    tuned = None
    if args.form == "batched":
        from paper_2309_09609_amd import tune as tuner
        if args.knobs:
            D.tune(**json.loads(args.knobs))
            tuned = {"knobs": json.loads(args.knobs)}
        else:
            print("# autotuning on a sample of the batch", file=sys.stderr, flush=True)
            tuned = tuner.tune(D, queries, sm, 10, 2, use_cache=False, verbose=True)
        print(f"# tuned: {tuned['knobs']}", file=sys.stderr, flush=True)
        top_s = torch.empty((len(queries), 10), dtype=torch.int32, device="cuda")
        top_i = torch.empty((len(queries), 10), dtype=torch.int64, device="cuda")
        qcat = np.concatenate(queries)
        qoff = np.concatenate([[0], np.cumsum(qlens)]).astype(np.int64)

    def step():
        if args.form == "plain":
            for q in queries:
                D.search(q, sm, 10, 2, out=out, mode=args.mode)
        else:
            sw.sw_search_batch(qcat, qoff, D.handle, sm, 10, 2, 10, None, top_s, top_i)

    if args.form == "batched":
        # a batch shape runs directly the first time and is captured as a graph the second time: one call
        # here, so that the warm-up captures and the timed steps replay (the graph, like the plan, is set-up)
        step()
        torch.cuda.synchronize()
    D.profile_kernels(True)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    D.kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = [t0]
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        marks.append(time.perf_counter())
        print(f"# step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    step_ms = np.diff(marks) * 1e3
    kt = D.kernel_times()           # ms per 16-bit sweep launch in the timed region
    st = D.stats()
    if args.form == "plain" and kt.size == args.steps * len(queries):
        per_q = kt.reshape(args.steps, len(queries)).mean(axis=0)
        for m, ms in zip(qlens, per_q):
            print(f"# m={m:5d}  sweep {ms:8.2f} ms  {m * total_res / ms / 1e6:7.0f} GCUPS", file=sys.stderr)
    elapsed = t1 - t0
    gcups = cells_step * args.steps / elapsed / 1e9
    # cells of each timed launch (the plain form times one bulk launch per query, the batched form
    # one per batch); if the library forgot the oldest launches, the newest ones are those kept
    per_launch = [int(q.size) * total_res for q in queries] * args.steps if args.form == "plain" \
        else [cells_step] * args.steps
    timed_cells = sum(per_launch[-kt.size:]) if kt.size else 0
    kernel_s = float(kt.sum()) / 1e3
    launches = int(kt.size)
    # every mode computes in packed 16-bit lanes: two cell operations per VALU lane-op.  The end-to-end
    # modes take 8 operations per cell: the recurrence's 7 (no running maximum) and the fold of H into
    # the running minimum and maximum that prove the 16-bit values exact (half a three-input fold each)
    packed = True
    peak_ops = perfmodel.int_valu_lane_ops_per_s() * 2
    ops_cell = CELL_OPS if args.mode == "local" else MODE_CELL_OPS
    achieved = ops_cell * timed_cells / kernel_s / 1e12 if kernel_s > 0 and 0 < kt.size <= len(per_launch) else None
    roof = {"bound": "alu", "achieved": round(achieved, 3) if achieved else None,
            "peak": round(peak_ops / 1e12, 3), "unit": "TOP/s (int16 lane-ops)" if packed else "TOP/s (int32 lane-ops)",
            "frac": round(achieved * 1e12 / peak_ops, 4) if achieved else None,
            "traffic": measured_traffic(args),
            "kernel": ("k_sweep<CellI16>" if args.mode == "local" else f"k_sweep<CellI16, 16, {args.mode}>")
                      if args.form == "plain" else "batched graph (sweeps + recompute + top-k)",
            "launches": launches,
            "avg_launch_ms": round(kernel_s * 1e3 / max(launches, 1), 3),
            "ops_per_cell": ops_cell}
    res = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "int16x2 saturating + int32 recompute" if args.mode == "local"
                 else "int16x2 biased + int32 recompute", "data": "synthetic",
        "config": {"workload": args.workload, "form": args.form, "mode": args.mode, "queries": len(queries),
                   "qlen_min": min(qlens), "qlen_max": max(qlens), "subjects": db.n, "residues": total_res,
                   "matrix": "BLOSUM62", "gap_open": 10, "gap_extend": 2},
        "roofline": roof,
        "extra": {"pct_int32_cell_peak": round(100 * gcups / perfmodel.mi355x_peak_gcups(), 2),
                  "pct_packed16_cell_peak": round(100 * gcups / perfmodel.mi355x_peak_gcups(cells_per_lane_op=2), 2),
                  "kernel_gcups": round(timed_cells / kernel_s / 1e9, 2) if kernel_s > 0 else None,
                  "rerun_pairs_last_call": st["rerun_pairs"], "waves": st["waves"],
                  "step_ms": {"mean": round(float(step_ms.mean()), 3), "min": round(float(step_ms.min()), 3),
                              "stdev": round(float(step_ms.std(ddof=1)), 3) if step_ms.size > 1 else 0.0},
                  "tuned_knobs": tuned["knobs"] if tuned else None},
    }
    res["extra"]["pack_s"] = round(pack_s, 3)
    if args.form == "plain":
        res["extra"]["topk"] = topk_timing(sw, out, 10)
        # latency of one query at a time (after the timed steps): from the call to its scores on the device
        lat = []
        for q in queries:
            torch.cuda.synchronize()
            a = time.perf_counter()
            D.search(q, sm, 10, 2, out=out, mode=args.mode)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - a) * 1e3)
        lat = np.asarray(lat)
        res["extra"]["query_latency_ms"] = {"p50": round(float(np.percentile(lat, 50)), 3),
                                            "p99": round(float(np.percentile(lat, 99)), 3),
                                            "max": round(float(lat.max()), 3), "queries": int(lat.size)}
    if args.form == "plain" and not args.no_batched_compare and args.mode == "local":
        # the same queries in the batched form: one graph launch for all of them
        from paper_2309_09609_amd import tune as tuner
        print("# batched form on the same queries (autotuned)", file=sys.stderr, flush=True)
        tb = tuner.tune(D, queries, sm, 10, 2, use_cache=False, sample=len(queries), repeats=1)   # the whole batch
        qcat = np.concatenate(queries)
        qoff = np.concatenate([[0], np.cumsum(qlens)]).astype(np.int64)
        bs = torch.empty((len(queries), db.n), dtype=torch.int32, device="cuda")
        for _ in range(2):          # the first call of a shape runs directly, the second captures its graph
            sw.sw_search_batch(qcat, qoff, D.handle, sm, 10, 2, 0, bs, None, None)
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        for _ in range(args.steps):
            sw.sw_search_batch(qcat, qoff, D.handle, sm, 10, 2, 0, bs, None, None)
        torch.cuda.synchronize()
        tb1 = time.perf_counter()
        bg = cells_step * args.steps / (tb1 - tb0) / 1e9
        # same scores as the plain form (the last plain step left query 19's scores in `out`)
        same = bool(torch.equal(bs[-1], out))
        # every query of a batch completes with the batch: its latency is the batch's time
        res["extra"]["batched_same_queries"] = {"gcups": round(bg, 2), "gain_vs_plain": round(bg / gcups, 3),
                                                "ms_per_step": round((tb1 - tb0) / args.steps * 1e3, 3),
                                                "query_latency_ms": round((tb1 - tb0) / args.steps * 1e3, 3),
                                                "knobs": tb["knobs"], "scores_equal_plain": same}
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(queries, db, sm, args.cpu_seconds, mode=args.mode)
    D.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
