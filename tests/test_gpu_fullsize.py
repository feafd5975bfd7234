"""GPU parity at the full size of the batched, long-subject and serving workloads.

Sec. IV-A's workload shape (a protein database searched with many queries of
uneven length) at the sizes the benchmark runs, in its launch configuration;
the oracle recomputes what it can in seconds (tolerance 0, Eq. 1-3):

* 256 queries of 50..5,000 residues against the 570,000-subject database in
  one batched call (query pairs per lane, top 10): every sampled subject for
  every query (every 1,000th, the planted homologs, the three sentinels, every
  subject longer than 3,000, and the subject each query was built from), all
  570,000 scores of the 8 shortest queries, and every query's top 10 against
  the oracle's top 10 of the GPU's own score row; the same batch with two
  subjects per lane instead, every 4th query on the sampled subjects;
* 64 queries of 500..5,000 against 10,000 subjects of 3,000..35,000: every
  500th subject and the planted homologs, for every query;
* the 10,000,000-subject serving database: every 10,000th subject for each of
  32 requests, and every one of the 10,000,000 scores of each request equal
  alone (one plain search) and in the served mix (all 32 admitted together,
  two queries per lane); the length-paired FIFO's top 10 of each request
  equal to the top 10 of its full score row.
"""
import sys

import numpy as np
import pytest

import oracle
from inputs import synth

pytestmark = pytest.mark.gpu

# the batched benchmark's knobs: two queries per lane, at least two lanes per subject
BATCH_KNOBS = dict(rows_per_lane=16, unit_share=250, force_lanes=2, lane_pack=2)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _eq(got, want, ctx):
    got = np.asarray(got, np.int64)
    want = np.asarray(want, np.int64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} mismatches at {bad[:5]}: got {got[bad[:5]]} want {want[bad[:5]]}"


def _topk_of_row(row, k):
    """oracle.topk of a long score row, on the entries that can be in it (every score at
    or above the k-th largest): the same result as on the whole row."""
    row = np.asarray(row, np.int64)
    if row.size <= k:
        return oracle.topk(row, k)
    kth = np.partition(row, row.size - k)[row.size - k]
    cand = np.nonzero(row >= kth)[0]
    s, i = oracle.topk(row[cand], k)
    return s, np.where(i >= 0, cand[np.maximum(i, 0)], -1)


# ------------------------------------------------------------------ 256 queries x 570,000 subjects
@pytest.fixture(scope="module")
def batch256(gpu, blosum):
    import torch
    db = synth.sp570k()
    qs, sources = synth.workload3_queries(db, with_sources=True)
    say(f"batch256: {len(qs)} queries x {db.n} subjects, knobs {BATCH_KNOBS}")
    D = gpu.Database(db.residues, db.offsets, **BATCH_KNOBS)
    scores, ts, ti = D.search_batch(qs, blosum, 10, 2, k=10)
    torch.cuda.synchronize()
    st = D.stats()
    S = scores.cpu().numpy()
    out = dict(db=db, qs=qs, sources=sources, S=S, ts=ts.cpu().numpy(), ti=ti.cpu().numpy(), stats=st)
    del scores
    D.close()
    return out


@pytest.mark.parametrize("part", range(4))
def test_batch256_sampled_subjects(batch256, blosum, part):
    b = batch256
    db = b["db"]
    idx = np.unique(np.concatenate([synth.parity_sample(db), b["sources"]]))
    for qi in range(64 * part, 64 * part + 64):
        want = oracle.scores(b["qs"][qi], db.residues, db.offsets, blosum, 10, 2, idx=idx)
        _eq(b["S"][qi, idx], want, f"batch256 query {qi}")
    say(f"batch256 part {part}: {idx.size} subjects x 64 queries equal")


@pytest.mark.parametrize("half", range(2))
def test_batch256_shortest_queries_every_score(batch256, blosum, half):
    b = batch256
    db = b["db"]
    order = np.argsort([q.size for q in b["qs"]], kind="stable")[:8]
    for qi in order[4 * half: 4 * half + 4]:
        want = oracle.scores(b["qs"][qi], db.residues, db.offsets, blosum, 10, 2)
        _eq(b["S"][qi], want, f"batch256 query {qi} (m={b['qs'][qi].size}), all subjects")


def test_batch256_top10_and_recompute(batch256):
    b = batch256
    db = b["db"]
    for qi in range(len(b["qs"])):
        ws, wi = _topk_of_row(b["S"][qi], 10)
        assert (b["ts"][qi] == ws).all() and (b["ti"][qi] == wi).all(), qi
    k = int(np.argmax([q.size for q in b["qs"]]))                 # carries the sentinel block
    assert (b["S"][k, db.sentinels] > 32767).all()
    st = b["stats"]
    assert st["rerun_pairs"] >= 3 and st["recomputed"] == st["rerun_pairs"]


def test_batch256_subject_pairs(gpu, blosum):
    """The same batch with two subjects per lane (one query per lane, lane_pack 1): every 4th query on
    the sampled subjects, every query's top 10 against the oracle's top 10 of the GPU's own row."""
    import torch
    db = synth.sp570k()
    qs, sources = synth.workload3_queries(db, with_sources=True)
    knobs = dict(rows_per_lane=16, unit_share=250, lane_pack=1)
    say(f"batch256, subject pairs: {len(qs)} queries x {db.n} subjects, knobs {knobs}")
    D = gpu.Database(db.residues, db.offsets, **knobs)
    scores, ts, ti = D.search_batch(qs, blosum, 10, 2, k=10)
    torch.cuda.synchronize()
    S, ts, ti = scores.cpu().numpy(), ts.cpu().numpy(), ti.cpu().numpy()
    st = D.stats()
    del scores
    D.close()
    idx = np.unique(np.concatenate([synth.parity_sample(db), sources]))
    for qi in range(0, len(qs), 4):
        want = oracle.scores(qs[qi], db.residues, db.offsets, blosum, 10, 2, idx=idx)
        _eq(S[qi, idx], want, f"batch256 subject pairs, query {qi}")
    for qi in range(len(qs)):
        ws, wi = _topk_of_row(S[qi], 10)
        assert (ts[qi] == ws).all() and (ti[qi] == wi).all(), qi
    assert st["rerun_pairs"] >= 3 and st["recomputed"] == st["rerun_pairs"]
    say(f"batch256, subject pairs: {idx.size} subjects x {len(range(0, len(qs), 4))} queries equal")


# ------------------------------------------------------------------ 64 queries x 10,000 long subjects
@pytest.fixture(scope="module")
def long10k(gpu, blosum):
    import torch
    qs, db = synth.workload4()
    say(f"long10k: {len(qs)} queries x {db.n} subjects ({int(db.offsets[-1])} residues)")
    D = gpu.Database(db.residues, db.offsets, **BATCH_KNOBS)
    scores, _, _ = D.search_batch(qs, blosum, 10, 2, k=0)
    torch.cuda.synchronize()
    S = scores.cpu().numpy()
    del scores
    D.close()
    return qs, db, S


@pytest.mark.parametrize("half", range(2))
def test_long10k_sampled_subjects(long10k, blosum, half):
    qs, db, S = long10k
    idx = np.unique(np.concatenate([np.arange(0, db.n, 500, dtype=np.int64)] + list(db.planted.values())))
    for qi in range(32 * half, 32 * half + 32):
        want = oracle.scores(qs[qi], db.residues, db.offsets, blosum, 10, 2, idx=idx)
        _eq(S[qi, idx], want, f"long10k query {qi}")
    assert S.max() > 1000            # the planted homologs score high


# ------------------------------------------------------------------ serving, 10,000,000 subjects
def test_serve10M_alone_and_in_the_mix(gpu, blosum):
    import torch
    from paper_2309_09609_amd.serve import GpuEngine, Server
    db = synth.workload5_db()
    qs = synth.workload5_queries(32)
    say(f"serve10M: {db.n} subjects ({int(db.offsets[-1])} residues), {len(qs)} requests")
    D = gpu.Database(db.residues, db.offsets, lane_pack=2)
    idx = np.arange(0, db.n, 10_000, dtype=np.int64)
    alone = []
    for i, q in enumerate(qs):
        out = D.search(q, blosum, 10, 2).clone()
        torch.cuda.synchronize()
        _eq(out.cpu().numpy()[idx], oracle.scores(q, db.residues, db.offsets, blosum, 10, 2, idx=idx),
            f"serve10M request {i}")
        alone.append(out)

    class Keeping(GpuEngine):
        """Keeps each request's whole score vector when it retires."""
        kept = {}

        def topk(self, req):
            self.kept[req.rid] = req.slot[: self.db.n].clone()
            return super().topk(req)

    eng = Keeping(D, blosum, 10, 2, k=10)
    mix = Server(eng, nchunks=8, mem_budget=4 << 30).run(qs, np.zeros(len(qs)))
    assert mix.max_active == len(qs)
    wants = []
    for i in range(len(qs)):
        assert torch.equal(eng.kept[i], alone[i]), f"request {i}: mix differs from alone"
        ws, wi = _topk_of_row(alone[i].cpu().numpy(), 10)
        wants.append((ws, wi))
        m_s, m_i = mix.results[i]
        assert (m_s == ws).all() and (m_i == wi).all(), i
    # the length-paired FIFO on the same requests, all waiting at once (query pairs, queued launches)
    from paper_2309_09609_amd.serve import paired_run
    D.tune(lane_pack=2, force_lanes=2)
    rep = paired_run(D, qs, np.zeros(len(qs)), blosum, 10, 2, k=10)
    say(f"serve10M paired FIFO: {rep.paired} pairs of {len(qs)} requests")
    assert rep.paired > 0
    for i, (ws, wi) in enumerate(wants):
        p_s, p_i = rep.results[i]
        assert (p_s == ws).all() and (p_i == wi).all(), f"paired FIFO request {i}"
    D.close()
