"""GPU: the exact 32-bit recompute of flagged pairs never loses one.

A pair is flagged when its 16-bit score saturates (local) or one of its
values leaves the exact range (global, semi-global); its 32-bit recompute is
what makes the int32 score exact (Sec. II-B, Eq. 1-3; 32-bit cells as in
Sec. III-B).  Two test hooks make a lost recompute visible:

* ``poison``: a flagged pair's 16-bit scores are written as -1,000,000,007,
  so a score is right only if the recompute rewrote it;
* ``rerun_cap``: the recompute's list holds at most this many entries, so
  the pairs past it must be found through their flag bits.

With both on, every score must still equal the oracle, in every form (plain,
batched with subject pairs and with query pairs per lane, multi-query, global
and semi-global), and the library must report as many pairs recomputed as
flagged.
"""
import numpy as np
import pytest

import oracle
from inputs import synth
from refs import identity_matrix

pytestmark = pytest.mark.gpu

POISON = -1000000007


def _saturating_db():
    """90 subjects of 3,000-3,099 residues around a block of 2,990 W (scores above
    2^15 against a W query under BLOSUM62, where W scores 11), mixed with 200
    random subjects; many saturating subjects share groups and pairs."""
    rng = np.random.default_rng(77)
    W = 17
    subs = []
    for i in range(90):
        L = int(rng.integers(3000, 3100))
        s = rng.integers(0, 20, L).astype(np.int8)
        s[5:5 + 2990] = W
        subs.append(s)
    subs += [rng.integers(0, 20, int(rng.integers(1, 500))).astype(np.int8) for _ in range(200)]
    subs = [subs[i] for i in rng.permutation(len(subs))]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    return synth.Database(np.concatenate(subs), offs, name="saturating")


def _check_stats(st, ctx, expect_overflow=True):
    assert st["recomputed"] == st["rerun_pairs"], (ctx, st)
    assert st["rerun_pairs"] > 0, (ctx, st)
    if expect_overflow:
        assert st["rerun_overflow"] > 0, (ctx, st)


def _eq(got, want, ctx):
    got = np.asarray(got, dtype=np.int64)
    want = np.asarray(want, dtype=np.int64)
    assert not (got == POISON).any(), f"{ctx}: {(got == POISON).sum()} scores never recomputed"
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} mismatches at {bad[:5]}: got {got[bad[:5]]} want {want[bad[:5]]}"


@pytest.mark.parametrize("cap", [1, 5, 0])
def test_plain_saturated_poison(gpu, blosum, cap):
    import torch
    db = _saturating_db()
    q = np.full(3000, 17, np.int8)
    D = gpu.Database(db.residues, db.offsets, poison=1, rerun_cap=cap)
    got = D.search(q, blosum, 10, 2)
    torch.cuda.synchronize()
    st = D.stats()
    want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
    assert (want > 32767).sum() >= 80
    _eq(got.cpu().numpy(), want, f"plain cap={cap}")
    _check_stats(st, f"plain cap={cap}", expect_overflow=cap > 0)
    D.close()


@pytest.mark.parametrize("lanes", [0, 4, 64])
def test_plain_everything_flagged_tiny_cap(gpu, blosum, lanes):
    """Threshold 1: every pair with a positive score is flagged; 3 list entries."""
    import torch
    db = synth.small_db(seed=141, n=700, lo=0, hi=400)
    q = synth.small_query(seed=141, m=230)
    D = gpu.Database(db.residues, db.offsets, poison=1, rerun_cap=3, rerun_threshold=1, force_lanes=lanes)
    got = D.search(q, blosum, 10, 2)
    torch.cuda.synchronize()
    st = D.stats()
    _eq(got.cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"lanes={lanes}")
    _check_stats(st, f"lanes={lanes}")
    assert st["rerun_pairs"] >= 300
    D.close()


@pytest.mark.parametrize("lane_pack", [1, 2])
def test_batch_saturated_poison(gpu, blosum, lane_pack):
    import torch
    db = _saturating_db()
    rng = np.random.default_rng(5)
    queries = [np.full(3000, 17, np.int8), np.full(2995, 17, np.int8), synth.small_query(3, 300),
               np.concatenate([rng.integers(0, 20, 30), np.full(2990, 17)]).astype(np.int8), synth.small_query(4, 1)]
    D = gpu.Database(db.residues, db.offsets, poison=1, rerun_cap=4, lane_pack=lane_pack)
    scores, ts, ti = D.search_batch(queries, blosum, 10, 2, k=10)
    torch.cuda.synchronize()
    st = D.stats()
    S = scores.cpu().numpy()
    for i, q in enumerate(queries):
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
        _eq(S[i], want, f"lane_pack={lane_pack} query {i}")
        ws, wi = oracle.topk(want, 10)
        assert (ts[i].cpu().numpy() == ws).all() and (ti[i].cpu().numpy() == wi).all(), i
    _check_stats(st, f"batch lane_pack={lane_pack}")
    D.close()


def test_query_pairs_flag_each_pair_once(gpu, blosum):
    """Two queries per lane: both subjects of a pair may saturate for one query,
    and the pair is still listed once per query, as with subject pairs."""
    import torch
    db = _saturating_db()
    queries = [np.full(3000, 17, np.int8), np.full(2990, 17, np.int8), np.full(2999, 17, np.int8)]
    counts = {}
    for lp in (1, 2):
        D = gpu.Database(db.residues, db.offsets, lane_pack=lp)
        scores, _, _ = D.search_batch(queries, blosum, 10, 2, k=0)
        torch.cuda.synchronize()
        st = D.stats()
        for i, q in enumerate(queries):
            _eq(scores[i].cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"lp={lp} q{i}")
        assert st["recomputed"] == st["rerun_pairs"], st
        counts[lp] = st["rerun_pairs"]
        D.close()
    assert counts[1] == counts[2], counts


def test_batch_everything_flagged_query_pairs(gpu, blosum):
    """Query pairs, threshold 1 and a 2-entry list: nearly every (query, pair) of
    the batch is recomputed from its flag bit."""
    import torch
    db = synth.small_db(seed=143, n=500, lo=0, hi=300)
    lens = [5, 300, 131, 129, 0, 47, 1]
    queries = [synth.small_query(seed=600 + i, m=L) for i, L in enumerate(lens)]
    D = gpu.Database(db.residues, db.offsets, poison=1, rerun_cap=2, rerun_threshold=1, lane_pack=2)
    scores, _, _ = D.search_batch(queries, blosum, 10, 2, k=0)
    torch.cuda.synchronize()
    st = D.stats()
    for i, q in enumerate(queries):
        _eq(scores[i].cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"query {i}")
    _check_stats(st, "batch q2 threshold 1")
    D.close()


def test_multi_everything_flagged(gpu, blosum):
    """Chunked multi-query launches (the served form's building block)."""
    import torch
    db = synth.small_db(seed=145, n=900, lo=0, hi=300)
    queries = [synth.small_query(seed=700 + i, m=L) for i, L in enumerate([90, 250, 17])]
    D = gpu.Database(db.residues, db.offsets, poison=1, rerun_cap=2, rerun_threshold=1)
    outs = [torch.full((db.n,), -5, dtype=torch.int32, device="cuda") for _ in queries]
    qcat = np.concatenate(queries)
    qo = np.concatenate([[0], np.cumsum([q.size for q in queries])])
    nch = 3
    for c in range(nch):
        chunks = [(c + i) % nch for i in range(len(queries))]
        gpu.sw_search_multi(qcat, qo, chunks, nch, D.handle, blosum, 10, 2, outs)
        torch.cuda.synchronize()
        st = D.stats()
        _check_stats(st, f"multi call {c}")
    for i, q in enumerate(queries):
        _eq(outs[i].cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"multi query {i}")
    D.close()


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_modes_everything_flagged(gpu, blosum, mode):
    import torch
    db = synth.small_db(seed=147, n=600, lo=0, hi=350)
    q = synth.small_query(seed=147, m=160)
    D = gpu.Database(db.residues, db.offsets, poison=1, rerun_cap=3, rerun_threshold=1)
    got = D.search(q, blosum, 10, 2, mode=mode)
    torch.cuda.synchronize()
    st = D.stats()
    _eq(got.cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2, mode=mode), mode)
    _check_stats(st, mode)
    D.close()


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_modes_out_of_range_poison(gpu, mode):
    """A +11/-128 matrix and long identical stretches push 16-bit end-to-end
    values out of the exact range for real, with a 1-entry list."""
    import torch
    rng = np.random.default_rng(149)
    sm = identity_matrix(11, -128)
    subs = [np.full(int(L), 3, np.int8) for L in rng.integers(2800, 3200, 30)]
    subs += [rng.integers(0, 20, int(rng.integers(1, 400))).astype(np.int8) for _ in range(120)]
    subs = [subs[i] for i in rng.permutation(len(subs))]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    res = np.concatenate(subs)
    q = np.full(3000, 3, np.int8)
    D = gpu.Database(res, offs, poison=1, rerun_cap=1)
    got = D.search(q, sm, 10, 2, mode=mode)
    torch.cuda.synchronize()
    st = D.stats()
    _eq(got.cpu().numpy(), oracle.scores(q, res, offs, sm, 10, 2, mode=mode), mode)
    _check_stats(st, mode)
    D.close()
