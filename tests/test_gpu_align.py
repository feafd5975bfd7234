"""GPU alignments (traceback) against the oracle's: the same alignment,
operation for operation, under the stated choice among equal-scoring ones."""
import numpy as np
import pytest

import oracle
from inputs import synth
from refs import score_ops

pytestmark = pytest.mark.gpu


def _subject(db, k):
    return db.residues[db.offsets[k]:db.offsets[k + 1]]


def _compare(got, q, db, subjects, sm, go, ge, ctx):
    assert len(got) == len(subjects)
    for a, k in zip(got, subjects):
        d = _subject(db, k)
        want = oracle.align(q, d, sm, go, ge)
        assert a["subject"] == k
        for key in ("score", "q_begin", "q_end", "s_begin", "s_end", "ops"):
            assert a[key] == want[key], f"{ctx} subject {k} {key}: got {a[key]!r} want {want[key]!r}"
        s, qe, se = score_ops(q, d, sm, go, ge, a["q_begin"], a["s_begin"], a["ops"])
        assert (s, qe, se) == (a["score"], a["q_end"], a["s_end"]), ctx


def test_alignments_of_a_small_database(gpu, blosum):
    db = synth.small_db(seed=61, n=120, lo=1, hi=400)
    q = synth.small_query(seed=61, m=230)
    D = gpu.Database(db.residues, db.offsets)
    subs = list(range(db.n))
    _compare(D.align(q, subs, blosum, 10, 2), q, db, subs, blosum, 10, 2, "small db")
    D.close()


def test_alignments_of_the_top_hits(gpu, blosum):
    """The intended use: search, take the top 10, align them."""
    import torch
    qs, db = synth.workload1()
    D = gpu.Database(db.residues, db.offsets)
    scores = D.search(qs[0], blosum, 10, 2)
    ts, ti = gpu.topk(scores, 10)
    torch.cuda.synchronize()
    top = ti.cpu().numpy().tolist()
    got = D.align(qs[0], top, blosum, 10, 2)
    assert [a["score"] for a in got] == ts.cpu().numpy().tolist()
    _compare(got, qs[0], db, top, blosum, 10, 2, "top hits")
    D.close()


@pytest.mark.parametrize("m", [1, 255, 256, 257, 700])
def test_query_lengths_across_passes(gpu, blosum, m):
    rng = np.random.default_rng(m)
    lens = [1, 2, 3, 63, 64, 65, 500, 1500] + list(rng.integers(1, 900, 12))
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    q = synth.background_residues(rng, m)
    for s in subs[6:9]:
        k = min(s.size, q.size) // 2
        s[: k] = q[: k]                      # shared segments: long alignments with gaps nearby
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets)
    idx = list(range(db.n))
    _compare(D.align(q, idx, blosum, 10, 2), q, db, idx, blosum, 10, 2, f"m={m}")
    D.close()


@pytest.mark.parametrize("go,ge", [(0, 0), (3, 5), (11, 1), (50000, 70000)])
def test_gap_settings(gpu, blosum, go, ge):
    db = synth.small_db(seed=71, n=40, lo=1, hi=300)
    q = synth.small_query(seed=72, m=180)
    D = gpu.Database(db.residues, db.offsets)
    idx = list(range(db.n))
    _compare(D.align(q, idx, blosum, go, ge), q, db, idx, blosum, go, ge, f"gaps {go}/{ge}")
    D.close()


def test_long_subject_and_high_scores(gpu, blosum):
    """A 35,000-residue subject, a score above 2^15 and repeated requests."""
    rng = np.random.default_rng(3)
    big = synth.background_residues(rng, 35000)
    W = np.full(3000, 17, np.int8)
    subs = [big, W, np.concatenate([big[:100], W[:2000], big[100:300]])]
    offs = np.zeros(4, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    db = synth.Database(np.concatenate(subs), offs)
    q = np.concatenate([big[20000:20400], W[:2950]])
    D = gpu.Database(db.residues, db.offsets)
    idx = [0, 1, 2, 1]
    got = D.align(q, idx, blosum, 10, 2)
    assert got[1]["score"] == 2950 * 11
    _compare(got, q, db, idx, blosum, 10, 2, "long")
    D.close()


def test_empty_and_zero(gpu, blosum):
    db = synth.small_db(seed=81, n=10, lo=1, hi=50)
    D = gpu.Database(db.residues, db.offsets)
    got = D.align(np.zeros(0, np.int8), [0, 1], blosum, 10, 2)
    assert all(a["score"] == 0 and a["ops"] == "" for a in got)
    sm = np.full((20, 20), -1, dtype=np.int8)
    got = D.align(synth.small_query(seed=82, m=30), list(range(10)), sm, 1, 1)
    assert all(a["score"] == 0 and a["ops"] == "" and a["q_end"] == 0 and a["s_end"] == 0 for a in got)
    assert D.align(synth.small_query(seed=83, m=30), [], blosum, 10, 2) == []
    D.close()


def test_invalid_requests(gpu, blosum):
    db = synth.small_db(seed=91, n=10, lo=1, hi=50)
    D = gpu.Database(db.residues, db.offsets)
    with pytest.raises(gpu.SwError):
        D.align(synth.small_query(seed=92, m=10), [10], blosum, 10, 2)
    with pytest.raises(gpu.SwError):
        D.align(np.array([1, 25], np.int8), [0], blosum, 10, 2)
    longest = int(np.argmax(np.diff(db.offsets)))
    assert np.diff(db.offsets)[longest] >= 2
    with pytest.raises(gpu.SwError):      # operation buffer too small for query + subject
        gpu.sw_align(synth.small_query(seed=93, m=10), D.handle, np.array([longest], np.int64), blosum, 10, 2,
                     longest=0)
    for bad in (-1, 3):                   # the tiled-fill setting is 0, 1 or 2; a refused setting changes nothing
        with pytest.raises(gpu.SwError):
            D.tune(align_tiles=bad)
    q = synth.small_query(seed=94, m=40)
    assert D.align(q, [0, 1], blosum, 10, 2) == [oracle_alignment(q, db, k, blosum) for k in (0, 1)]
    D.close()


def oracle_alignment(q, db, k, sm, go=10, ge=2):
    d = db.residues[db.offsets[k]:db.offsets[k + 1]]
    a = oracle.align(q, d, sm, go, ge)
    return {"subject": k, **{key: a[key] for key in ("score", "q_begin", "q_end", "s_begin", "s_end", "ops")}}


def test_alignments_with_the_extended_alphabet(gpu):
    from inputs import blosum62_24
    sm = blosum62_24()
    rng = np.random.default_rng(240)
    lens = rng.integers(1, 500, 30)
    res = rng.integers(0, 24, int(lens.sum())).astype(np.int8)
    offs = np.zeros(lens.size + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(res, offs)
    q = rng.integers(0, 24, 300).astype(np.int8)
    q[50:150] = res[offs[3]:offs[3] + 100] if lens[3] >= 100 else q[50:150]
    D = gpu.Database(res, offs, alphabet=24)
    idx = list(range(db.n))
    _compare(D.align(q, idx, sm, 10, 2), q, db, idx, sm, 10, 2, "alphabet 24")
    D.close()


def _plant(rng, q, s, a, k):
    """Copy query residues q[a:a+k] into s with a 3-residue insertion halfway, so
    the alignment crosses many bands of query rows and includes a gap."""
    k = min(k, q.size - a, s.size - 13)
    if k < 8:
        return
    h = k // 2
    seg = np.concatenate([q[a:a + h], synth.background_residues(rng, 3), q[a + h:a + k]])
    s[10:10 + seg.size] = seg[: s.size - 10]


@pytest.mark.parametrize("m,lens", [
    (1300, [1, 5, 127, 128, 129, 600, 9000]),
    (3072, [64, 700, 2500]),
    (4200, [1, 300, 1800, 3000]),
])
def test_many_bands_in_flight(gpu, blosum, m, lens):
    """Queries of several to 17 bands of 256 rows, more bands than waves per
    pair, subjects from 1 residue to many stages of columns."""
    rng = np.random.default_rng(m)
    q = synth.background_residues(rng, m)
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    for s in subs:
        _plant(rng, q, s, 7, s.size)
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets)
    idx = list(range(db.n))
    got = D.align(q, idx, blosum, 10, 2)
    assert max(len(a["ops"]) for a in got) > 1000 or m < 2000
    _compare(got, q, db, idx, blosum, 10, 2, f"m={m}")
    D.close()


def test_many_bands_with_the_extended_alphabet(gpu):
    """24 letters: larger per-wave profiles; 18 bands wrap around the waves."""
    from inputs import blosum62_24
    sm = blosum62_24()
    rng = np.random.default_rng(2900)
    q = rng.integers(0, 24, 4400).astype(np.int8)
    subs = [rng.integers(0, 24, int(L)).astype(np.int8) for L in (2, 900, 2600)]
    for s in subs:
        _plant(rng, q, s, 100, s.size)
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets, alphabet=24)
    idx = list(range(db.n))
    _compare(D.align(q, idx, sm, 10, 2), q, db, idx, sm, 10, 2, "alphabet 24, 18 bands")
    D.close()


def test_align_batch_equals_one_call_per_query(gpu, blosum):
    """Several queries (one empty, one of 17 bands) with their own subject lists
    (one empty, repeats) in one call: each alignment equals sw_align's and the
    oracle's."""
    rng = np.random.default_rng(515)
    lens = [1, 40, 300, 700, 2000, 3500]
    subs = [synth.background_residues(rng, L) for L in lens]
    qs = [synth.background_residues(rng, m) for m in (0, 120, 900, 4200, 260)]
    for i, s in enumerate(subs):
        _plant(rng, qs[1 + i % 4], s, 3, s.size)
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets)
    lists = [[0, 1], [0, 1, 2, 3, 4, 5], [], [5, 4, 3, 2, 1, 0, 5], [2, 2, 3]]
    got = D.align_batch(qs, lists, blosum, 10, 2)
    assert [len(g) for g in got] == [len(x) for x in lists]
    for q, idx, g in zip(qs, lists, got):
        assert g == D.align(q, idx, blosum, 10, 2)
        _compare(g, q, db, idx, blosum, 10, 2, f"batch m={q.size}")
    assert D.align_batch([], [], blosum, 10, 2) == []
    with pytest.raises(gpu.SwError):
        D.align_batch([qs[1]], [[len(lens)]], blosum, 10, 2)
    D.close()
