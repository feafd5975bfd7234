"""GPU alignments with the tiled fill (a long pair's matrix as tiles of 256
query rows by 128 or 256 subject columns, one anti-diagonal of tiles per
launch) against the oracle's, operation for operation, and against the
one-workgroup fill on the same pairs."""
import numpy as np
import pytest

import oracle
from inputs import synth
from refs import score_ops

pytestmark = pytest.mark.gpu


def _plant(rng, q, s, a, k):
    """Copy q[a:a+k] into s with a 3-residue insertion halfway (an alignment across many tiles, with a gap)."""
    k = min(k, q.size - a, s.size - 13)
    if k < 8:
        return
    h = k // 2
    seg = np.concatenate([q[a:a + h], synth.background_residues(rng, 3), q[a + h:a + k]])
    s[10:10 + seg.size] = seg[: s.size - 10]


def _db(subs):
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    return synth.Database(np.concatenate(subs), offs)


def _compare(got, q, db, subjects, sm, go, ge, ctx):
    assert len(got) == len(subjects)
    for a, k in zip(got, subjects):
        d = db.residues[db.offsets[k]:db.offsets[k + 1]]
        want = oracle.align(q, d, sm, go, ge)
        assert a["subject"] == k
        for key in ("score", "q_begin", "q_end", "s_begin", "s_end", "ops"):
            assert a[key] == want[key], f"{ctx} subject {k} (n={d.size}) {key}: got {a[key]!r} want {want[key]!r}"
        s, qe, se = score_ops(q, d, sm, go, ge, a["q_begin"], a["s_begin"], a["ops"])
        assert (s, qe, se) == (a["score"], a["q_end"], a["s_end"]), ctx


# subject lengths around the tile widths (128 below 4,096 columns, 256 from there) and the 64-lane ramp
EDGE_LENS = [1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1000, 4095, 4096, 4097, 6000]


@pytest.mark.parametrize("m", [1, 64, 255, 256, 257, 1300])
def test_tiled_fill_equals_the_oracle(gpu, blosum, m):
    rng = np.random.default_rng(700 + m)
    q = synth.background_residues(rng, m)
    subs = [synth.background_residues(rng, L) for L in EDGE_LENS]
    for i, s in enumerate(subs):
        _plant(rng, q, s, 3 * i % max(m // 2, 1), s.size)
    db = _db(subs)
    idx = list(range(db.n))
    print(f"tiled fill: m={m}, {db.n} subjects of {EDGE_LENS}", flush=True)
    D = gpu.Database(db.residues, db.offsets, align_tiles=2)
    got = D.align(q, idx, blosum, 10, 2)
    _compare(got, q, db, idx, blosum, 10, 2, f"tiles m={m}")
    D.tune(align_tiles=1)
    assert D.align(q, idx, blosum, 10, 2) == got
    D.close()


def test_auto_tiles_long_pairs_beside_one_workgroup_fills(gpu, blosum):
    """Default setting: pairs with both sides >= 2,048 residues are tiled, the rest fill on one workgroup
    each, concurrently, in the same call; several queries with their own subject lists."""
    rng = np.random.default_rng(808)
    lens = [2048, 2047, 5000, 300, 1, 9000]
    subs = [synth.background_residues(rng, L) for L in lens]
    qs = [synth.background_residues(rng, m) for m in (2600, 2048, 700, 0)]
    for i, s in enumerate(subs):
        _plant(rng, qs[i % 3], s, 5, s.size)
    db = _db(subs)
    lists = [[0, 1, 2, 3, 4, 5], [5, 0, 2], [2, 1], [0]]
    print(f"auto tiles: queries {[q.size for q in qs]}, subjects {lens}", flush=True)
    D = gpu.Database(db.residues, db.offsets)
    got = D.align_batch(qs, lists, blosum, 10, 2)
    for q, idx, g in zip(qs, lists, got):
        if q.size:
            _compare(g, q, db, idx, blosum, 10, 2, f"auto m={q.size}")
        else:
            assert all(a["score"] == 0 and a["ops"] == "" for a in g)
    D.tune(align_tiles=1)
    assert D.align_batch(qs, lists, blosum, 10, 2) == got
    D.close()


@pytest.mark.parametrize("go,ge", [(0, 0), (3, 5), (50000, 70000)])
def test_tiled_fill_gap_settings(gpu, blosum, go, ge):
    rng = np.random.default_rng(go * 7 + ge)
    q = synth.background_residues(rng, 600)
    subs = [synth.background_residues(rng, L) for L in (129, 700, 4200)]
    for s in subs:
        _plant(rng, q, s, 11, s.size)
    db = _db(subs)
    idx = list(range(db.n))
    D = gpu.Database(db.residues, db.offsets, align_tiles=2)
    _compare(D.align(q, idx, blosum, go, ge), q, db, idx, blosum, go, ge, f"tiles gaps {go}/{ge}")
    D.close()


def test_tiled_fill_extended_alphabet_and_high_scores(gpu):
    """24 letters, and a 3,000-residue run of W on both sides (score 33,000, above 2^15) across 13 bands and
    12 tiles of the subject."""
    from inputs import blosum62_24
    sm = blosum62_24()
    rng = np.random.default_rng(2424)
    w = 17                                             # W in ARNDCQEGHILKMFPSTWYV: 11 against itself
    q = rng.integers(0, 24, 3300).astype(np.int8)
    q[150:3150] = w
    run = np.concatenate([rng.integers(0, 24, 60).astype(np.int8), np.full(3000, w, np.int8),
                          rng.integers(0, 24, 40).astype(np.int8)])
    subs = [rng.integers(0, 24, 3000).astype(np.int8), run]
    _plant(rng, q, subs[0], 40, 3000)
    db = _db(subs)
    D = gpu.Database(db.residues, db.offsets, alphabet=24, align_tiles=2)
    got = D.align(q, [0, 1], sm, 10, 2)
    assert got[1]["score"] >= 33000
    _compare(got, q, db, [0, 1], sm, 10, 2, "tiles alphabet 24")
    D.close()


def test_full_size_top10_alignments(gpu, blosum):
    """The benchmark's traceback workload: every query of the 570k-subject workload searched, its top 10
    aligned in one call (the 60 pairs with both sides >= 2,048 residues tiled, the rest on one workgroup
    each), every alignment equal to the oracle's operation for operation."""
    import torch
    db = synth.sp570k()
    qs = synth.workload2_queries()
    D = gpu.Database(db.residues, db.offsets)
    tops = []
    for q in qs:
        scores = D.search(q, blosum, 10, 2)
        _, ti = gpu.topk(scores, 10)
        torch.cuda.synchronize()
        tops.append(ti.cpu().numpy().tolist())
    got = D.align_batch(qs, tops, blosum, 10, 2)
    lens = np.diff(db.offsets)
    tiled = sum(1 for q, t in zip(qs, tops) for k in t if q.size >= 2048 and lens[k] >= 2048)
    print(f"top-10 alignments of {len(qs)} queries, {tiled} pairs tiled", flush=True)
    assert tiled > 0
    for q, t, g in zip(qs, tops, got):
        _compare(g, q, db, t, blosum, 10, 2, f"top10 m={q.size}")
    D.close()
