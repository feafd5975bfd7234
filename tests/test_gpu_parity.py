"""GPU parity: every score from the HIP path equals the CPU oracle exactly.

Integer arithmetic end to end, so the bar is bit-exact equality (tolerance 0)
on every subject compared.  Cases span several groups and passes, ragged
tails, empty subjects, every lane-cooperation degree B (forced through the
``force_lanes`` hook), the 32-bit recompute path, extreme matrices and gap
penalties, and the full-size workload on a sampled subject set.
"""
import sys

import numpy as np
import pytest

import oracle
from inputs import synth
from refs import identity_matrix

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_scores(sw, db, q, sm, go, ge, **kw):
    import torch
    D = sw.Database(db.residues, db.offsets, **kw)
    out = D.search(q, sm, go, ge)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.int64)
    stats = D.stats()
    D.close()
    return res, stats


def assert_equal_scores(got, want, ctx=""):
    got = np.asarray(got, dtype=np.int64)
    want = np.asarray(want, dtype=np.int64)
    assert got.shape == want.shape, ctx
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} mismatches, first at {bad[:5]}: got {got[bad[:5]]} want {want[bad[:5]]}"


def test_workload1_all_scores(gpu, blosum):
    qs, db = synth.workload1()
    say("workload1: 1 x 144 vs 2000")
    got, st = gpu_scores(gpu, db, qs[0], blosum, 10, 2)
    want = oracle.scores(qs[0], db.residues, db.offsets, blosum, 10, 2)
    assert_equal_scores(got, want, "workload1")
    assert want.max() > 100   # planted homologs score high


@pytest.mark.parametrize("lanes", [0, 1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("m", [1, 16, 37, 300])
def test_every_lane_degree(gpu, blosum, lanes, m):
    db = synth.small_db(seed=11 + m, n=300, lo=0, hi=700)
    q = synth.small_query(seed=m, m=m)
    say(f"lanes={lanes} m={m}")
    got, st = gpu_scores(gpu, db, q, blosum, 10, 2, force_lanes=lanes)
    want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
    assert_equal_scores(got, want, f"lanes={lanes} m={m}")


@pytest.mark.parametrize("rows", [4, 8, 16])
@pytest.mark.parametrize("lanes", [0, 1, 4, 16, 64])
@pytest.mark.parametrize("m", [1, 37, 300])
def test_every_rows_per_lane(gpu, blosum, rows, lanes, m):
    db = synth.small_db(seed=71 + m, n=260, lo=0, hi=600)
    q = synth.small_query(seed=7 * m, m=m)
    say(f"rows={rows} lanes={lanes} m={m}")
    got, st = gpu_scores(gpu, db, q, blosum, 10, 2, force_lanes=lanes, rows_per_lane=rows)
    assert st["rows_per_lane"] == rows
    want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
    assert_equal_scores(got, want, f"rows={rows} lanes={lanes} m={m}")


@pytest.mark.parametrize("m", [20, 144, 700])
def test_short_query_long_subjects_side_stream(gpu, blosum, m):
    """A large database whose few longest subjects go to the small-R launch on
    the side stream when the query is short."""
    rng = np.random.default_rng(m)
    base = synth.small_db(seed=m, n=6000, lo=20, hi=900, median=300)
    lens = list(base.lengths) + [35000, 30000, 12000, 9000, 6000]
    subs = [base.subject(k) for k in range(base.n)] + [synth.background_residues(rng, L) for L in lens[base.n:]]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    q = synth.small_query(seed=m + 5, m=m)
    got, st = gpu_scores(gpu, db, q, blosum, 10, 2)
    want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
    assert_equal_scores(got, want, f"side stream m={m}")
    if m <= 144:
        assert st["side_items"] > 0 and st["side_rows_per_lane"] < 16, st


@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 257])
def test_ragged_database_sizes(gpu, blosum, n):
    db = synth.small_db(seed=n, n=n, lo=0, hi=90)
    q = synth.small_query(seed=n + 1, m=33)
    say(f"n={n}")
    got, _ = gpu_scores(gpu, db, q, blosum, 10, 2)
    assert_equal_scores(got, oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"n={n}")


def test_empty_subjects_and_empty_query(gpu, blosum):
    db = synth.small_db(seed=5, n=200, lo=0, hi=3)     # many zero-length subjects
    q = synth.small_query(seed=5, m=20)
    got, _ = gpu_scores(gpu, db, q, blosum, 10, 2)
    assert_equal_scores(got, oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), "tiny subjects")
    got, _ = gpu_scores(gpu, db, np.zeros(0, np.int8), blosum, 10, 2)
    assert (got == 0).all()


@pytest.mark.parametrize("go,ge", [(0, 0), (1, 11), (11, 1), (50000, 3), (3, 70000), (12, 12)])
def test_gap_penalties(gpu, blosum, go, ge):
    db = synth.small_db(seed=21, n=200, lo=1, hi=400)
    q = synth.small_query(seed=21, m=150)
    say(f"go={go} ge={ge}")
    for lanes in (0, 1, 16):
        got, _ = gpu_scores(gpu, db, q, blosum, go, ge, force_lanes=lanes)
        assert_equal_scores(got, oracle.scores(q, db.residues, db.offsets, blosum, go, ge), f"{go}/{ge} lanes={lanes}")


@pytest.mark.parametrize("kind", ["random_extreme", "identity", "lcs"])
def test_substitution_matrices(gpu, kind):
    rng = np.random.default_rng(3)
    if kind == "random_extreme":
        sm = rng.integers(-128, 128, size=(20, 20)).astype(np.int8)
        go, ge = 40, 5
    elif kind == "identity":
        sm = identity_matrix(1, -128)
        go, ge = 127, 127
    else:
        sm = identity_matrix(1, 0)
        go, ge = 0, 0
    db = synth.small_db(seed=31, n=150, lo=1, hi=300)
    q = synth.small_query(seed=31, m=120)
    for lanes in (0, 1, 8, 64):
        got, _ = gpu_scores(gpu, db, q, sm, go, ge, force_lanes=lanes)
        assert_equal_scores(got, oracle.scores(q, db.residues, db.offsets, sm, go, ge), f"{kind} lanes={lanes}")


def _overflow_db():
    """Subjects built around a W^3000 block: self scores far above 32767."""
    rng = np.random.default_rng(7)
    W = 17
    subs = [np.full(3000, W, np.int8), np.concatenate([rng.integers(0, 20, 50), np.full(3000, W), rng.integers(0, 20, 70)]),
            np.full(2990, W, np.int8), np.full(100, W, np.int8)]
    subs += [rng.integers(0, 20, int(rng.integers(1, 400))).astype(np.int8) for _ in range(140)]
    perm = rng.permutation(len(subs))
    subs = [np.asarray(subs[i], np.int8) for i in perm]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    return synth.Database(np.concatenate(subs), offs, name="overflow")


@pytest.mark.parametrize("lanes", [0, 1, 64])
def test_scores_above_int16_are_exact(gpu, blosum, lanes):
    db = _overflow_db()
    q = np.full(3000, 17, np.int8)
    got, st = gpu_scores(gpu, db, q, blosum, 10, 2, force_lanes=lanes)
    want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
    assert want.max() == 33000
    assert_equal_scores(got, want, f"overflow lanes={lanes}")
    assert st["rerun_pairs"] >= 2


def _threshold_db():
    """Self scores just below, at and above 31740: 16-bit cells carry the score
    plus the bias 4 (minus BLOSUM62's lowest score), and 0x7C00 = 31744 is the
    first 16-bit pattern that the packed maximum does not order as a number
    (W scores 11, A 4 and R 5 on the BLOSUM62 diagonal)."""
    W, A, R = 17, 0, 1
    rng = np.random.default_rng(23)
    core = [np.concatenate([np.full(2885, W), [A]]), np.concatenate([np.full(2885, W), [R]]), np.full(2890, W)]
    subs = [np.asarray(x, np.int8) for x in core] + [rng.integers(0, 20, int(rng.integers(1, 300))).astype(np.int8)
                                                       for _ in range(60)]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([x.size for x in subs])
    return synth.Database(np.concatenate(subs), offs, name="threshold"), core


@pytest.mark.parametrize("lanes", [0, 1, 64])
def test_scores_at_the_16bit_threshold(gpu, blosum, lanes):
    db, core = _threshold_db()
    for i, (q, self_score, reruns) in enumerate(zip(core, (31739, 31740, 31790), (False, True, True))):
        got, st = gpu_scores(gpu, db, q, blosum, 10, 2, force_lanes=lanes)
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
        assert want[i] == self_score
        assert_equal_scores(got, want, f"threshold q{i} lanes={lanes}")
        assert (st["rerun_pairs"] > 0) == reruns, (i, st)


def test_query_pairs_at_the_16bit_threshold(gpu, blosum):
    import torch
    db, core = _threshold_db()
    D = gpu.Database(db.residues, db.offsets, lane_pack=2)
    scores, _, _ = D.search_batch(core, blosum, 10, 2, k=0)
    torch.cuda.synchronize()
    for i, q in enumerate(core):
        assert_equal_scores(scores[i].cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"q{i}")
    D.close()


@pytest.mark.parametrize("lanes", [0, 4])
def test_forced_rerun_everything(gpu, blosum, lanes):
    """With the rerun threshold at 1 every pair goes through the 32-bit sweep."""
    db = synth.small_db(seed=41, n=260, lo=0, hi=500)
    q = synth.small_query(seed=41, m=200)
    got, st = gpu_scores(gpu, db, q, blosum, 10, 2, rerun_threshold=1, force_lanes=lanes)
    assert_equal_scores(got, oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), "forced rerun")
    assert st["rerun_pairs"] >= 120


def test_long_subjects(gpu, blosum):
    """Subjects up to 35,000 residues (multi-pass, many-lane units)."""
    rng = np.random.default_rng(9)
    lens = [35000, 20000, 9000, 5000, 3000] + list(rng.integers(50, 500, 40))
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    subs[1][5000:5400] = subs[0][100:500]        # a shared segment gives a strong local hit
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    q = np.concatenate([subs[0][100:500], synth.background_residues(rng, 1100)])
    got, _ = gpu_scores(gpu, db, q, blosum, 10, 2)
    want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
    assert_equal_scores(got, want, "long subjects")
    assert want[0] > 1500 and want[1] > 1500


def test_repeat_is_deterministic(gpu, blosum):
    import torch
    qs, db = synth.workload1()
    D = gpu.Database(db.residues, db.offsets)
    a = D.search(qs[0], blosum, 10, 2).clone()
    b = D.search(qs[0], blosum, 10, 2).clone()
    c = D.search(qs[0][::-1].copy(), blosum, 10, 2).clone()
    d = D.search(qs[0], blosum, 10, 2).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, d)
    want = oracle.scores(qs[0][::-1].copy(), db.residues, db.offsets, blosum, 10, 2)
    assert_equal_scores(c.cpu().numpy(), want, "second query on the same handle")
    D.close()


@pytest.mark.parametrize("k", [1, 10, 100, 1024])
def test_topk_matches_oracle(gpu, k):
    import torch
    rng = np.random.default_rng(k)
    s = rng.integers(0, 60, size=5000).astype(np.int32)    # many ties
    d = torch.from_numpy(s).cuda()
    ts, ti = gpu.topk(d, k)
    torch.cuda.synchronize()
    ws, wi = oracle.topk(s, k)
    assert (ts.cpu().numpy() == ws).all() and (ti.cpu().numpy() == wi).all()


@pytest.mark.parametrize("n", [0, 1, 7])
def test_topk_short_vectors(gpu, n):
    import torch
    s = np.arange(n, dtype=np.int32)[::-1].copy()
    d = torch.from_numpy(s).cuda() if n else torch.zeros(1, dtype=torch.int32, device="cuda")
    ts = torch.empty(10, dtype=torch.int32, device="cuda")
    ti = torch.empty(10, dtype=torch.int64, device="cuda")
    gpu.sw_topk(d, n, 10, ts, ti)
    torch.cuda.synchronize()
    ws, wi = oracle.topk(s, 10)
    assert (ts.cpu().numpy() == ws).all() and (ti.cpu().numpy() == wi).all()


def test_batch_matches_oracle(gpu, blosum):
    import torch
    qs, db = synth.workload1()
    rng = np.random.default_rng(2)
    queries = [qs[0], synth.small_query(1, 1), synth.small_query(2, 530), np.zeros(0, np.int8),
               db.subject(17).copy(), synth.small_query(3, 64)]
    D = gpu.Database(db.residues, db.offsets)
    scores, ts, ti = D.search_batch(queries, blosum, 10, 2, k=10)
    torch.cuda.synchronize()
    S = scores.cpu().numpy()
    for i, q in enumerate(queries):
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
        assert_equal_scores(S[i], want, f"batch query {i}")
        ws, wi = oracle.topk(want, 10)
        assert (ts[i].cpu().numpy() == ws).all() and (ti[i].cpu().numpy() == wi).all(), i
    # top-k only (no score matrix kept)
    _, ts2, ti2 = D.search_batch(queries, blosum, 10, 2, k=10, keep_scores=False)
    torch.cuda.synchronize()
    assert torch.equal(ts, ts2) and torch.equal(ti, ti2)
    D.close()


def test_batch_graph_replay(gpu, blosum):
    """The batched launch sequence is captured once per shape and replayed: replay
    it several times with new query contents of the same lengths, eager work and
    synchronisations in between, and check every replay against the oracle."""
    import torch
    db = synth.small_db(seed=91, n=700, lo=1, hi=600)
    lens = [5, 130, 47, 800, 1]
    D = gpu.Database(db.residues, db.offsets)
    scores = torch.empty((len(lens), db.n), dtype=torch.int32, device="cuda")
    ts = torch.empty((len(lens), 10), dtype=torch.int32, device="cuda")
    ti = torch.empty((len(lens), 10), dtype=torch.int64, device="cuda")
    for rep in range(4):
        queries = [synth.small_query(seed=1000 * rep + i, m=L) for i, L in enumerate(lens)]
        qo = np.concatenate([[0], np.cumsum(lens)])
        gpu.sw_search_batch(np.concatenate(queries), qo, D.handle, blosum, 10, 2, 10, scores, ts, ti)
        torch.cuda.synchronize()
        eager = torch.arange(1000, device="cuda").sum()      # unrelated eager work between replays
        S = scores.cpu().numpy()
        for i, q in enumerate(queries):
            want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
            assert_equal_scores(S[i], want, f"replay {rep} query {i}")
            ws, wi = oracle.topk(want, 10)
            assert (ts[i].cpu().numpy() == ws).all() and (ti[i].cpu().numpy() == wi).all()
        assert int(eager) == 499500
    # the same shapes with matrices of other lowest scores (the 16-bit bias): no stale replay
    for rep, sm in enumerate([identity_matrix(1, -128), identity_matrix(2, 0), blosum]):
        queries = [synth.small_query(seed=7000 + 10 * rep + i, m=L) for i, L in enumerate(lens)]
        qo = np.concatenate([[0], np.cumsum(lens)])
        gpu.sw_search_batch(np.concatenate(queries), qo, D.handle, sm, 3, 1, 10, scores, ts, ti)
        torch.cuda.synchronize()
        S = scores.cpu().numpy()
        for i, q in enumerate(queries):
            assert_equal_scores(S[i], oracle.scores(q, db.residues, db.offsets, sm, 3, 1), f"matrix {rep} query {i}")
    D.close()


@pytest.mark.parametrize("knobs", [dict(rows_per_lane=8), dict(rows_per_lane=16, unit_share=50),
                                   dict(force_lanes=4), dict(unit_share=2000)])
def test_tuning_knobs_do_not_change_results(gpu, blosum, knobs):
    import torch
    qs, db = synth.workload1()
    D = gpu.Database(db.residues, db.offsets)
    base = D.search(qs[0], blosum, 10, 2).clone()
    D.tune(**knobs)
    other = D.search(qs[0], blosum, 10, 2).clone()
    torch.cuda.synchronize()
    assert torch.equal(base, other), knobs
    D.close()


@pytest.mark.parametrize("knobs", [dict(lane_pack=2), dict(lane_pack=2, rows_per_lane=8),
                                   dict(lane_pack=2, force_lanes=4), dict(lane_pack=2, force_lanes=32),
                                   dict(lane_pack=2, rerun_threshold=1)])
def test_query_pair_packing(gpu, blosum, knobs):
    """Two queries per lane: pairs of very different lengths, an odd leftover
    query, an empty query, every score and top-k against the oracle."""
    import torch
    db = synth.small_db(seed=93, n=900, lo=0, hi=700)
    lens = [5, 800, 130, 129, 0, 47, 1]
    queries = [synth.small_query(seed=500 + i, m=L) for i, L in enumerate(lens)]
    D = gpu.Database(db.residues, db.offsets, **knobs)
    scores, ts, ti = D.search_batch(queries, blosum, 10, 2, k=10)
    torch.cuda.synchronize()
    S = scores.cpu().numpy()
    for i, q in enumerate(queries):
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
        assert_equal_scores(S[i], want, f"{knobs} query {i}")
        ws, wi = oracle.topk(want, 10)
        assert (ts[i].cpu().numpy() == ws).all() and (ti[i].cpu().numpy() == wi).all()
    D.close()


def test_query_pair_packing_overflow(gpu, blosum):
    """Saturating pairs recomputed for each query of a query pair."""
    import torch
    db = _overflow_db()
    queries = [np.full(3000, 17, np.int8), np.full(2995, 17, np.int8), synth.small_query(3, 300)]
    D = gpu.Database(db.residues, db.offsets, lane_pack=2)
    scores, _, _ = D.search_batch(queries, blosum, 10, 2, k=0)
    torch.cuda.synchronize()
    for i, q in enumerate(queries):
        assert_equal_scores(scores[i].cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"q{i}")
    assert D.stats()["rerun_pairs"] >= 4
    D.close()


def test_query_pair_long_subjects(gpu, blosum):
    """Query pairs over subjects up to 35,000 residues (widest scratch slots)."""
    import torch
    rng = np.random.default_rng(19)
    lens = [35000, 34000, 15000, 3000] + list(rng.integers(10, 600, 300))
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    queries = [synth.small_query(seed=40 + i, m=m) for i, m in enumerate([700, 650, 90])]
    D = gpu.Database(db.residues, db.offsets, lane_pack=2)
    scores, _, _ = D.search_batch(queries, blosum, 10, 2, k=0)
    torch.cuda.synchronize()
    for i, q in enumerate(queries):
        assert_equal_scores(scores[i].cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), f"q{i}")
    D.close()


def test_invalid_residues_are_rejected(gpu, blosum):
    qs, db = synth.workload1()
    D = gpu.Database(db.residues, db.offsets)
    bad = qs[0].copy()
    bad[5] = 20
    with pytest.raises(gpu.SwError) as e:
        D.search(bad, blosum, 10, 2)
    assert e.value.status == -2
    with pytest.raises(gpu.SwError):
        D.search(qs[0], blosum, -1, 2)
    D.close()
    res = db.residues.copy()
    res[100] = 25
    with pytest.raises(gpu.SwError) as e:
        gpu.Database(res, db.offsets)
    assert e.value.status == -2


def test_offsets_must_match_the_packed_database(gpu, blosum):
    """Offsets passed to a search are checked against the packed ones in full:
    same endpoints but a moved interior boundary is rejected."""
    import torch
    qs, db = synth.workload1()
    D = gpu.Database(db.residues, db.offsets)
    out = torch.empty(db.n, dtype=torch.int32, device="cuda")
    gpu.sw_search(qs[0], D.handle, db.offsets, db.n, blosum, 10, 2, out)     # the packed offsets: accepted
    torch.cuda.synchronize()
    assert_equal_scores(out.cpu().numpy(), oracle.scores(qs[0], db.residues, db.offsets, blosum, 10, 2), "offsets")
    moved = db.offsets.copy()
    moved[7] += 1
    for bad in (moved, db.offsets[::-1].copy()):
        with pytest.raises(gpu.SwError) as e:
            gpu.sw_search(qs[0], D.handle, bad, db.n, blosum, 10, 2, out)
        assert e.value.status == -1
    with pytest.raises(gpu.SwError):
        gpu.sw_search_mode(1, qs[0], D.handle, moved, db.n, blosum, 10, 2, out)
    D.close()


def test_full_size_workload2_sampled(gpu, blosum):
    """570k-subject database: every score of the sample (every 1000th subject,
    planted homologs, overflow sentinels, all subjects longer than 3,000) for the
    shortest query and the sentinel query, in the launch configuration the
    benchmark times."""
    import torch
    db = synth.sp570k()
    qs = synth.workload2_queries()
    idx = synth.parity_sample(db)
    say(f"workload2 full size: n={db.n} sample={idx.size}")
    D = gpu.Database(db.residues, db.offsets)
    for k in (0, synth.WL2_QLENS.index(3735)):
        out = D.search(qs[k], blosum, 10, 2)
        torch.cuda.synchronize()
        got = out.cpu().numpy()[idx]
        want = oracle.scores(qs[k], db.residues, db.offsets, blosum, 10, 2, idx=idx)
        assert_equal_scores(got, want, f"workload2 query {k}")
        if k:
            assert (want[np.isin(idx, db.sentinels)] > 32767).all()
    D.close()


def test_full_size_workload2_every_score(gpu, blosum):
    """570k-subject database, the shortest query (m = 144, 3.0e10 cells): every
    one of the 570,000 scores, local, global and semi-global, in the launch
    configuration the benchmark times."""
    import torch
    db = synth.sp570k()
    q = synth.workload2_queries()[0]
    D = gpu.Database(db.residues, db.offsets)
    for mode in ("local", "global", "semiglobal"):
        say(f"workload2 full size, every score: m={q.size} mode={mode}")
        out = D.search(q, blosum, 10, 2, mode=mode)
        torch.cuda.synchronize()
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2, mode=mode)
        assert_equal_scores(out.cpu().numpy(), want, f"workload2 query 0 {mode}")
    D.close()


@pytest.fixture(scope="module")
def workload2_scores(gpu, blosum):
    """Every query of the 570k-subject workload searched in the benchmark's launch configuration (one
    query per launch sequence); the score rows stay on the host."""
    import torch
    db = synth.sp570k()
    qs = synth.workload2_queries()
    D = gpu.Database(db.residues, db.offsets)
    rows = []
    for k, q in enumerate(qs):
        out = D.search(q, blosum, 10, 2)
        torch.cuda.synchronize()
        rows.append(out.cpu().numpy().copy())
    D.close()
    say(f"workload2: {len(qs)} queries searched")
    return db, qs, rows


def test_full_size_workload2_sample_for_every_query(workload2_scores, blosum):
    """All 20 queries on the parity sample (every 1000th subject, every planted homolog, the sentinels and
    every subject longer than 3,000 residues)."""
    db, qs, rows = workload2_scores
    idx = synth.parity_sample(db)
    for k, q in enumerate(qs):
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2, idx=idx)
        assert_equal_scores(rows[k][idx], want, f"workload2 query {k} (m={q.size}) sample")
    say(f"workload2: {idx.size} sampled subjects equal for all {len(qs)} queries")


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_full_size_workload2_short_queries_every_score(workload2_scores, blosum, k):
    """Every one of the 570,000 scores of the 2nd..5th shortest queries (the shortest is checked in all
    three modes above)."""
    db, qs, rows = workload2_scores
    want = oracle.scores(qs[k], db.residues, db.offsets, blosum, 10, 2)
    assert_equal_scores(rows[k], want, f"workload2 query {k} (m={qs[k].size}), all subjects")


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_full_size_workload2_modes_sample_for_every_query(gpu, blosum, mode):
    """End-to-end modes at full size: all 20 queries on the parity sample, which holds every subject
    longer than 3,000 residues (in global mode the groups of the longest run in 32-bit cells beside the
    16-bit launch, and out-of-range pairs are recomputed)."""
    import torch
    db = synth.sp570k()
    qs = synth.workload2_queries()
    idx = synth.parity_sample(db)
    D = gpu.Database(db.residues, db.offsets)
    for k, q in enumerate(qs):
        out = D.search(q, blosum, 10, 2, mode=mode)
        torch.cuda.synchronize()
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2, idx=idx, mode=mode)
        assert_equal_scores(out.cpu().numpy()[idx], want, f"workload2 {mode} query {k} (m={q.size}) sample")
    say(f"workload2 {mode}: {idx.size} sampled subjects equal for all {len(qs)} queries")
    D.close()


def test_extended_alphabet(gpu):
    """24-letter alphabet (B, Z, X, * after the 20 residues) with the full BLOSUM62."""
    import torch
    from inputs import blosum62_24
    sm = blosum62_24()
    rng = np.random.default_rng(24)
    lens = rng.integers(1, 600, 300)
    res = rng.integers(0, 24, int(lens.sum())).astype(np.int8)
    offs = np.zeros(lens.size + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    q = rng.integers(0, 24, 333).astype(np.int8)
    for lanes in (0, 1, 16):
        D = gpu.Database(res, offs, alphabet=24, force_lanes=lanes)
        got = D.search(q, sm, 10, 2)
        torch.cuda.synchronize()
        assert_equal_scores(got.cpu().numpy(), oracle.scores(q, res, offs, sm, 10, 2), f"alphabet 24 lanes={lanes}")
        D.close()
    D = gpu.Database(res, offs, alphabet=24, lane_pack=2)
    qs = [q, rng.integers(0, 24, 100).astype(np.int8), rng.integers(0, 24, 700).astype(np.int8)]
    scores, _, _ = D.search_batch(qs, sm, 10, 2, k=0)
    torch.cuda.synchronize()
    for i, x in enumerate(qs):
        assert_equal_scores(scores[i].cpu().numpy(), oracle.scores(x, res, offs, sm, 10, 2), f"alphabet 24 batch q{i}")
    with pytest.raises(ValueError):
        D.search(q, np.zeros((20, 20), np.int8), 10, 2)        # matrix of the wrong alphabet
    D.close()


def test_small_alphabet(gpu):
    """A 4-letter alphabet with a +5/-4 matrix (nucleotide-style scoring)."""
    import torch
    sm = np.full((4, 4), -4, np.int8)
    np.fill_diagonal(sm, 5)
    rng = np.random.default_rng(4)
    lens = rng.integers(1, 900, 200)
    res = rng.integers(0, 4, int(lens.sum())).astype(np.int8)
    offs = np.zeros(lens.size + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    q = rng.integers(0, 4, 500).astype(np.int8)
    D = gpu.Database(res, offs, alphabet=4)
    got = D.search(q, sm, 12, 4)
    torch.cuda.synchronize()
    assert_equal_scores(got.cpu().numpy(), oracle.scores(q, res, offs, sm, 12, 4), "alphabet 4")
    with pytest.raises(gpu.SwError):
        D.search(np.array([0, 4], np.int8), sm, 12, 4)        # code outside the alphabet
    D.close()
    bad = res.copy()
    bad[7] = 4
    with pytest.raises(gpu.SwError):
        gpu.Database(bad, offs, alphabet=4)
    with pytest.raises(gpu.SwError):
        gpu.Database(res, offs, alphabet=25)
