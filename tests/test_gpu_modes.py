"""GPU global and semi-global scores against the oracle (tolerance 0)."""
import numpy as np
import pytest

import oracle
from inputs import synth
from refs import edit_distance

pytestmark = pytest.mark.gpu


def _db(seed, n, lo, hi, extra=()):
    rng = np.random.default_rng(seed)
    lens = [0, 1, 2, 3, 4, 5] + list(extra) + list(rng.integers(lo, hi, n))
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    return synth.Database(np.concatenate(subs), offs)


def _check(gpu, D, db, q, sm, go, ge, mode, ctx):
    import torch
    got = D.search(q, sm, go, ge, mode=mode)
    torch.cuda.synchronize()
    want = oracle.scores(q, db.residues, db.offsets, sm, go, ge, mode=mode)
    got = got.cpu().numpy().astype(np.int64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} mismatches, first {bad[:5]}: got {got[bad[:5]]} want {want[bad[:5]]}"


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
@pytest.mark.parametrize("lanes", [0, 1, 8, 64])
def test_modes_against_the_oracle(gpu, blosum, mode, lanes):
    db = _db(31, 200, 1, 700)
    D = gpu.Database(db.residues, db.offsets, force_lanes=lanes)
    for m in (1, 7, 8, 9, 200, 513):
        q = synth.small_query(seed=m, m=m)
        _check(gpu, D, db, q, blosum, 10, 2, mode, f"{mode} lanes={lanes} m={m}")
    D.close()


@pytest.mark.parametrize("go,ge", [(0, 0), (3, 5), (11, 1), (40, 40)])
def test_mode_gap_settings(gpu, blosum, go, ge):
    db = _db(32, 80, 1, 400)
    D = gpu.Database(db.residues, db.offsets)
    q = synth.small_query(seed=5, m=150)
    for mode in ("global", "semiglobal"):
        _check(gpu, D, db, q, blosum, go, ge, mode, f"{mode} {go}/{ge}")
    D.close()


def test_modes_with_long_subjects(gpu, blosum):
    db = _db(33, 40, 100, 900, extra=(35000, 12000, 3000))
    D = gpu.Database(db.residues, db.offsets)
    q = np.concatenate([db.residues[db.offsets[7] + 100: db.offsets[7] + 600], synth.small_query(seed=9, m=300)])
    for mode in ("global", "semiglobal"):
        _check(gpu, D, db, q, blosum, 10, 2, mode, f"{mode} long")
    D.close()


def test_empty_query_and_edit_distance(gpu):
    import torch
    db = _db(34, 60, 0, 120)
    sm = np.full((20, 20), -1, dtype=np.int8)
    np.fill_diagonal(sm, 0)
    D = gpu.Database(db.residues, db.offsets)
    lens = np.diff(db.offsets)
    got = D.search(np.zeros(0, np.int8), sm, 10, 2, mode="global").cpu().numpy()
    assert (got == np.where(lens > 0, -(10 + (lens - 1) * 2), 0)).all()
    assert (D.search(np.zeros(0, np.int8), sm, 10, 2, mode="semiglobal").cpu().numpy() == 0).all()
    q = synth.small_query(seed=11, m=90)
    got = D.search(q, sm, 1, 1, mode="global")
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    for k in range(db.n):
        assert got[k] == -edit_distance(q, db.residues[db.offsets[k]:db.offsets[k + 1]]), k
    D.close()


def test_modes_extended_alphabet(gpu):
    from inputs import blosum62_24
    sm = blosum62_24()
    rng = np.random.default_rng(35)
    lens = rng.integers(0, 400, 100)
    res = rng.integers(0, 24, int(lens.sum())).astype(np.int8)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    db = synth.Database(res, offs)
    D = gpu.Database(res, offs, alphabet=24)
    q = rng.integers(0, 24, 222).astype(np.int8)
    for mode in ("global", "semiglobal"):
        _check(gpu, D, db, q, sm, 10, 2, mode, f"{mode} alphabet 24")
    D.close()


def test_mode_range_and_argument_errors(gpu, blosum):
    db = _db(36, 10, 1, 50)
    D = gpu.Database(db.residues, db.offsets)
    q = synth.small_query(seed=1, m=20)
    with pytest.raises(gpu.SwError):
        D.search(q, blosum, 1 << 28, 1 << 28, mode="global")
    out = __import__("torch").empty(db.n, dtype=__import__("torch").int32, device="cuda")
    with pytest.raises(gpu.SwError):
        gpu.sw_search_mode(3, q, D.handle, db.offsets, db.n, blosum, 10, 2, out)
    D.close()


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_mode_scores_beyond_the_16bit_range(gpu, blosum, mode):
    """16-bit cells start just above the lowest value the query allows
    (-(Go + (m - 1) Ge)): semi-global H, and global H - g(j) on column-offset
    cells, never fall below it.  A 33,000-point self alignment leaves the range
    and goes to the 32-bit recompute, exactly; a 22,000-point one stays in it."""
    W = 17
    rng = np.random.default_rng(44)
    subs = [np.full(3000, W, np.int8), np.concatenate([np.full(1000, W, np.int8), synth.background_residues(rng, 300)])]
    subs += [synth.background_residues(rng, int(L)) for L in rng.integers(1, 600, 60)]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets)
    _check(gpu, D, db, np.full(3000, W, np.int8), blosum, 10, 2, mode, f"{mode} W-run 3000")
    assert D.stats()["rerun_pairs"] >= 1
    _check(gpu, D, db, np.full(2000, W, np.int8), blosum, 10, 2, mode, f"{mode} W-run 2000")
    assert D.stats()["rerun_pairs"] == 0
    _check(gpu, D, db, synth.small_query(seed=45, m=300), blosum, 10, 2, mode, f"{mode} short query")
    D.close()


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
@pytest.mark.parametrize("lanes", [0, 8])
def test_mode_forced_recompute(gpu, blosum, mode, lanes):
    """With the recompute threshold at 1 every pair with a positive H goes through
    the 32-bit sweep as well; the scores do not change."""
    db = _db(34, 150, 1, 500)
    D = gpu.Database(db.residues, db.offsets, rerun_threshold=1, force_lanes=lanes)
    for m in (5, 170):
        _check(gpu, D, db, synth.small_query(seed=m, m=m), blosum, 10, 2, mode, f"{mode} forced m={m}")
    assert D.stats()["rerun_pairs"] >= 10
    D.close()


@pytest.mark.parametrize("mode,go,ge", [("global", 3, 5), ("global", 10, 2), ("semiglobal", 10, 2)])
def test_modes_with_the_longest_group_in_32bit_cells(gpu, blosum, mode, go, ge):
    """Global mode on plain cells (Ge > Go): subjects whose row-0 border leaves the
    16-bit range form the first length-sorted group and run in 32-bit cells beside
    the 16-bit launch of the other groups.  With Ge <= Go the column-offset cells
    hold the same subjects in 16 bits."""
    rng = np.random.default_rng(46)
    lens = [20000, 9000, 8000] + list(rng.integers(1, 900, 400))
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets)
    for m in (90, 700, 900):
        _check(gpu, D, db, synth.small_query(seed=m, m=m), blosum, go, ge, mode, f"{mode} {go}/{ge} m={m}")
        st = D.stats()
        assert st["items"] + st["side_items"] > 0
        if mode == "global" and ge > go:
            assert st["side_items"] > 0
    D.close()


def test_global_offset_cells_and_the_32bit_fallback(gpu, blosum):
    """Global scores with Ge <= Go: short queries against subjects up to 12,000
    residues on column-offset 16-bit cells; a query of 8,000 residues, whose own
    gap run leaves any 16-bit range, wholly in 32-bit cells; Ge > Go on plain cells."""
    rng = np.random.default_rng(48)
    lens = [12000, 9000, 7000] + list(rng.integers(0, 700, 120))
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    subs[5] = synth.small_query(seed=49, m=300)                   # equal to the second query below
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([x.size for x in subs])
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets)
    for m, seed in ((1, 50), (300, 49), (2000, 51), (8000, 52)):
        q = synth.small_query(seed=seed, m=m)
        for go, ge in ((10, 2), (5, 5), (2, 7)):
            _check(gpu, D, db, q, blosum, go, ge, "global", f"global m={m} {go}/{ge}")
    D.close()


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_modes_short_queries_with_long_pairs_beside(gpu, blosum, mode):
    """A short query against a few long subjects: the long pairs run at 4 or 8
    rows per lane on a side stream beside the 16-row launch (a 64-lane pass of
    16 rows would be mostly padding); the scores do not change."""
    rng = np.random.default_rng(47)
    lens = [6000, 5000, 4000, 3500] + list(rng.integers(1, 400, 600))
    subs = [synth.background_residues(rng, int(L)) for L in lens]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    db = synth.Database(np.concatenate(subs), offs)
    D = gpu.Database(db.residues, db.offsets)
    rows = set()
    for m in (1, 30, 100, 300, 600):
        _check(gpu, D, db, synth.small_query(seed=m, m=m), blosum, 10, 2, mode, f"{mode} m={m}")
        st = D.stats()
        if st["side_items"] > 0:
            rows.add(st["side_rows_per_lane"])
    assert rows and rows <= {4, 8}, rows
    D.close()
