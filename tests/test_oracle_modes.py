"""Pins of the oracle's global and semi-global scores: brute force, the
textbook edit-distance and approximate-matching tables, closed forms."""
import numpy as np
import pytest

import oracle
from refs import bf_end_to_end, best_substring_distance, edit_distance


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_modes_match_brute_force(mode):
    rng = np.random.default_rng(11 if mode == "global" else 12)
    for case in range(250):
        sm = rng.integers(-6, 7, size=(20, 20)).astype(np.int8)
        m, n = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        q = rng.integers(0, 3, m).astype(np.int8)
        d = rng.integers(0, 3, n).astype(np.int8)
        go, ge = int(rng.integers(0, 9)), int(rng.integers(0, 9))
        want = bf_end_to_end(q, d, sm, go, ge, semi=(mode == "semiglobal"))
        assert oracle.pair_mode(q, d, sm, go, ge, mode) == want, (case, m, n, go, ge)


def _unit_costs():
    sm = np.full((20, 20), -1, dtype=np.int8)
    np.fill_diagonal(sm, 0)
    return sm


def test_global_is_minus_edit_distance():
    """Match 0, mismatch -1, every gap residue 1 (Go = Ge = 1): the global score
    is minus the Levenshtein distance."""
    rng = np.random.default_rng(3)
    sm = _unit_costs()
    for _ in range(40):
        q = rng.integers(0, 4, int(rng.integers(0, 60))).astype(np.int8)
        d = rng.integers(0, 4, int(rng.integers(0, 60))).astype(np.int8)
        assert oracle.pair_mode(q, d, sm, 1, 1, "global") == -edit_distance(q, d)


def test_semiglobal_is_minus_best_substring_distance():
    rng = np.random.default_rng(4)
    sm = _unit_costs()
    for _ in range(40):
        q = rng.integers(0, 4, int(rng.integers(0, 40))).astype(np.int8)
        d = rng.integers(0, 4, int(rng.integers(0, 80))).astype(np.int8)
        assert oracle.pair_mode(q, d, sm, 1, 1, "semiglobal") == -best_substring_distance(q, d)


def test_closed_forms(blosum):
    rng = np.random.default_rng(5)
    q = rng.integers(0, 20, 400).astype(np.int8)
    diag = int(sum(int(blosum[c, c]) for c in q))
    assert oracle.pair_mode(q, q, blosum, 10, 2, "global") == diag
    # the query embedded in a longer subject: semi-global pays nothing for the flanks
    d = np.concatenate([rng.integers(0, 20, 300), q, rng.integers(0, 20, 200)]).astype(np.int8)
    assert oracle.pair_mode(q, d, blosum, 10, 2, "semiglobal") == diag
    # against an empty sequence: one gap run
    e = np.zeros(0, np.int8)
    assert oracle.pair_mode(q, e, blosum, 10, 2, "global") == -(10 + 399 * 2)
    assert oracle.pair_mode(e, q, blosum, 10, 2, "global") == -(10 + 399 * 2)
    assert oracle.pair_mode(e, q, blosum, 10, 2, "semiglobal") == 0
    assert oracle.pair_mode(q, e, blosum, 3, 5, "semiglobal") == -(3 + 399 * 3)


def test_local_mode_is_the_local_score(blosum):
    rng = np.random.default_rng(6)
    for _ in range(20):
        q = rng.integers(0, 20, int(rng.integers(0, 80))).astype(np.int8)
        d = rng.integers(0, 20, int(rng.integers(0, 80))).astype(np.int8)
        assert oracle.pair_mode(q, d, blosum, 10, 2, "local") == oracle.pair(q, d, blosum, 10, 2)


def test_scores_in_modes(blosum):
    rng = np.random.default_rng(7)
    lens = rng.integers(0, 50, 30)
    res = rng.integers(0, 20, int(lens.sum())).astype(np.int8)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    q = rng.integers(0, 20, 37).astype(np.int8)
    for mode in ("global", "semiglobal"):
        got = oracle.scores(q, res, offs, blosum, 10, 2, mode=mode)
        want = [oracle.pair_mode(q, res[offs[k]:offs[k + 1]], blosum, 10, 2, mode) for k in range(lens.size)]
        assert got.tolist() == want
