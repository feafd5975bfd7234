"""Pins of the oracle's alignment (traceback): brute-force optimality, closed
forms, and the stated choice among equal-scoring alignments."""
import numpy as np
import pytest

import oracle
from refs import bf_score, score_ops


def _check_valid(q, d, sm, go, ge, al):
    s, qe, se = score_ops(q, d, sm, go, ge, al["q_begin"], al["s_begin"], al["ops"])
    assert s == al["score"]
    assert (qe, se) == (al["q_end"], al["s_end"])
    assert 0 <= al["q_begin"] <= al["q_end"] <= len(q)
    assert 0 <= al["s_begin"] <= al["s_end"] <= len(d)
    if al["score"] > 0:
        assert al["ops"][0] == "M" and al["ops"][-1] == "M"
    else:
        assert al["ops"] == "" and al["q_end"] == 0 and al["s_end"] == 0


def test_alignment_is_optimal_by_brute_force():
    rng = np.random.default_rng(2024)
    for case in range(300):
        sm = rng.integers(-6, 7, size=(20, 20)).astype(np.int8)
        m, n = int(rng.integers(1, 6)), int(rng.integers(1, 6))
        q = rng.integers(0, 3, m).astype(np.int8)
        d = rng.integers(0, 3, n).astype(np.int8)
        go, ge = int(rng.integers(0, 9)), int(rng.integers(0, 9))
        al = oracle.align(q, d, sm, go, ge)
        want = bf_score(q, d, sm, go, ge)
        assert al["score"] == want == oracle.pair(q, d, sm, go, ge), (case, al, want)
        _check_valid(q, d, sm, go, ge, al)


def _plus_minus():
    sm = np.full((20, 20), -128, dtype=np.int8)
    np.fill_diagonal(sm, 1)
    return sm


@pytest.mark.parametrize("a,b,k,go,ge", [(40, 40, 3, 10, 2), (30, 25, 1, 5, 5), (50, 50, 10, 20, 1)])
def test_affine_gap_alignment_closed_form(a, b, k, go, ge):
    """Q = x^a y^b against D = x^a z^k y^b (identity +1, else -128): the best
    alignment bridges the z block with one gap run when a + b - Go - (k-1) Ge
    beats max(a, b); the mirrored case puts the run in the query."""
    assert a + b - go - (k - 1) * ge > max(a, b)
    sm = _plus_minus()
    x, y, z = 0, 1, 2
    q = np.array([x] * a + [y] * b, np.int8)
    d = np.array([x] * a + [z] * k + [y] * b, np.int8)
    al = oracle.align(q, d, sm, go, ge)
    assert al["ops"] == "M" * a + "D" * k + "M" * b
    assert (al["q_begin"], al["q_end"], al["s_begin"], al["s_end"]) == (0, a + b, 0, a + k + b)
    al = oracle.align(d, q, sm, go, ge)
    assert al["ops"] == "M" * a + "I" * k + "M" * b
    assert (al["q_begin"], al["q_end"], al["s_begin"], al["s_end"]) == (0, a + k + b, 0, a + b)


def test_self_alignment_is_the_diagonal(blosum):
    rng = np.random.default_rng(5)
    q = rng.integers(0, 20, 300).astype(np.int8)
    al = oracle.align(q, q, blosum, 10, 2)
    assert al["ops"] == "M" * q.size
    assert al["score"] == int(sum(int(blosum[c, c]) for c in q))
    assert (al["q_begin"], al["q_end"], al["s_begin"], al["s_end"]) == (0, q.size, 0, q.size)


def test_equal_hits_take_the_first_end_cell(blosum):
    """Two identical hits: the end cell is the first with H = S in row-major
    order, here the earlier subject position."""
    W, A = 17, 0
    q = np.array([W, W, W], np.int8)
    d = np.array([A, W, W, W, A, A, W, W, W, A], np.int8)
    al = oracle.align(q, d, blosum, 10, 2)
    assert al["score"] == 33
    assert (al["s_begin"], al["s_end"], al["ops"]) == (1, 4, "MMM")


def test_empty_and_zero_score(blosum):
    assert oracle.align(np.zeros(0, np.int8), np.array([1, 2], np.int8), blosum, 10, 2)["ops"] == ""
    sm = np.full((20, 20), -1, dtype=np.int8)
    al = oracle.align(np.array([1, 2, 3], np.int8), np.array([1, 2], np.int8), sm, 1, 1)
    assert al["score"] == 0 and al["ops"] == "" and al["q_end"] == 0


def test_random_protein_pairs_are_valid(blosum):
    rng = np.random.default_rng(77)
    for _ in range(30):
        q = rng.integers(0, 20, int(rng.integers(1, 120))).astype(np.int8)
        d = rng.integers(0, 20, int(rng.integers(1, 200))).astype(np.int8)
        d[5:5 + min(40, q.size)] = q[: min(40, q.size)][: d[5:5 + 40].size]
        for go, ge in ((10, 2), (3, 5), (0, 0)):
            al = oracle.align(q, d, blosum, go, ge)
            assert al["score"] == oracle.pair(q, d, blosum, go, ge)
            _check_valid(q, d, blosum, go, ge, al)
