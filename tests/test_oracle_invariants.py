"""Invariants of the local alignment score that the oracle must satisfy
(consequences of Eq. 1-3 with Go, Ge >= 0 and zero borders, Sec. II-B)."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle

seq = st.lists(st.integers(0, 19), min_size=0, max_size=24)
small_seq = st.lists(st.integers(0, 19), min_size=0, max_size=9)
gap = st.integers(0, 15)


def sym_matrix(draw_ints):
    a = np.array(draw_ints, dtype=np.int64).reshape(20, 20)
    return np.clip((a + a.T) // 2, -128, 127).astype(np.int8)


mat = st.lists(st.integers(-8, 11), min_size=400, max_size=400).map(sym_matrix)


@settings(max_examples=150, deadline=None)
@given(seq, seq, mat, gap, gap)
def test_swap_symmetry(q, d, sm, go, ge):
    """Swapping query and subject transposes the DP; with a symmetric matrix S is unchanged."""
    assert oracle.pair(q, d, sm, go, ge) == oracle.pair(d, q, sm, go, ge)


@settings(max_examples=150, deadline=None)
@given(seq, seq, mat, gap, gap)
def test_reversal(q, d, sm, go, ge):
    """Reversing both sequences maps alignments one-to-one with equal scores."""
    assert oracle.pair(q, d, sm, go, ge) == oracle.pair(q[::-1], d[::-1], sm, go, ge)


@settings(max_examples=150, deadline=None)
@given(seq, seq, mat, gap, gap)
def test_bounds(q, d, sm, go, ge):
    s = oracle.pair(q, d, sm, go, ge)
    assert s >= 0
    if q and d:
        best_pair = max(int(sm[a, b]) for a in q for b in d)
        assert s >= max(0, best_pair)
        assert s <= max(0, int(sm.max())) * min(len(q), len(d))
    else:
        assert s == 0


@settings(max_examples=100, deadline=None)
@given(seq, seq, mat, gap, gap, st.integers(0, 5), st.integers(0, 5))
def test_monotone_in_gap_penalties(q, d, sm, go, ge, dgo, dge):
    assert oracle.pair(q, d, sm, go + dgo, ge) <= oracle.pair(q, d, sm, go, ge)
    assert oracle.pair(q, d, sm, go, ge + dge) <= oracle.pair(q, d, sm, go, ge)


@settings(max_examples=100, deadline=None)
@given(seq, seq, seq, mat, gap, gap)
def test_appending_never_decreases(q, d, extra, sm, go, ge):
    s = oracle.pair(q, d, sm, go, ge)
    assert oracle.pair(q + extra, d, sm, go, ge) >= s
    assert oracle.pair(q, extra + d, sm, go, ge) >= s


@settings(max_examples=100, deadline=None)
@given(seq, seq, mat, gap, gap, st.integers(1, 10), st.integers(-20, 0))
def test_nonpositive_padding_is_invisible(q, d, sm, go, ge, k, pad_score):
    """Columns (or rows) whose substitution scores are all <= 0 never change S:
    this licenses padded layouts.  Residue 19 is turned into such a pad here."""
    sm = sm.copy()
    q = [min(x, 18) for x in q]
    d = [min(x, 18) for x in d]
    sm[:, 19] = pad_score
    sm[19, :] = pad_score
    s = oracle.pair(q, d, sm, go, ge)
    assert oracle.pair(q, d + [19] * k, sm, go, ge) == s
    assert oracle.pair(q + [19] * k, d, sm, go, ge) == s
    assert oracle.pair(q + [19] * k, d + [19] * k, sm, go, ge) == s


@settings(max_examples=150, deadline=None)
@given(small_seq, small_seq, mat, gap, gap)
def test_neginf_border_variant_agrees(q, d, sm, go, ge):
    """Zero E/F borders (as the paper initialises them) and minus-infinity
    borders give the same S whenever Go, Ge >= 0."""
    assert oracle.pair(q, d, sm, go, ge) == oracle.pair_neginf(q, d, sm, go, ge)


@settings(max_examples=80, deadline=None)
@given(seq, seq, mat, gap, gap)
def test_substitution_shift(q, d, sm, go, ge):
    """Raising every substitution score by c >= 0 raises S by at most c * min(m, n)
    and never lowers it."""
    c = 2
    sm2 = np.clip(sm.astype(np.int64) + c, -128, 127).astype(np.int8)
    s1, s2 = oracle.pair(q, d, sm, go, ge), oracle.pair(q, d, sm2, go, ge)
    assert s1 <= s2 <= s1 + c * min(len(q), len(d))
