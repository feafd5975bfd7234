"""Pins of the CPU oracle against brute force, closed forms and textbook cases.

The paper prints no alignment scores, so every pin here is derived from the
definitions of Sec. II-B (Eq. 1-3, zero borders, S = largest H) and from
results that follow from them mathematically.
"""
import itertools

import numpy as np
import pytest

import oracle
from refs import bf_score, identity_matrix, kadane_diagonals, lcs_len, lcsubstr_len


def rnd(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- brute force
def test_bruteforce_exhaustive_tiny():
    """Every pair of sequences of length 1..3 over a 3-letter sub-alphabet, with
    three matrices and several gap settings (Ge <= Go, Ge > Go, zero gaps)."""
    g = rnd(1)
    mats = [identity_matrix(2, -1), g.integers(-4, 6, size=(20, 20)).astype(np.int8),
            g.integers(-2, 3, size=(20, 20)).astype(np.int8)]
    letters = [0, 7, 17]
    seqs = [list(p) for L in (1, 2, 3) for p in itertools.product(letters, repeat=L)]
    gaps = [(3, 1), (1, 3), (0, 0), (5, 5)]
    count = 0
    for mi, sm in enumerate(mats):
        go, ge = gaps[mi % len(gaps)] if mi else (2, 1)
        for a in seqs:
            for b in seqs:
                assert oracle.pair(a, b, sm, go, ge) == bf_score(a, b, sm, go, ge), (a, b, mi)
                count += 1
    assert count == 3 * len(seqs) ** 2


@pytest.mark.parametrize("seed", range(60))
def test_bruteforce_random(seed, blosum):
    g = rnd(100 + seed)
    m, n = int(g.integers(1, 7)), int(g.integers(1, 7))
    q, d = g.integers(0, 20, m), g.integers(0, 20, n)
    if seed % 3 == 0:
        sm = g.integers(-6, 8, size=(20, 20)).astype(np.int8)
    elif seed % 3 == 1:
        sm = blosum
    else:   # few letters so that gapped alignments matter
        q, d = g.integers(0, 3, m), g.integers(0, 3, n)
        sm = g.integers(-3, 5, size=(20, 20)).astype(np.int8)
    go, ge = int(g.integers(0, 13)), int(g.integers(0, 13))
    assert oracle.pair(q, d, sm, go, ge) == bf_score(q, d, sm, go, ge)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("a,b,k,go,ge", [(40, 40, 3, 10, 2), (5, 7, 1, 4, 4), (30, 2, 6, 3, 1),
                                         (12, 12, 10, 0, 0), (20, 25, 2, 12, 12), (60, 60, 40, 2, 1)])
def test_affine_gap_length_convention(a, b, k, go, ge):
    """Q = x^a y^b, D = x^a z^k y^b with a +1/-128 identity matrix: the best
    alignment either keeps one block or bridges the k-residue insertion with one
    gap run, so S = max(a, b, a + b - Go - (k-1)Ge) (Ge <= Go)."""
    assert ge <= go
    sm = identity_matrix(1, -128)
    x, y, z = 3, 9, 15
    q = [x] * a + [y] * b
    d = [x] * a + [z] * k + [y] * b
    want = max(a, b, a + b - go - (k - 1) * ge)
    assert oracle.pair(q, d, sm, go, ge) == want
    assert oracle.pair(d, q, sm, go, ge) == want


def test_affine_worked_example():
    """a = b = 40, Go/Ge = 10/2, k = 3 gives 80 - 10 - 4 = 66 (64 if a gap of k
    residues were charged Go + k*Ge instead)."""
    sm = identity_matrix(1, -128)
    assert oracle.pair([3] * 40 + [9] * 40, [3] * 40 + [15] * 3 + [9] * 40, sm, 10, 2) == 66


@pytest.mark.parametrize("s,go,plen,tlen", [(-3, 10, 6, 7), (1, 10, 5, 5), (-128, 1, 8, 8),
                                            (-10, 3, 1, 9), (0, 0, 4, 4), (-2, 1, 9, 7)])
def test_single_mismatch(s, go, plen, tlen):
    """Q = P a T, D = P b T where P and T use distinct letters (none repeated,
    none shared, neither a nor b), identity +1/-128 except SM(a,b) = s:
    S = max(|P|+|T|+s, |P|+|T|-2Go, |P|, |T|)."""
    sm = identity_matrix(1, -128)
    a_, b_ = 0, 1
    sm[a_, b_] = sm[b_, a_] = s
    P = list(range(2, 2 + plen))
    T = list(range(2 + plen, 2 + plen + tlen))
    assert len(P) + len(T) <= 18
    q, d = P + [a_] + T, P + [b_] + T
    want = max(plen + tlen + s, plen + tlen - 2 * go, plen, tlen)
    assert oracle.pair(q, d, sm, go, 1) == want


@pytest.mark.parametrize("L,seed", [(1, 0), (50, 1), (997, 2), (4000, 3)])
def test_self_score_is_diagonal_sum(L, seed, blosum):
    """For BLOSUM62 (positive diagonal, SM(x,y) <= (SM(x,x)+SM(y,y))/2) the best
    self-alignment is the gap-free identity alignment: S(Q,Q) = sum SM(q,q)."""
    q = rnd(seed).integers(0, 20, L)
    assert oracle.pair(q, q, blosum, 10, 2) == int(sum(int(blosum[c, c]) for c in q))


def test_self_score_above_int16(blosum):
    """W^3000 against itself: 3000 * 11 = 33000 > 32767."""
    w = [17] * 3000
    assert oracle.pair(w, w, blosum, 10, 2) == 33000


@pytest.mark.parametrize("seed", range(12))
def test_ungapped_equals_kadane(seed, blosum):
    """With Go larger than any achievable gain no gap pays off: S is the best
    diagonal maximum-subarray sum."""
    g = rnd(300 + seed)
    m, n = int(g.integers(1, 60)), int(g.integers(1, 60))
    q, d = g.integers(0, 20, m), g.integers(0, 20, n)
    go = int(blosum.max()) * min(m, n) + 1
    assert oracle.pair(q, d, blosum, go, int(g.integers(0, go + 1))) == kadane_diagonals(q, d, blosum)


@pytest.mark.parametrize("seed", range(12))
def test_lcs_special_case(seed):
    """SM = 1 on identity, 0 otherwise, free gaps: S = longest common subsequence."""
    g = rnd(400 + seed)
    k = int(g.integers(2, 6))
    q, d = g.integers(0, k, int(g.integers(1, 40))), g.integers(0, k, int(g.integers(1, 40)))
    assert oracle.pair(q, d, identity_matrix(1, 0), 0, 0) == lcs_len(q, d)


@pytest.mark.parametrize("seed", range(12))
def test_longest_common_substring_special_case(seed):
    """SM = +1/-128 and Go = Ge = 127 with lengths < 127: S = longest common substring."""
    g = rnd(500 + seed)
    k = int(g.integers(2, 5))
    q, d = g.integers(0, k, int(g.integers(1, 60))), g.integers(0, k, int(g.integers(1, 60)))
    assert oracle.pair(q, d, identity_matrix(1, -128), 127, 127) == lcsubstr_len(q, d)


def test_empty_sequences(blosum):
    assert oracle.pair([], [1, 2, 3], blosum, 10, 2) == 0
    assert oracle.pair([1, 2], [], blosum, 10, 2) == 0
    assert oracle.pair([], [], blosum, 10, 2) == 0


def test_all_negative_is_zero():
    sm = np.full((20, 20), -5, dtype=np.int8)
    assert oracle.pair([1, 2, 3], [1, 2, 3], sm, 1, 1) == 0


# ---------------------------------------------------------------- batch entry point
def test_scores_matches_pairs(blosum):
    g = rnd(7)
    lens = g.integers(1, 80, 40)
    offs = np.concatenate([[0], np.cumsum(lens)])
    res = g.integers(0, 20, offs[-1]).astype(np.int8)
    q = g.integers(0, 20, 33)
    allv = oracle.scores(q, res, offs, blosum, 10, 2, threads=3)
    for k in range(40):
        assert allv[k] == oracle.pair(q, res[offs[k]:offs[k + 1]], blosum, 10, 2)
    idx = np.array([39, 0, 5, 5])
    assert list(oracle.scores(q, res, offs, blosum, 10, 2, idx=idx, threads=2)) == [allv[i] for i in idx]


def test_topk_oracle():
    s = np.array([5, 9, 9, 1, 0, 9, 7])
    ts, ti = oracle.topk(s, 4)
    assert list(ts) == [9, 9, 9, 7] and list(ti) == [1, 2, 5, 6]
    ts, ti = oracle.topk(np.array([3, 4]), 4)
    assert list(ts) == [4, 3, -1, -1] and list(ti) == [1, 0, -1, -1]
