"""CPU emulation of the 16-bit cell arithmetic of the GPU sweep, against the oracle.

The sweep keeps Eq. 1-3 (Sec. II-B) in packed 16-bit lanes and takes its
three-input maxima with a half-float instruction on biased integers.  That is
exact only because of facts about 16-bit patterns that this file checks on the
CPU, with numpy's IEEE half floats (which keep subnormals):

* non-negative 16-bit integers below 0x7C00 order like the half floats with the
  same bits -- most of them (1..1023) are subnormal halves, so the kernels need
  f16 subnormals preserved (a flush-to-zero maximum gets scores wrong, shown
  below);
* 0x7C00 and above are +infinity or NaN, which the IEEE maximum propagates, so
  a score that reached them is detected and recomputed in 32 bits;
* the local form (bias c = minus the lowest score, floors, saturating
  subtractions, padding that scores 0) gives S - c = the oracle's score for
  every pair whose S stays below 0x7C00, and flags exactly the others;
* the end-to-end form (global, semi-global: bias in the middle of the range,
  no floor, running minimum and maximum of H) is exact for every pair whose
  values stay in [128, 0x7C00 - 128) and flags the rest.

The emulation follows the kernels' per-cell order, vectorised over many
subjects at once as the lanes of a wave are.  It shares nothing with the GPU
code and only checks the arithmetic; the GPU parity tests check the kernels.
"""
import numpy as np
import pytest

import oracle
from inputs import blosum62, synth
from refs import identity_matrix

KSAT = 0x7C00
MODE_BIAS = 0x3E00
MODE_LO, MODE_TOP = 128, 0x7C00 - 128


# ------------------------------------------------------------------ 16-bit primitives
def f16max(*xs, ftz=False):
    """IEEE maximum of half floats given as uint16 patterns (NaN propagates).
    ftz=True flushes subnormal inputs to zero first (what a flushing mode does)."""
    vals = []
    for x in xs:
        v = np.asarray(x, dtype=np.uint16).view(np.float16)
        if ftz:
            v = np.where(np.abs(v) < np.float16(2.0 ** -14), np.float16(0), v)
        vals.append(v)
    out = vals[0]
    for v in vals[1:]:
        out = np.maximum(out, v)
    return out.astype(np.float16).view(np.uint16)


def f16min(*xs):
    vals = [np.asarray(x, dtype=np.uint16).view(np.float16) for x in xs]
    out = vals[0]
    for v in vals[1:]:
        out = np.minimum(out, v)
    return out.view(np.uint16)


def add_i16_clamp(a, b):
    """Signed 16-bit addition with saturation (patterns in, patterns out)."""
    s = np.asarray(a, np.uint16).view(np.int16).astype(np.int32) + np.asarray(b, np.int32)
    return np.clip(s, -32768, 32767).astype(np.int16).view(np.uint16)


def sub_u16_clamp(a, g):
    """Unsigned 16-bit subtraction saturating at 0."""
    return np.maximum(np.asarray(a, np.uint16).astype(np.int32) - int(min(g, 65535)), 0).astype(np.uint16)


def max_i16(a, b):
    return np.maximum(np.asarray(a, np.uint16).view(np.int16), np.asarray(b, np.uint16).view(np.int16)).view(np.uint16)


# ------------------------------------------------------------------ pattern facts
def test_nonnegative_patterns_below_0x7c00_order_as_half_floats():
    x = np.arange(0, KSAT, dtype=np.uint16)
    f = x.view(np.float16).astype(np.float64)
    assert np.all(np.diff(f) > 0)                      # strictly increasing: max of halves = max of integers
    sub = f[1:1024]
    assert np.all((sub > 0) & (sub < 2.0 ** -14))       # 1..1023 are subnormal halves


def test_infinity_and_nan_patterns_propagate_through_maxima():
    special = np.arange(KSAT, 0x8000, dtype=np.uint16)              # +inf and positive NaNs
    every = np.arange(0, 0x8000, dtype=np.uint16)
    a = np.repeat(special, every.size)
    b = np.tile(every, special.size)
    assert (f16max(a, b) >= KSAT).all() and (f16max(b, a) >= KSAT).all()
    assert (f16max(b, a, b[::-1]) >= KSAT).all()
    # a saturating sum lands at 0x7FFF, a NaN pattern: it is flagged, never mistaken for a score
    assert add_i16_clamp(np.uint16(0x7F90), 127) == 0x7FFF


def test_sums_below_0x7c00_are_never_clamped():
    """hd = H + SM with H below 0x7C00 and H + SM >= 0 is exact: a clamped sum
    needs an H that was already flagged."""
    x = np.repeat(np.arange(0, KSAT, dtype=np.int64), 256)
    s = np.tile(np.arange(-128, 128, dtype=np.int64), KSAT)
    keep = x + s >= 0
    assert (add_i16_clamp(x[keep].astype(np.uint16), s[keep]).astype(np.int64) == (x + s)[keep]).all()


def test_integer_and_half_maxima_agree_below_0x7c00():
    rng = np.random.default_rng(1)
    a = rng.integers(0, KSAT, 200_000).astype(np.uint16)
    b = rng.integers(0, KSAT, 200_000).astype(np.uint16)
    c = rng.integers(0, KSAT, 200_000).astype(np.uint16)
    assert (f16max(a, b, c) == np.maximum(np.maximum(a, b), c)).all()
    assert (f16min(a, b, c) == np.minimum(np.minimum(a, b), c)).all()
    assert (max_i16(a, b) == np.maximum(a, b)).all()
    # with subnormals flushed the maximum of two small values is not the larger one
    assert (f16max(np.uint16(3), np.uint16(9), ftz=True) != 9).all()


# ------------------------------------------------------------------ local form
def _pad_batch(q, subjects, rows_mult=16, cols_mult=4):
    """Query padded to a whole pass (rows_mult rows) and subjects padded to the
    widest one rounded up to 4 columns, with -1 marking padding (scores 0)."""
    m = q.size
    hq = -(-m // rows_mult) * rows_mult
    width = max([s.size for s in subjects] + [1])
    width = -(-width // cols_mult) * cols_mult
    Q = np.full(hq, -1, np.int64)
    Q[:m] = q
    D = np.full((len(subjects), width), -1, np.int64)
    for k, s in enumerate(subjects):
        D[k, :s.size] = s
    return Q, D


def _scores(sm, Q, D):
    """P[i, k, j] = SM(Q[i], D[k, j]) with padding (-1 on either side) scoring 0, as the profile does."""
    A = sm.shape[0]
    ext = np.zeros((A + 1, A + 1), np.int32)          # index A = padding
    ext[:A, :A] = sm
    qi = np.where(Q >= 0, Q, A)
    dj = np.where(D >= 0, D, A)
    return ext[qi[:, None, None], dj[None, :, :]]


def emulate_local16(q, subjects, sm, go, ge, ftz=False):
    """The 16-bit local sweep: (score - c or -1 when flagged, flagged) per subject."""
    sm = np.asarray(sm, np.int32)
    c = max(0, -int(sm.min()))
    Q, D = _pad_batch(q, subjects)
    nsub, width = D.shape
    P = _scores(sm, Q, D)
    cc = np.full(nsub, c, np.uint16)
    H = np.full((Q.size, nsub), c, np.uint16)     # H of every row at the last column done (column 0: c)
    E = np.full((Q.size, nsub), c, np.uint16)     # E advanced to the next column (floored at c)
    S = np.full(nsub, c, np.uint16)
    for j in range(width):
        diag = cc.copy()                         # H[0][j-1]: the zero border, raised to c
        F = np.zeros(nsub, np.uint16)            # F[1][j]: the zero border read as 0 (may stay below c)
        for i in range(Q.size):
            hd = add_i16_clamp(diag, P[i, :, j])
            h = f16max(hd, E[i], F, ftz=ftz)
            es = sub_u16_clamp(E[i], ge)
            hgo = sub_u16_clamp(h, go)
            fs = sub_u16_clamp(F, ge)
            E[i] = f16max(es, hgo, cc, ftz=ftz)
            F = max_i16(fs, hgo)
            S = f16max(S, h, ftz=ftz)
            diag = H[i].copy()
            H[i] = h
    flagged = S >= KSAT
    return np.where(flagged, -1, S.astype(np.int64) - c), flagged


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_local16_blosum62_equals_oracle(seed):
    rng = np.random.default_rng(seed)
    sm = blosum62()
    q = synth.background_residues(rng, int(rng.integers(20, 70)))
    subs = [synth.background_residues(rng, int(L)) for L in rng.integers(0, 90, 48)]
    subs[3] = q[5:40].copy()                                        # a strong hit
    got, flagged = emulate_local16(q, subs, sm, 10, 2)
    want = np.array([oracle.pair(q, s, sm, 10, 2) for s in subs])
    assert not flagged.any()
    assert (got == want).all(), np.nonzero(got != want)


@pytest.mark.parametrize("go,ge", [(0, 0), (1, 9), (40, 3), (70000, 70000)])
def test_local16_extreme_matrices_and_gaps(go, ge):
    rng = np.random.default_rng(go + 7 * ge)
    for sm in (rng.integers(-128, 128, (20, 20)).astype(np.int8), np.abs(rng.integers(0, 5, (20, 20))).astype(np.int8)):
        q = rng.integers(0, 20, 37).astype(np.int8)
        subs = [rng.integers(0, 20, int(L)).astype(np.int8) for L in rng.integers(0, 60, 40)]
        got, flagged = emulate_local16(q, subs, sm, go, ge)
        want = np.array([oracle.pair(q, s, sm, go, ge) for s in subs])
        assert (want[~flagged] == got[~flagged]).all()
        assert (flagged == (want + max(0, -int(sm.min())) >= KSAT)).all()


def test_local16_flags_exactly_the_saturated_pairs():
    """+127 on the diagonal: a run of 250 identical residues crosses 0x7C00 - c."""
    sm = identity_matrix(127, -128)
    rng = np.random.default_rng(5)
    q = np.full(260, 4, np.int8)
    subs = [np.full(int(L), 4, np.int8) for L in (240, 244, 245, 246, 250, 259)]
    subs += [rng.integers(0, 20, 120).astype(np.int8) for _ in range(4)]
    got, flagged = emulate_local16(q, subs, sm, 10, 2)
    want = np.array([oracle.pair(q, s, sm, 10, 2) for s in subs])
    c = 128
    assert (flagged == (want + c >= KSAT)).all()
    assert flagged.sum() >= 2 and (~flagged).sum() >= 4
    assert (got[~flagged] == want[~flagged]).all()


def test_flushing_subnormals_breaks_the_scores():
    """The same arithmetic with a flush-to-zero maximum is wrong: the kernels rely
    on the f16 denormal mode that preserves subnormals."""
    rng = np.random.default_rng(11)
    sm = blosum62()
    q = synth.background_residues(rng, 40)
    subs = [synth.background_residues(rng, 50) for _ in range(16)]
    got, _ = emulate_local16(q, subs, sm, 10, 2, ftz=True)
    want = np.array([oracle.pair(q, s, sm, 10, 2) for s in subs])
    assert (got != want).any()


# ------------------------------------------------------------------ end-to-end modes
def _border(k, go, ge):
    return 0 if k <= 0 else -(go + (k - 1) * min(go, ge))


def emulate_mode16(q, subjects, sm, go, ge, mode, bias):
    """The 16-bit end-to-end sweep (mode "global" or "semiglobal"): (score, in_range)."""
    sm = np.asarray(sm, np.int32)
    m = q.size
    Q, D = _pad_batch(q, subjects)
    nsub, width = D.shape
    P = _scores(sm, Q, D)
    lens = np.array([s.size for s in subjects])
    enc = lambda v: np.clip(np.asarray(v, np.int64) + bias, 0, 0x7FFF).astype(np.uint16)  # noqa: E731
    rows = Q.size
    H = np.stack([np.full(nsub, enc(_border(min(i + 1, m), go, ge)), np.uint16) for i in range(rows)])
    E = np.stack([sub_u16_clamp(H[i], go) for i in range(rows)])
    hm = enc(_border(m, go, ge))
    S = np.where((mode == "semiglobal") | (lens == 0), hm, 0).astype(np.uint16)
    ta = np.array([enc(_border(n, go, ge)) if mode == "global" else hm for n in lens], np.uint16)
    lmin = np.minimum(np.full(nsub, hm, np.uint16), ta)
    lmax = np.zeros(nsub, np.uint16)
    for j in range(width):
        col_border = [_border(min(j + 1, n), go, ge) if mode == "global" else 0 for n in lens]
        top = enc(col_border)
        diag = enc(_border(0, go, ge)) if j == 0 else prev_top
        diag = np.broadcast_to(diag, (nsub,)).astype(np.uint16)
        F = sub_u16_clamp(top, go)
        prev_top = top
        for i in range(rows):
            hd = add_i16_clamp(diag, P[i, :, j])
            h = f16max(hd, E[i], F)
            es = sub_u16_clamp(E[i], ge)
            hgo = sub_u16_clamp(h, go)
            fs = sub_u16_clamp(F, ge)
            E[i] = max_i16(es, hgo)
            F = max_i16(fs, hgo)
            lmax = f16max(lmax, h)
            lmin = f16min(lmin, h)
            if i == m - 1:
                if mode == "global":
                    S = np.where(j == lens - 1, h, S)
                else:
                    S = np.where(j < lens, f16max(S, h), S)
            diag = H[i].copy()
            H[i] = h
    in_range = (lmin >= MODE_LO) & (lmax < MODE_TOP)
    return S.astype(np.int64) - bias, in_range


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
@pytest.mark.parametrize("seed", [0, 1])
def test_mode16_in_range_pairs_equal_oracle(mode, seed):
    rng = np.random.default_rng(40 + seed)
    sm = blosum62()
    q = synth.background_residues(rng, int(rng.integers(5, 60)))
    subs = [synth.background_residues(rng, int(L)) for L in rng.integers(0, 80, 40)]
    subs[1] = q.copy()
    bias = MODE_BIAS if mode == "global" else min(MODE_BIAS, 128 + 10 + (q.size - 1) * 2)
    got, ok = emulate_mode16(q, subs, sm, 10, 2, mode, bias)
    want = np.array([oracle.pair_mode(q, s, sm, 10, 2, mode) for s in subs])
    assert ok.all()
    assert (got == want).all(), (np.nonzero(got != want), got, want)


@pytest.mark.parametrize("mode", ["global", "semiglobal"])
def test_mode16_out_of_range_pairs_are_flagged(mode):
    """-128 mismatches drive global values below the range and runs of +127 matches
    drive values above it (semi-global H never falls below the gap run down the
    query, so there only the top can be left); every pair whose score the 16-bit
    form does not reproduce must be flagged."""
    rng = np.random.default_rng(7)
    sm = identity_matrix(127, -128)
    m = 140 if mode == "global" else 252
    q = np.full(m, 4, np.int8)
    subs = [np.full(int(L), 4, np.int8) for L in (0, 3, 60, 130, m)]
    subs += [rng.integers(0, 20, int(L)).astype(np.int8) for L in (10, 90, 200)]
    for go, ge in ((10, 2), (300, 60)):
        bias = MODE_BIAS if mode == "global" else min(MODE_BIAS, 128 + go + (q.size - 1) * ge)
        got, ok = emulate_mode16(q, subs, sm, go, ge, mode, bias)
        want = np.array([oracle.pair_mode(q, s, sm, go, ge, mode) for s in subs])
        assert (got[ok] == want[ok]).all()
        assert (~ok).any()
        wrong = got != want
        assert not (wrong & ok).any()


# ------------------------------------------------------------------ global mode, column-offset cells
def emulate_global_offset16(q, subjects, sm, go, ge, bias):
    """The 16-bit global sweep on column-offset cells (Ge <= Go): every cell holds H'[i][j] = H[i][j] - g(j),
    g the row-0 gap run, so that the row-0 border is 0 and a long subject's border no longer leaves the
    range.  Then the diagonal gains Ge (the profile carries SM + Ge on real residues, 0 on padding), E
    extends for free and opens at Go - Ge, F is unchanged; column 0 as a diagonal reads g(i) + Go - Ge,
    E'[i][1] = g(i).  Returns (H'[m][n] + g(n), in_range) per subject."""
    assert ge <= go
    sm = np.asarray(sm, np.int32)
    m = q.size
    Q, D = _pad_batch(q, subjects)
    nsub, width = D.shape
    P = _scores(sm, Q, D)
    real = (Q[:, None, None] >= 0) & (D[None, :, :] >= 0)
    P = np.where(real, P + ge, 0)
    lens = np.array([s.size for s in subjects])
    enc = lambda v: np.clip(np.asarray(v, np.int64) + bias, 0, 0x7FFF).astype(np.uint16)  # noqa: E731
    rows = Q.size
    H = np.stack([np.full(nsub, enc(_border(min(i + 1, m), go, ge) + go - ge), np.uint16) for i in range(rows)])
    E = np.stack([np.full(nsub, enc(_border(min(i + 1, m), go, ge)), np.uint16) for i in range(rows)])
    hm = enc(_border(m, go, ge))
    S = np.where(lens == 0, hm, 0).astype(np.uint16)
    lmin = np.full(nsub, hm, np.uint16)
    lmax = np.zeros(nsub, np.uint16)
    top = np.full(nsub, enc(0), np.uint16)
    for j in range(width):
        diag = np.full(nsub, enc(go - ge), np.uint16) if j == 0 else top
        F = sub_u16_clamp(top, go)
        for i in range(rows):
            hd = add_i16_clamp(diag, P[i, :, j])
            h = f16max(hd, E[i], F)
            hge = sub_u16_clamp(h, go - ge)
            hgo = sub_u16_clamp(h, go)
            fs = sub_u16_clamp(F, ge)
            E[i] = max_i16(E[i], hge)
            F = max_i16(fs, hgo)
            lmax = f16max(lmax, h)
            lmin = f16min(lmin, h)
            if i == m - 1:
                S = np.where(j == lens - 1, h, S)
            diag = H[i].copy()
            H[i] = h
    in_range = (lmin >= MODE_LO) & (lmax < MODE_TOP)
    out = S.astype(np.int64) - bias + np.array([_border(n, go, ge) for n in lens])
    return out, in_range


def _offset_bias(m, go, ge):
    return min(MODE_BIAS, 128 + go + (m - 1) * ge)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_global_offset16_equals_oracle(seed):
    """In-range pairs equal the oracle's global score, including subjects far longer than the query whose
    row-0 gap run alone would leave the range of plain biased cells."""
    rng = np.random.default_rng(60 + seed)
    sm = blosum62()
    q = synth.background_residues(rng, int(rng.integers(1, 50)))
    subs = [synth.background_residues(rng, int(L)) for L in rng.integers(0, 90, 30)]
    subs[1] = q.copy()
    subs[2] = np.zeros(0, np.int8)
    for go, ge in ((10, 2), (3, 3), (11, 1), (0, 0)):
        got, ok = emulate_global_offset16(q, subs, sm, go, ge, _offset_bias(q.size, go, ge))
        want = np.array([oracle.pair_mode(q, s, sm, go, ge, "global") for s in subs])
        assert ok.all(), (go, ge)
        assert (got == want).all(), (go, ge, np.nonzero(got != want), got, want)


def test_global_offset16_long_subjects_stay_in_range():
    """A 20-residue query against subjects of up to 9,000 residues: the gap runs along the subjects reach
    -18,000, below what plain biased cells hold, while the offset cells stay in range and exact."""
    rng = np.random.default_rng(70)
    sm = blosum62()
    q = synth.background_residues(rng, 20)
    subs = [synth.background_residues(rng, L) for L in (1, 19, 20, 21, 500, 9000)]
    bias = _offset_bias(q.size, 10, 2)
    assert _border(9000, 10, 2) + MODE_BIAS < MODE_LO          # out of range for the plain cells
    got, ok = emulate_global_offset16(q, subs, sm, 10, 2, bias)
    want = np.array([oracle.pair_mode(q, s, sm, 10, 2, "global") for s in subs])
    assert ok.all()
    assert (got == want).all(), (got, want)


def test_global_offset16_out_of_range_pairs_are_flagged():
    """Runs of +127 matches drive H' above the range (it never falls below g(m), which the bias covers,
    -128 mismatches included); every pair whose score the offset cells do not reproduce is flagged."""
    rng = np.random.default_rng(71)
    sm = identity_matrix(127, -128)
    q = np.full(260, 4, np.int8)
    subs = [np.full(int(L), 4, np.int8) for L in (0, 3, 60, 250, 260, 400)]
    subs += [rng.integers(0, 20, int(L)).astype(np.int8) for L in (10, 90, 200)]
    for go, ge in ((10, 2), (300, 60)):
        got, ok = emulate_global_offset16(q, subs, sm, go, ge, _offset_bias(q.size, go, ge))
        want = np.array([oracle.pair_mode(q, s, sm, go, ge, "global") for s in subs])
        assert (got[ok] == want[ok]).all()
        assert (~ok).any()
        assert not ((got != want) & ok).any()
