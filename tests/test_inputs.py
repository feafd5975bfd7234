"""Inputs: BLOSUM62 transcription checks, alphabet, synthetic workload recipe."""
import os

import numpy as np
import pytest

import oracle
from inputs import ALPHABET, background_frequencies, blosum62, decode, encode, synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_blosum62_properties():
    B = blosum62().astype(np.int64)
    assert B.shape == (20, 20)
    assert (B == B.T).all()
    assert B.min() == -4 and B.max() == 11
    diag = dict(zip(ALPHABET, np.diag(B)))
    assert diag == dict(A=4, R=5, N=6, D=6, C=9, Q=5, E=5, G=6, H=8, I=4, L=4, K=5, M=5,
                        F=6, P=7, S=4, T=5, W=11, Y=7, V=4)
    assert int(np.trace(B)) == 116
    # weak diagonal dominance, needed for the self-score closed form
    assert (2 * B <= np.add.outer(np.diag(B), np.diag(B))).all()
    # a log-odds matrix has negative expected score under the background
    f = background_frequencies()
    assert float(f @ B @ f) < 0
    # spot values of the published table
    for a, b, v in [("W", "Y", 2), ("I", "V", 3), ("D", "E", 2), ("C", "E", -4), ("F", "P", -4),
                    ("L", "D", -4), ("H", "Y", 2), ("S", "T", 1), ("N", "W", -4), ("K", "R", 2)]:
        assert B[ALPHABET.index(a), ALPHABET.index(b)] == v


def test_background_frequencies():
    f = background_frequencies()
    assert f.shape == (20,) and abs(f.sum() - 1) < 1e-12 and (f > 0.01).all()
    assert ALPHABET[int(np.argmax(f))] == "L" and ALPHABET[int(np.argmin(f))] == "W"


def test_encode_decode():
    s = "MKTAYIAKQRW"
    assert decode(encode(s)) == s
    with pytest.raises(ValueError):
        encode("MKX")


def test_generator_is_deterministic():
    q1, db1 = synth.workload1()
    q2, db2 = synth.workload1()
    assert (q1[0] == q2[0]).all() and (db1.residues == db2.residues).all()
    assert (db1.offsets == db2.offsets).all()


def test_workload1_shape():
    qs, db = synth.workload1()
    assert len(qs) == 1 and qs[0].size == 144
    assert db.n == 2000 and db.lengths.min() >= 20 and db.lengths.max() <= 1100
    assert 250 < np.median(db.lengths) < 350
    assert db.residues.min() >= 0 and db.residues.max() <= 19


def test_workload2_query_lengths():
    assert synth.WL2_QLENS[0] == 144 and synth.WL2_QLENS[-1] == 5478 and len(synth.WL2_QLENS) == 20
    assert sum(synth.WL2_QLENS) == 30747


def test_small_sp_db_recipe():
    db = synth.sp570k(n=20_000)
    L = db.lengths
    assert L.max() == 35_000 and (L[-16:] >= 5000).all()
    assert len(db.sentinels) == 3 and (L[db.sentinels] >= synth.SENTINEL_BLOCK).all()
    assert 270 < np.median(L[:-16]) < 330


def test_sentinel_scores_exceed_int16(blosum):
    """The W-rich block alone self-aligns above 2^15 - 1, so sentinel subjects
    exercise the exact 32-bit recompute path."""
    qs = synth.workload2_queries()
    k = synth.WL2_QLENS.index(3735)
    block = qs[k][60:60 + synth.SENTINEL_BLOCK]
    assert int(sum(int(blosum[c, c]) for c in block)) > 32767
    db = synth.sp570k(n=20_000)
    s = oracle.scores(qs[k], db.residues, db.offsets, blosum, 10, 2, idx=db.sentinels)
    assert (s > 32767).all()


def test_poisson_arrivals():
    t = synth.poisson_arrivals(2.0, 4000)
    assert (np.diff(t) > 0).all()
    assert abs(4000 / t[-1] - 2.0) < 0.15


def test_golden_closed_forms(blosum):
    """Hand-derived scores in tests/golden/closed_forms.txt."""
    def expand(tok):
        out = []
        for part in tok.split():
            if "^" in part:
                c, k = part.split("^")
                out += [c] * int(k)
            else:
                out += list(part)
        return encode("".join(out))
    from refs import identity_matrix
    n = 0
    for line in open(os.path.join(GOLDEN, "closed_forms.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        q, d, mname, go, ge, s, _ = [x.strip() for x in line.split("|")]
        sm = blosum if mname == "BLOSUM62" else identity_matrix(1, -128)
        assert oracle.pair(expand(q), expand(d), sm, int(go), int(ge)) == int(s), line
        n += 1
    assert n >= 5


def test_blosum62_extended_alphabet():
    from inputs import ALPHABET24, blosum62, blosum62_24
    m = blosum62_24()
    assert ALPHABET24 == "ARNDCQEGHILKMFPSTWYVBZX*"
    assert m.shape == (24, 24) and (m == m.T).all()
    assert (m[:20, :20] == blosum62()).all()
    b = blosum62()
    N, D, Q, E = (ALPHABET24.index(c) for c in "NDQE")
    # the ambiguity codes lie between the scores of the residues they stand for
    assert ((m[20, :20] >= np.minimum(b[N], b[D])) & (m[20, :20] <= np.maximum(b[N], b[D]))).all()
    assert ((m[21, :20] >= np.minimum(b[Q], b[E])) & (m[21, :20] <= np.maximum(b[Q], b[E]))).all()
    assert (m[22, :23] <= 0).all() and m[22, 22] == -1
    assert (m[23, :23] == -4).all() and m[23, 23] == 1
