"""Amino-acid alphabet, the BLOSUM62 substitution matrix and background
residue frequencies.

These are *inputs* to the search (the paper configures its runs with BLOSUM62
and gap penalties 10/2, Sec. IV-A "Experimental Design"); they hold no part of
the alignment arithmetic.  Both the GPU library and the CPU oracle receive the
matrix as an argument.

Provenance
----------
* BLOSUM62: Henikoff & Henikoff, "Amino acid substitution matrices from protein
  blocks", PNAS 89:10915 (1992); the 20x20 standard-amino-acid block of the
  table distributed by NCBI as ``BLOSUM62`` (half-bit units).  The paper names
  the matrix but does not print it.
* Background frequencies: Robinson & Robinson, "Distribution of glutamine and
  asparagine residues and their near neighbors in peptides and proteins",
  PNAS 88:8880 (1991), the set BLAST uses for its composition statistics.
  The paper does not state a distribution; these only shape synthetic inputs.

Alphabet order and codes: ``ARNDCQEGHILKMFPSTWYV`` -> 0..19.  The extended
alphabet ``ARNDCQEGHILKMFPSTWYVBZX*`` -> 0..23 adds the ambiguity codes B (N or
D), Z (Q or E), X (any) and the stop/terminal symbol *, with the extra rows and
columns of the same NCBI table (``blosum62_24``).
"""
from __future__ import annotations

import numpy as np

ALPHABET = "ARNDCQEGHILKMFPSTWYV"
N_RES = 20

_BLOSUM62_ROWS = """
A  4 -1 -2 -2  0 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -3 -2  0
R -1  5  0 -2 -3  1  0 -2  0 -3 -2  2 -1 -3 -2 -1 -1 -3 -2 -3
N -2  0  6  1 -3  0  0  0  1 -3 -3  0 -2 -3 -2  1  0 -4 -2 -3
D -2 -2  1  6 -3  0  2 -1 -1 -3 -4 -1 -3 -3 -1  0 -1 -4 -3 -3
C  0 -3 -3 -3  9 -3 -4 -3 -3 -1 -1 -3 -1 -2 -3 -1 -1 -2 -2 -1
Q -1  1  0  0 -3  5  2 -2  0 -3 -2  1  0 -3 -1  0 -1 -2 -1 -2
E -1  0  0  2 -4  2  5 -2  0 -3 -3  1 -2 -3 -1  0 -1 -3 -2 -2
G  0 -2  0 -1 -3 -2 -2  6 -2 -4 -4 -2 -3 -3 -2  0 -2 -2 -3 -3
H -2  0  1 -1 -3  0  0 -2  8 -3 -3 -1 -2 -1 -2 -1 -2 -2  2 -3
I -1 -3 -3 -3 -1 -3 -3 -4 -3  4  2 -3  1  0 -3 -2 -1 -3 -1  3
L -1 -2 -3 -4 -1 -2 -3 -4 -3  2  4 -2  2  0 -3 -2 -1 -2 -1  1
K -1  2  0 -1 -3  1  1 -2 -1 -3 -2  5 -1 -3 -1  0 -1 -3 -2 -2
M -1 -1 -2 -3 -1  0 -2 -3 -2  1  2 -1  5  0 -2 -1 -1 -1 -1  1
F -2 -3 -3 -3 -2 -3 -3 -3 -1  0  0 -3  0  6 -4 -2 -2  1  3 -1
P -1 -2 -2 -1 -3 -1 -1 -2 -2 -3 -3 -1 -2 -4  7 -1 -1 -4 -3 -2
S  1 -1  1  0 -1  0  0  0 -1 -2 -2  0 -1 -2 -1  4  1 -3 -2 -2
T  0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  1  5 -2 -2  0
W -3 -3 -4 -4 -2 -2 -3 -2 -2 -3 -2 -3 -1  1 -4 -3 -2 11  2 -3
Y -2 -2 -2 -3 -2 -1 -2 -3  2 -1 -1 -2 -1  3 -3 -2 -2  2  7 -1
V  0 -3 -3 -3 -1 -2 -2 -3 -3  3  1 -2  1 -1 -2 -2  0 -3 -1  4
"""

ALPHABET24 = ALPHABET + "BZX*"

# The rows and columns B, Z, X, * of the NCBI BLOSUM62 table, in ALPHABET24
# column order (the 20 x 20 block above is unchanged).
_BLOSUM62_EXTRA = """
B -2 -1  3  4 -3  0  1 -1  0 -3 -4  0 -3 -3 -2  0 -1 -4 -3 -3  4  1 -1 -4
Z -1  0  0  1 -3  3  4 -2  0 -3 -3  1 -1 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
X  0 -1 -1 -1 -2 -1 -1 -1 -1 -1 -1 -1 -1 -1 -2  0  0 -2 -1 -1 -1 -1 -1 -4
* -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4  1
"""

# Robinson & Robinson (1991) background frequencies, in ALPHABET order.
_ROBINSON = {
    "A": 0.07805, "R": 0.05129, "N": 0.04487, "D": 0.05364, "C": 0.01925,
    "Q": 0.04264, "E": 0.06295, "G": 0.07377, "H": 0.02199, "I": 0.05142,
    "L": 0.09019, "K": 0.05744, "M": 0.02243, "F": 0.03856, "P": 0.05203,
    "S": 0.07120, "T": 0.05841, "W": 0.01330, "Y": 0.03216, "V": 0.06441,
}


def blosum62() -> np.ndarray:
    """BLOSUM62 as int8[20, 20], row = query residue, column = subject residue."""
    rows = [ln.split() for ln in _BLOSUM62_ROWS.strip().splitlines()]
    order = "".join(r[0] for r in rows)
    if order != ALPHABET:
        raise AssertionError("BLOSUM62 row order does not match the alphabet")
    return np.array([[int(v) for v in r[1:]] for r in rows], dtype=np.int8)


def blosum62_24() -> np.ndarray:
    """BLOSUM62 over ALPHABET24 as int8[24, 24] (symmetric)."""
    m = np.zeros((24, 24), dtype=np.int8)
    m[:20, :20] = blosum62()
    rows = [ln.split() for ln in _BLOSUM62_EXTRA.strip().splitlines()]
    if "".join(r[0] for r in rows) != "BZX*":
        raise AssertionError("extra BLOSUM62 rows out of order")
    for k, r in enumerate(rows):
        m[20 + k, :] = [int(v) for v in r[1:]]
        m[:, 20 + k] = m[20 + k, :]
    return m


def background_frequencies() -> np.ndarray:
    """float64[20] residue frequencies (normalised to sum to 1)."""
    f = np.array([_ROBINSON[a] for a in ALPHABET], dtype=np.float64)
    return f / f.sum()


def encode(seq: str) -> np.ndarray:
    """Letters -> int8 codes 0..19.  Raises ValueError on any other letter."""
    lut = {c: i for i, c in enumerate(ALPHABET)}
    try:
        return np.array([lut[c] for c in seq.upper()], dtype=np.int8)
    except KeyError as e:
        raise ValueError(f"residue {e.args[0]!r} is not one of {ALPHABET}") from None


def decode(codes) -> str:
    return "".join(ALPHABET[int(c)] for c in np.asarray(codes).ravel())
