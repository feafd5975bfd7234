"""CPU oracle for the Smith-Waterman / Gotoh protein database search.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links
or executes anything here, and nothing here uses the GPU library.

* ``pair`` / ``scores``: the score S of Eq. 1-3 (Sec. II-B) computed by the
  plain C implementation in ``sw_oracle.c`` (int64 cells, one row at a time).
* ``align``: the alignment behind a score (traceback from the highest H,
  Sec. II-B), with a stated canonical choice among equal-scoring alignments;
  full matrices, small inputs only.
* ``topk``: the top-ranked subjects of a score vector (Sec. II-B, database
  search keeps alignments only for the top-ranked subjects), ordered by score
  descending then subject index ascending, padded with (-1, -1).
* ``pair_neginf``: a second, independently written form of the same
  recurrence (minus-infinity borders, column-major sweep) in pure Python, for
  small inputs only.

Parity pins (tests marked ``not gpu``): brute-force enumeration of local
alignments, closed forms, textbook special cases and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no vector intrinsics)."""
    if force or not os.path.exists(LIB_PATH):
        src = os.path.join(_HERE, "sw_oracle.c")
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
                        src, "-o", tmp], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.sw_oracle_pair.restype = ctypes.c_int64
        lib.sw_oracle_pair.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64]
        lib.sw_oracle_scores.restype = ctypes.c_int
        lib.sw_oracle_scores.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int64, P, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P]
        lib.sw_oracle_pair_mode.restype = ctypes.c_int64
        lib.sw_oracle_pair_mode.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int64, ctypes.c_int64]
        lib.sw_oracle_align.restype = ctypes.c_int64
        lib.sw_oracle_align.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, P, ctypes.c_char_p, ctypes.c_int64]
        _lib = lib
    return _lib


def _i8(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int8))


def _matrix(sm):
    """int8 square substitution matrix (alphabet x alphabet, indexed [query, subject])."""
    sm = _i8(sm)
    assert sm.ndim == 2 and sm.shape[0] == sm.shape[1] and sm.shape[0] >= 1
    return sm


def pair(q, d, sm, go: int, ge: int) -> int:
    """Score of one pair; q, d residue codes 0..A-1, sm int8[A,A] indexed [query, subject]."""
    q, d, sm = _i8(q), _i8(d), _matrix(sm)
    v = _load().sw_oracle_pair(q.ctypes.data, q.size, d.ctypes.data, d.size, sm.ctypes.data, sm.shape[0],
                               int(go), int(ge))
    if v < 0:
        raise MemoryError("oracle allocation failed")
    return int(v)


MODES = {"local": 0, "global": 1, "semiglobal": 2}


def pair_mode(q, d, sm, go: int, ge: int, mode: str) -> int:
    """Score of one pair in ``mode`` ("local", "global" or "semiglobal"; see
    ``sw_oracle_pair_mode``)."""
    q, d, sm = _i8(q), _i8(d), _matrix(sm)
    v = _load().sw_oracle_pair_mode(q.ctypes.data, q.size, d.ctypes.data, d.size, sm.ctypes.data, sm.shape[0],
                                    int(go), int(ge), MODES[mode])
    if v == -(1 << 63):
        raise MemoryError("oracle allocation failed")
    return int(v)


def default_threads() -> int:
    """Threads for a call that names none: the cores this process may run on,
    at most 16 (a GPU host's share per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def scores(q, residues, offsets, sm, go: int, ge: int, idx=None, threads: int | None = None,
           mode: str = "local") -> np.ndarray:
    """int64 scores of query ``q`` against subjects ``idx`` (default: all) of a
    database given by concatenated ``residues`` and ``offsets[n+1]``."""
    q, residues, sm = _i8(q), _i8(residues), _matrix(sm)
    offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    n = offsets.size - 1
    if idx is None:
        count, idx_ptr, keep = n, None, None
    else:
        keep = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        if keep.size and (keep.min() < 0 or keep.max() >= n):
            raise IndexError("subject index out of range")
        count, idx_ptr = keep.size, keep.ctypes.data
    out = np.zeros(count, dtype=np.int64)
    if count == 0:
        return out
    threads = threads or default_threads()
    rc = _load().sw_oracle_scores(q.ctypes.data, q.size, residues.ctypes.data, offsets.ctypes.data,
                                  idx_ptr, count, sm.ctypes.data, sm.shape[0], int(go), int(ge), MODES[mode],
                                  int(threads),
                                  out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle failed (allocation or thread creation)")
    return out


def topk(scores_vec, k: int):
    """Top ``k`` of a score vector: (scores, indices) ordered by score descending,
    then index ascending; positions beyond the vector length hold (-1, -1)."""
    s = np.asarray(scores_vec, dtype=np.int64)
    order = np.lexsort((np.arange(s.size), -s))[:k]
    top_s = np.full(k, -1, dtype=np.int64)
    top_i = np.full(k, -1, dtype=np.int64)
    top_s[:order.size] = s[order]
    top_i[:order.size] = order
    return top_s, top_i


def pair_neginf(q, d, sm, go: int, ge: int) -> int:
    """The same score with E and F borders at minus infinity and the matrix swept
    column by column (outer loop over the subject).  Pure Python: tiny inputs only."""
    NEG = float("-inf")
    m, n = len(q), len(d)
    if m == 0 or n == 0:
        return 0
    Hc = [0] * (m + 1)          # H[.][j-1]
    Ec = [NEG] * (m + 1)        # E[.][j-1]
    S = 0
    for j in range(1, n + 1):
        Hn = [0] * (m + 1)
        En = [NEG] * (m + 1)
        F = NEG
        for i in range(1, m + 1):
            En[i] = max(Hc[i] - go, Ec[i] - ge)
            F = max(Hn[i - 1] - go, F - ge)
            Hn[i] = max(0, Hc[i - 1] + int(sm[q[i - 1]][d[j - 1]]), En[i], F)
            S = max(S, Hn[i])
        Hc, Ec = Hn, En
    return int(S)


def align(q, d, sm, go: int, ge: int) -> dict:
    """Optimal local alignment of one pair (see ``sw_oracle_align`` for the
    canonical choice among equal-scoring alignments).  Returns score, q_begin,
    q_end, s_begin, s_end (0-based, end exclusive) and ``ops``: 'M' for an
    aligned residue pair, 'I' for a query residue against a gap, 'D' for a
    subject residue against a gap."""
    q, d, sm = _i8(q), _i8(d), _matrix(sm)
    out = np.zeros(5, dtype=np.int64)
    cap = int(q.size + d.size + 1)
    buf = ctypes.create_string_buffer(cap)
    n = _load().sw_oracle_align(q.ctypes.data, q.size, d.ctypes.data, d.size, sm.ctypes.data, sm.shape[0],
                                int(go), int(ge),
                                out.ctypes.data, buf, cap)
    if n < 0:
        raise MemoryError("oracle allocation failed")
    return {"score": int(out[0]), "q_begin": int(out[1]), "q_end": int(out[2]), "s_begin": int(out[3]),
            "s_end": int(out[4]), "ops": buf.raw[:n].decode()}
