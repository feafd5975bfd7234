"""Independent references that pin the oracle: brute-force enumeration of local
alignments and textbook special cases.  None of them evaluates Eq. 1-3."""
from __future__ import annotations

import numpy as np


def bf_score(q, d, sm, go: int, ge: int) -> int:
    """Best local alignment score by enumerating every alignment path.

    An alignment is a lattice path from any grid point made of diagonal steps
    (pair q[i] with d[j], score SM) and gap steps; a maximal run of k gap steps
    in one direction costs Go + (k-1) * min(Go, Ge).  For Ge <= Go (the paper's
    10/2 setting) that is the literal affine cost Go + (k-1) * Ge read off
    Eq. 2-3; for Ge > Go reopening a gap is cheaper than extending it and the
    recurrence charges min(Go, Ge) per extra gap step.  The empty alignment
    scores 0.  Cost grows like the Delannoy numbers: keep m, n <= 7.
    """
    q = [int(x) for x in q]
    d = [int(x) for x in d]
    m, n = len(q), len(d)
    ext = min(go, ge)
    best = 0
    for i0 in range(m + 1):
        for j0 in range(n + 1):
            stack = [(i0, j0, 0, 0)]          # (i, j, score, last step: 0 pair/start, 1 horiz, 2 vert)
            while stack:
                i, j, s, st = stack.pop()
                if s > best:
                    best = s
                if i < m and j < n:
                    stack.append((i + 1, j + 1, s + int(sm[q[i]][d[j]]), 0))
                if j < n:
                    stack.append((i, j + 1, s - (ext if st == 1 else go), 1))
                if i < m:
                    stack.append((i + 1, j, s - (ext if st == 2 else go), 2))
    return best


def kadane_diagonals(q, d, sm) -> int:
    """Best ungapped local alignment: max over all diagonals of the maximum
    subarray sum (Kadane) of the substitution scores along that diagonal."""
    m, n = len(q), len(d)
    best = 0
    for off in range(-(m - 1), n):
        run = 0
        i = max(0, -off)
        j = i + off
        while i < m and j < n:
            run = max(0, run + int(sm[q[i]][d[j]]))
            best = max(best, run)
            i += 1
            j += 1
    return best


def lcs_len(a, b) -> int:
    """Longest common subsequence length (textbook table)."""
    a, b = list(a), list(b)
    prev = [0] * (len(b) + 1)
    for x in a:
        cur = [0]
        for j, y in enumerate(b):
            cur.append(prev[j] + 1 if x == y else max(prev[j + 1], cur[j]))
        prev = cur
    return prev[-1]


def lcsubstr_len(a, b) -> int:
    """Longest common substring length (textbook run-length table)."""
    a, b = list(a), list(b)
    best = 0
    prev = [0] * (len(b) + 1)
    for x in a:
        cur = [0]
        for j, y in enumerate(b):
            v = prev[j] + 1 if x == y else 0
            cur.append(v)
            best = max(best, v)
        prev = cur
    return best


def identity_matrix(match: int = 1, mismatch: int = -128) -> np.ndarray:
    sm = np.full((20, 20), mismatch, dtype=np.int8)
    np.fill_diagonal(sm, match)
    return sm


def score_ops(q, d, sm, go: int, ge: int, q_begin: int, s_begin: int, ops: str):
    """Score of an alignment given as operations from (q_begin, s_begin):
    'M' pairs q[i] with d[j]; 'I' puts q[i] against a gap, 'D' puts d[j]
    against a gap.  A maximal run of k gap operations of one kind costs
    Go + (k-1) * min(Go, Ge), as in ``bf_score``.  Returns (score, q_end, s_end)."""
    i, j, s, last = q_begin, s_begin, 0, ""
    ext = min(go, ge)
    for op in ops:
        if op == "M":
            s += int(sm[int(q[i])][int(d[j])])
            i += 1
            j += 1
        elif op == "I":
            s -= ext if last == "I" else go
            i += 1
        elif op == "D":
            s -= ext if last == "D" else go
            j += 1
        else:
            raise ValueError(op)
        last = op
    return s, i, j


def bf_end_to_end(q, d, sm, go: int, ge: int, semi: bool) -> int:
    """Best global (every residue of both sequences aligned or gapped) or
    semi-global (every query residue; the subject's leading and trailing
    residues free) alignment score by enumerating every path.  A maximal run of
    k gap steps in one direction costs Go + (k-1) * min(Go, Ge), also at the
    ends.  Keep m, n <= 5."""
    q = [int(x) for x in q]
    d = [int(x) for x in d]
    m, n = len(q), len(d)
    ext = min(go, ge)
    best = None
    starts = range(n + 1) if semi else [0]
    for j0 in starts:
        stack = [(0, j0, 0, 0)]
        while stack:
            i, j, s, st = stack.pop()
            if i == m and (semi or j == n):
                best = s if best is None else max(best, s)
            if i < m and j < n:
                stack.append((i + 1, j + 1, s + int(sm[q[i]][d[j]]), 0))
            if j < n:
                stack.append((i, j + 1, s - (ext if st == 1 else go), 1))
            if i < m:
                stack.append((i + 1, j, s - (ext if st == 2 else go), 2))
    return best


def edit_distance(a, b) -> int:
    """Levenshtein distance (unit costs), textbook table."""
    a, b = list(a), list(b)
    prev = list(range(len(b) + 1))
    for i, x in enumerate(a, 1):
        cur = [i]
        for j, y in enumerate(b, 1):
            cur.append(min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (x != y)))
        prev = cur
    return prev[-1]


def best_substring_distance(a, b) -> int:
    """Smallest edit distance between a and any substring of b (Sellers' table:
    row 0 is all zeros, the answer is the minimum of the last row)."""
    a, b = list(a), list(b)
    prev = [0] * (len(b) + 1)
    for i, x in enumerate(a, 1):
        cur = [i]
        for j, y in enumerate(b, 1):
            cur.append(min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (x != y)))
        prev = cur
    return min(prev)
