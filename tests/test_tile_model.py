"""CPU model of the tile decomposition of one long pair (the score of `sw_pair`
and the tiled traceback fill): Eq. 1-3 computed tile by tile in launch order
(one anti-diagonal of tiles at a time), each tile seeing only what the device
kernels pass between launches -- the band above's last row (H, and F already
advanced to the band's first row), the previous tile's last column (H, and E
already advanced to the next column) and the saved corner H -- with small
tiles so that a pair spans many bands and column tiles.  Every H of the score
form, and every direction byte and the end cell of the traceback form, must
equal a direct computation over the whole matrix, and the score and end cell
the oracle's.  (Planting a wrong corner, an F not advanced to the band below
or an E not advanced to the next tile in these models makes every case fail.)"""
import numpy as np
import pytest

import oracle
from inputs import blosum62, synth


def _tiles(m, n, th, tw):
    nb, nc = -(-m // th), -(-n // tw)
    for d in range(nb + nc - 1):                       # launch d: the tiles of anti-diagonal d
        for bi in range(max(0, d - nc + 1), min(d, nb - 1) + 1):
            yield bi, d - bi


def pair_by_tiles(q, s, sm, go, ge, th, tw):
    """(score, every H) with E and F floored at 0 (H is unchanged by it), as the pair kernel keeps them."""
    m, n = q.size, s.size
    Hall = np.zeros((m, n), np.int64)
    if m == 0 or n == 0:
        return 0, Hall
    hrow, frow = np.zeros(n, np.int64), np.zeros(n, np.int64)      # band above: H, F advanced
    hcol, ecol = np.zeros(m, np.int64), np.zeros(m, np.int64)      # previous tile: H, E advanced
    corner = {}                                                     # band -> H above-left of the next tile
    best = 0
    for bi, tj in _tiles(m, n, th, tw):
        i0, j0 = bi * th, tj * tw
        rows, cols = range(i0, min(m, i0 + th)), range(j0, min(n, j0 + tw))
        H = {}
        E = {}
        top_h = {j: hrow[j] for j in cols}
        top_f = {j: frow[j] for j in cols}
        diag0 = corner.get(bi, 0) if tj > 0 else 0                 # H[i0 - 1][j0 - 1]
        for j in cols:
            F = top_f[j]
            for i in rows:
                el = ecol[i] if j == j0 else E[(i, j - 1)]        # E already advanced to column j
                if i == i0:
                    hd = (diag0 if j == j0 else top_h[j - 1]) if j > 0 else 0
                else:
                    hd = (hcol[i - 1] if j == j0 else H[(i - 1, j - 1)]) if j > 0 else 0
                if j == 0:
                    hd = 0
                h = max(hd + sm[q[i], s[j]], el, F, 0)
                best = max(best, h)
                H[(i, j)] = h
                Hall[i, j] = h
                E[(i, j)] = max(el - ge, h - go, 0)               # E for column j + 1
                F = max(F - ge, h - go, 0)                         # F for row i + 1
            if i0 + th < m:                                        # the band below's top row
                frow[j] = F
        last_row, last_col = rows[-1], cols[-1]
        corner[bi] = top_h[last_col] if bi > 0 else 0              # saved before the row is overwritten
        for j in cols:
            if i0 + th < m:
                hrow[j] = H[(last_row, j)]
        for i in rows:
            hcol[i] = H[(i, last_col)]
            ecol[i] = E[(i, last_col)]
    return best, Hall


def h_full(q, s, sm, go, ge):
    """Every H of Eq. 1-3 over the whole matrix (zero borders), row by row."""
    m, n = q.size, s.size
    H = np.zeros((m + 1, n + 1), np.int64)
    E = np.zeros((m + 1, n + 1), np.int64)
    F = np.zeros((m + 1, n + 1), np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            E[i, j] = max(H[i, j - 1] - go, E[i, j - 1] - ge)
            F[i, j] = max(H[i - 1, j] - go, F[i - 1, j] - ge)
            H[i, j] = max(H[i - 1, j - 1] + sm[q[i - 1], s[j - 1]], E[i, j], F[i, j], 0)
    return H[1:, 1:]


def direction_bytes_full(q, s, sm, go, ge):
    """Direction byte of every cell and the first end cell (row-major) over the whole matrix, with the
    unfloored E and F of the traceback fill (zero borders)."""
    m, n = q.size, s.size
    H = np.zeros((m + 1, n + 1), np.int64)
    E = np.zeros((m + 1, n + 1), np.int64)
    F = np.zeros((m + 1, n + 1), np.int64)
    byte = np.zeros((m + 1, n + 1), np.int64)
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            eo, ee = H[i, j - 1] - go, E[i, j - 1] - ge
            fo, fe = H[i - 1, j] - go, F[i - 1, j] - ge
            e, f = max(eo, ee), max(fo, fe)
            hd = H[i - 1, j - 1] + sm[q[i - 1], s[j - 1]]
            h = max(hd, e, f, 0)
            src = 0 if h == 0 else 1 if h == hd else 2 if h == e else 3
            byte[i, j] = src | (4 if eo >= ee else 0) | (8 if fo >= fe else 0)
            H[i, j], E[i, j], F[i, j] = h, e, f
    S = int(H.max())
    if S <= 0:
        return byte, (0, 0, 0)
    i, j = np.argwhere(H == S)[0]                                   # row-major first
    return byte, (S, int(i), int(j))


def direction_bytes_by_tiles(q, s, sm, go, ge, th, tw):
    """The same bytes and end cell, tile by tile: each tile gets the band above's last row (H, F), the
    previous tile's last column (H, E), the saved corner, and reports its own first end cell."""
    m, n = q.size, s.size
    byte = np.zeros((m + 1, n + 1), np.int64)
    hrow, frow = np.zeros(n + 1, np.int64), np.zeros(n + 1, np.int64)      # 1-based columns
    hcol, ecol = np.zeros(m + 1, np.int64), np.zeros(m + 1, np.int64)      # 1-based rows
    corner = {}
    ends = []
    for bi, tj in _tiles(m, n, th, tw):
        r0, c0 = bi * th + 1, tj * tw + 1
        rows, cols = range(r0, min(m, r0 + th - 1) + 1), range(c0, min(n, c0 + tw - 1) + 1)
        H, E, F = {}, {}, {}
        top_h = {j: (hrow[j] if bi > 0 else 0) for j in cols}
        top_f = {j: (frow[j] if bi > 0 else 0) for j in cols}
        for i in rows:
            H[(i, c0 - 1)] = hcol[i] if tj > 0 else 0
            E[(i, c0 - 1)] = ecol[i] if tj > 0 else 0
        for j in cols:
            H[(r0 - 1, j)] = top_h[j]
            F[(r0 - 1, j)] = top_f[j]
        H[(r0 - 1, c0 - 1)] = corner.get(bi, 0) if tj > 0 else 0
        best = (0, 0, 0)
        for i in rows:
            for j in cols:
                eo, ee = H[(i, j - 1)] - go, E[(i, j - 1)] - ge
                fo, fe = H[(i - 1, j)] - go, F[(i - 1, j)] - ge
                e, f = max(eo, ee), max(fo, fe)
                hd = H[(i - 1, j - 1)] + sm[q[i - 1], s[j - 1]]
                h = max(hd, e, f, 0)
                src = 0 if h == 0 else 1 if h == hd else 2 if h == e else 3
                byte[i, j] = src | (4 if eo >= ee else 0) | (8 if fo >= fe else 0)
                H[(i, j)], E[(i, j)], F[(i, j)] = h, e, f
                if h > best[0]:
                    best = (h, i, j)
        ends.append(best)
        last_row, last_col = rows[-1], cols[-1]
        corner[bi] = top_h[last_col]
        for j in cols:
            hrow[j], frow[j] = H[(last_row, j)], F[(last_row, j)]
        for i in rows:
            hcol[i], ecol[i] = H[(i, last_col)], E[(i, last_col)]
    S = max(e[0] for e in ends)
    if S <= 0:
        return byte, (0, 0, 0)
    return byte, min((e for e in ends if e[0] == S), key=lambda e: (e[1], e[2]))


def _pair(seed, m, n, plant=True):
    rng = np.random.default_rng(seed)
    q = synth.background_residues(rng, m)
    s = synth.background_residues(rng, n)
    if plant and m > 12 and n > 12:
        k = min(m, n) // 2
        s[3:3 + k] = synth.mutate(rng, q[2:2 + k], 0.2, 0.05)[: k]
    return q, s


@pytest.mark.parametrize("th,tw", [(8, 4), (4, 8), (8, 8), (16, 5)])
@pytest.mark.parametrize("seed,m,n", [(1, 37, 41), (2, 1, 30), (3, 30, 1), (4, 64, 17), (5, 23, 71), (6, 8, 8)])
def test_pair_by_tiles_equals_the_whole_matrix(th, tw, seed, m, n):
    sm = blosum62()
    q, s = _pair(seed, m, n)
    best, H = pair_by_tiles(q, s, sm, 10, 2, th, tw)
    assert (H == h_full(q, s, sm, 10, 2)).all()
    assert best == oracle.pair(q, s, sm, 10, 2)


@pytest.mark.parametrize("go,ge", [(0, 0), (3, 5), (11, 1), (40, 60)])
def test_pair_by_tiles_gap_settings(go, ge):
    sm = blosum62()
    q, s = _pair(7 + go, 45, 38)
    best, H = pair_by_tiles(q, s, sm, go, ge, 8, 4)
    assert (H == h_full(q, s, sm, go, ge)).all()
    assert best == oracle.pair(q, s, sm, go, ge)


@pytest.mark.parametrize("th,tw", [(8, 4), (4, 8), (16, 5)])
@pytest.mark.parametrize("seed,m,n", [(11, 37, 41), (12, 1, 30), (13, 30, 1), (14, 33, 29)])
def test_direction_bytes_by_tiles_equal_the_whole_matrix(th, tw, seed, m, n):
    sm = blosum62()
    q, s = _pair(seed, m, n)
    full, end_full = direction_bytes_full(q, s, sm, 10, 2)
    tiled, end_tiled = direction_bytes_by_tiles(q, s, sm, 10, 2, th, tw)
    assert (full == tiled).all()
    assert end_full == end_tiled
    a = oracle.align(q, s, sm, 10, 2)
    assert (a["score"], a["q_end"], a["s_end"]) == end_full
