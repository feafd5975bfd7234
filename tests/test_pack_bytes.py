"""Sizing of the caller-owned packed image, on the host (no GPU needed)."""
import ctypes

import numpy as np

import paper_2309_09609_amd as sw


def _bytes(offs):
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    out = ctypes.c_int64()
    st = sw.load().sw_db_pack_bytes(offs.ctypes.data, offs.size - 1, None, ctypes.byref(out))
    return st, out.value


def test_pack_bytes_covers_the_interleaved_image():
    rng = np.random.default_rng(1)
    lens = rng.integers(0, 900, 1000)
    offs = np.concatenate([[0], np.cumsum(lens)])
    st, b = _bytes(offs)
    assert st == 0
    # every group of 128 length-sorted subjects is as wide as its longest, rounded up to 4 columns
    srt = np.sort(lens)[::-1]
    image = sum(int(-(-srt[g] // 4) * 4) * 128 for g in range(0, lens.size, 128))
    assert image <= b <= image + 40 * 1024 + 64 * lens.size


def test_pack_bytes_errors():
    assert _bytes(np.array([0, 5, 3]))[0] == -1                 # decreasing offsets
    assert _bytes(np.array([-1, 5]))[0] == -1
    assert _bytes(np.array([0], np.int64))[0] == 0              # empty database
