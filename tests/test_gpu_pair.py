"""GPU: one long pair scored across the whole GPU (tiles of one anti-diagonal
per launch) equals the oracle's score (Eq. 1-3, tolerance 0), from single
residues and ragged tile edges to a 50,000 x 50,000 pair."""
import numpy as np
import pytest

import oracle
from inputs import synth
from refs import identity_matrix

pytestmark = pytest.mark.gpu


def _pair(gpu, q, d, sm, go, ge, alphabet=0):
    import torch
    s = gpu.sw_pair(q, d, sm, go, ge, alphabet=alphabet)
    torch.cuda.synchronize()
    return int(s.item())


@pytest.mark.parametrize("m,n", [(1, 1), (1, 700), (700, 1), (63, 64), (255, 257), (256, 256), (257, 4095),
                                 (1000, 3000), (3001, 999), (5000, 4097)])
def test_pair_ragged_sizes(gpu, blosum, m, n):
    rng = np.random.default_rng(m * 7919 + n)
    q = synth.background_residues(rng, m)
    d = synth.background_residues(rng, n)
    if m > 40 and n > 40:                          # a shared stretch makes a strong local hit
        L = min(m, n) // 3
        d[n // 3: n // 3 + L] = q[m // 4: m // 4 + L]
    assert _pair(gpu, q, d, blosum, 10, 2) == oracle.pair(q, d, blosum, 10, 2), (m, n)


@pytest.mark.parametrize("seed", range(6))
def test_pair_random_matrices_and_gaps(gpu, seed):
    rng = np.random.default_rng(100 + seed)
    A = int(rng.choice([4, 20, 24]))
    sm = rng.integers(-128, 128, (A, A)).astype(np.int8) if seed % 2 else rng.integers(-6, 12, (A, A)).astype(np.int8)
    go, ge = int(rng.integers(0, 60)), int(rng.integers(0, 20))
    m, n = int(rng.integers(1, 2000)), int(rng.integers(1, 2000))
    q = rng.integers(0, A, m).astype(np.int8)
    d = rng.integers(0, A, n).astype(np.int8)
    assert _pair(gpu, q, d, sm, go, ge, alphabet=A) == oracle.pair(q, d, sm, go, ge), (seed, A, go, ge, m, n)


def test_pair_high_scores_and_empty(gpu, blosum):
    q = np.full(3000, 17, np.int8)                 # W x 3000 against itself: 33,000 (above 16 bits)
    assert _pair(gpu, q, q, blosum, 10, 2) == 33000
    assert _pair(gpu, q, np.zeros(0, np.int8), blosum, 10, 2) == 0
    assert _pair(gpu, np.zeros(0, np.int8), q, blosum, 10, 2) == 0
    sm = identity_matrix(1, -128)
    a = np.array([0] * 40 + [2] * 3 + [1] * 40, np.int8)          # a gap of 3 between two runs of 40
    b = np.array([0] * 40 + [1] * 40, np.int8)
    assert _pair(gpu, a, b, sm, 10, 2) == max(40, 40, 80 - 10 - 2 * 2)


def test_pair_rejects_bad_input(gpu, blosum):
    with pytest.raises(gpu.SwError) as e:
        gpu.sw_pair(np.array([0, 20], np.int8), np.array([1, 2], np.int8), blosum, 10, 2)
    assert e.value.status == -2
    with pytest.raises(gpu.SwError):
        gpu.sw_pair(np.array([0, 1], np.int8), np.array([1, 2], np.int8), blosum, -1, 2)


def test_pair_50k_by_50k(gpu, blosum):
    """Two 50,000-residue sequences with a mutated shared stretch: 196 x 196 tiles."""
    rng = np.random.default_rng(50)
    q = synth.background_residues(rng, 50_000)
    d = synth.background_residues(rng, 50_000)
    hom = synth.mutate(rng, q[20_000:40_000], 0.3, 0.02)[:20_000]
    d[10_000:10_000 + hom.size] = hom
    got = _pair(gpu, q, d, blosum, 10, 2)
    want = oracle.pair(q, d, blosum, 10, 2)
    assert got == want and want > 10_000, (got, want)
