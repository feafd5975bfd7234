"""Top-k of long score vectors (two-launch form) and of signed scores against
numpy's lexsort (score descending, index ascending), tolerance 0."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,k,spread", [(200_000, 10, 50), (1_000_003, 1, 7), (3_000_000, 1024, 300),
                                        (10_000_000, 10, 2000), (150_000, 1024, 3), (131_071, 5, 100),
                                        (16_383, 5, 100), (16_384, 7, 30), (570_000, 10, 40)])
def test_long_vectors(gpu, n, k, spread):
    import torch
    rng = np.random.default_rng(n + k)
    s = rng.integers(0, spread, n).astype(np.int32)          # many ties
    d = torch.from_numpy(s).cuda()
    ts, ti = gpu.topk(d, k)
    torch.cuda.synchronize()
    ws, wi = oracle.topk(s, k)
    assert (ts.cpu().numpy() == ws).all() and (ti.cpu().numpy() == wi).all()


def test_signed_scores(gpu):
    import torch
    rng = np.random.default_rng(9)
    for n in (1000, 500_000):
        s = rng.integers(-5000, 50, n).astype(np.int32)
        d = torch.from_numpy(s).cuda()
        for k in (1, 17, 1024):
            ts, ti = gpu.topk(d, k)
            torch.cuda.synchronize()
            ws, wi = oracle.topk(s, k)
            assert (ts.cpu().numpy() == ws).all() and (ti.cpu().numpy() == wi).all(), (n, k)


def test_workspace_errors(gpu):
    import ctypes
    import torch
    lib = gpu.load()
    need = ctypes.c_int64()
    assert lib.sw_topk_ws_bytes(10_000_000, 10, ctypes.byref(need)) == 0 and need.value > 0
    assert lib.sw_topk_ws_bytes(1000, 10, ctypes.byref(need)) == 0 and need.value == 0
    d = torch.zeros(10_000_000, dtype=torch.int32, device="cuda")
    ts = torch.empty(10, dtype=torch.int32, device="cuda")
    ti = torch.empty(10, dtype=torch.int64, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert lib.sw_topk_ws(ctypes.c_void_p(d.data_ptr()), d.numel(), 10, ctypes.c_void_p(ts.data_ptr()),
                          ctypes.c_void_p(ti.data_ptr()), ctypes.c_void_p(small.data_ptr()), 16, None) == -6
