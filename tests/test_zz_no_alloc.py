"""GPU: the allocation-free top-k (fixed device array) equals sw_topk_ws with a
caller workspace, call after call, and the oracle's top k."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _case(gpu, n, k, seed):
    import torch
    rng = np.random.default_rng(seed)
    s = rng.integers(-40, 900, size=max(n, 1)).astype(np.int32)[:n]       # many ties
    d = torch.from_numpy(s).cuda() if n else torch.zeros(1, dtype=torch.int32, device="cuda")
    a_s = torch.empty(k, dtype=torch.int32, device="cuda")
    a_i = torch.empty(k, dtype=torch.int64, device="cuda")
    gpu.sw_topk_noalloc(d, n, k, a_s, a_i)
    need = gpu.sw_topk_ws_bytes(n, k)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    b_s = torch.empty(k, dtype=torch.int32, device="cuda")
    b_i = torch.empty(k, dtype=torch.int64, device="cuda")
    gpu.sw_topk_ws(d, n, k, b_s, b_i, ws if need else None, need)
    torch.cuda.synchronize()
    assert torch.equal(a_s, b_s) and torch.equal(a_i, b_i), (n, k)
    ws_, wi_ = oracle.topk(s, k)
    assert (a_s.cpu().numpy() == ws_).all() and (a_i.cpu().numpy() == wi_).all(), (n, k)
    return need


def test_noalloc_topk_two_calls_second_smaller(gpu):
    assert _case(gpu, 570_000, 1000, 1) > 0            # two launches through the fixed array
    assert _case(gpu, 40_000, 10, 2) > 0               # a smaller one after it: no stale candidates
    assert _case(gpu, 3_000, 5, 3) == 0                # one launch, no array
    assert _case(gpu, 0, 4, 4) == 0


def test_noalloc_topk_rejects_bad_arguments(gpu):
    import torch
    d = torch.zeros(10, dtype=torch.int32, device="cuda")
    o_s = torch.empty(2000, dtype=torch.int32, device="cuda")
    o_i = torch.empty(2000, dtype=torch.int64, device="cuda")
    with pytest.raises(gpu.SwError) as e:
        gpu.sw_topk_noalloc(d, 10, 2000, o_s, o_i)
    assert e.value.status == -5
    with pytest.raises(gpu.SwError):
        gpu.sw_topk_noalloc(d, -1, 5, o_s, o_i)
