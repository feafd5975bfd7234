"""GPU: searches on caller-owned device memory only (the problem of Sec. II-B:
one query or many against a database, a score per subject).  torch allocates
the packed image (sw_db_pack_into) and every workspace (sw_search_ws,
sw_search_batch_ws); every score equals the oracle's and the handle holds no
device memory of its own."""
import numpy as np
import pytest

import oracle
from inputs import synth

pytestmark = pytest.mark.gpu


def _eq(got, want, ctx):
    got = np.asarray(got, np.int64)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} mismatches at {bad[:5]}"


@pytest.mark.parametrize("lane_pack", [1, 2])
def test_plain_and_batched_on_torch_memory(gpu, blosum, lane_pack):
    import torch
    db = synth.small_db(seed=501, n=2500, lo=0, hi=1500, median=300)
    D = gpu.Database(db.residues, db.offsets, memory="torch", lane_pack=lane_pack)
    assert D.info()["device_bytes"] == 0
    queries = [synth.small_query(seed=510 + i, m=m) for i, m in enumerate([144, 1, 700, 0, 333, 90])]
    want = [oracle.scores(q, db.residues, db.offsets, blosum, 10, 2) for q in queries]
    for i, q in enumerate(queries):
        got = D.search(q, blosum, 10, 2)
        torch.cuda.synchronize()
        _eq(got.cpu().numpy(), want[i], f"plain query {i}")
    for keep in (True, False):
        for rep in range(2):                          # the second call replays the captured graph
            scores, ts, ti = D.search_batch(queries, blosum, 10, 2, k=10, keep_scores=keep)
            torch.cuda.synchronize()
            for i in range(len(queries)):
                if keep:
                    _eq(scores[i].cpu().numpy(), want[i], f"batch query {i}")
                ws_, wi_ = oracle.topk(want[i], 10)
                assert (ts[i].cpu().numpy() == ws_).all() and (ti[i].cpu().numpy() == wi_).all(), (keep, rep, i)
    st = D.stats()
    assert st["recomputed"] == st["rerun_pairs"]
    assert D.info()["device_bytes"] == 0
    D.close()


def test_saturated_pairs_on_torch_memory(gpu, blosum):
    """The 32-bit recompute (list and flag bits) in a caller's workspace."""
    import torch
    rng = np.random.default_rng(7)
    subs = [np.full(3000, 17, np.int8), np.full(2990, 17, np.int8)]
    subs += [rng.integers(0, 20, int(rng.integers(1, 400))).astype(np.int8) for _ in range(300)]
    offs = np.zeros(len(subs) + 1, np.int64)
    offs[1:] = np.cumsum([s.size for s in subs])
    res = np.concatenate(subs)
    D = gpu.Database(res, offs, memory="torch", rerun_cap=1, poison=1)
    q = np.full(3000, 17, np.int8)
    got = D.search(q, blosum, 10, 2)
    torch.cuda.synchronize()
    _eq(got.cpu().numpy(), oracle.scores(q, res, offs, blosum, 10, 2), "saturated")
    st = D.stats()
    assert st["rerun_pairs"] >= 1 and st["recomputed"] == st["rerun_pairs"]
    assert D.info()["device_bytes"] == 0
    D.close()


def test_workspace_and_image_sizes_are_checked(gpu, blosum):
    import torch
    db = synth.small_db(seed=503, n=400, lo=1, hi=300)
    need = gpu.sw_db_pack_bytes(db.offsets)
    d_res = torch.from_numpy(db.residues).cuda()
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu.SwError) as e:
        gpu.sw_db_pack_into(d_res, db.offsets, small)
    assert e.value.status == -6
    img = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu.SwError) as e:
        gpu.sw_db_pack_into(d_res, db.offsets, img[1:])            # not 256-byte aligned
    assert e.value.status == -1
    h = gpu.sw_db_pack_into(d_res, db.offsets, img)
    q = synth.small_query(seed=503, m=120)
    out = torch.empty(db.n, dtype=torch.int32, device="cuda")
    wsb = gpu.sw_batch_workspace_bytes(h, np.array([0, q.size]))
    with pytest.raises(gpu.SwError) as e:
        gpu.sw_search_ws(q, h, None, db.n, blosum, 10, 2, out, torch.empty(wsb - 256, dtype=torch.uint8, device="cuda"))
    assert e.value.status == -6
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    gpu.sw_search_ws(q, h, db.offsets, db.n, blosum, 10, 2, out, ws)
    torch.cuda.synchronize()
    _eq(out.cpu().numpy(), oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), "explicit ws")
    gpu.load().sw_db_free(h)


def test_batched_calls_queued_back_to_back(gpu, blosum):
    """Seven sw_search_batch_ws calls of different query-length mixes queued on one stream without a wait
    in between (more calls than the library's pinned staging buffers), each on its own workspace; the
    host query array is overwritten as soon as each call returns.  Every score and top 5 equals the oracle's."""
    import torch
    db = synth.small_db(seed=520, n=1800, lo=0, hi=900, median=250)
    D = gpu.Database(db.residues, db.offsets, memory="torch", lane_pack=2)
    mixes = [[144], [300, 280], [1], [700, 650], [90, 0], [512], [200, 210]]
    calls, want = [], []
    stream = torch.cuda.current_stream()
    for c, lens in enumerate(mixes):
        qs = [synth.small_query(seed=530 + 10 * c + i, m=m) for i, m in enumerate(lens)]
        want.append([oracle.scores(q, db.residues, db.offsets, blosum, 10, 2) for q in qs])
        qo = np.zeros(len(qs) + 1, np.int64)
        qo[1:] = np.cumsum([q.size for q in qs])
        flat = np.concatenate(qs) if qo[-1] else np.zeros(0, np.int8)
        ws = torch.empty(gpu.sw_batch_workspace_bytes(D.handle, qo, 5, False), dtype=torch.uint8, device="cuda")
        scores = torch.empty((len(qs), db.n), dtype=torch.int32, device="cuda")
        ts = torch.empty((len(qs), 5), dtype=torch.int32, device="cuda")
        ti = torch.empty((len(qs), 5), dtype=torch.int64, device="cuda")
        gpu.sw_search_batch_ws(flat, qo, D.handle, blosum, 10, 2, 5, scores, ts, ti, ws, stream)
        flat[:] = 0                                   # the call has staged its own copy
        calls.append((scores, ts, ti, ws))
    torch.cuda.synchronize()
    for c, (scores, ts, ti, _) in enumerate(calls):
        for i, w in enumerate(want[c]):
            _eq(scores[i].cpu().numpy(), w, f"call {c} query {i}")
            ws_, wi_ = oracle.topk(w, 5)
            assert (ts[i].cpu().numpy() == ws_).all() and (ti[i].cpu().numpy() == wi_).all(), (c, i)
    assert D.info()["device_bytes"] == 0
    D.close()
