"""GPU: chunked multi-query launches, the continuous-batching server and the
length-paired FIFO give exactly the oracle's scores and top-k, and each
request's result is the same alone and in the mix (tolerance 0)."""
import numpy as np
import pytest

import oracle
from inputs import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lane_pack", [1, 2])
@pytest.mark.parametrize("nchunks", [1, 3, 7])
def test_search_multi_covers_all_chunks(gpu, blosum, nchunks, lane_pack):
    import torch
    db = synth.small_db(seed=5 + nchunks, n=2500, lo=1, hi=700, median=250)
    D = gpu.Database(db.residues, db.offsets, lane_pack=lane_pack)
    qs = [synth.small_query(seed=s, m=m) for s, m in [(1, 33), (2, 260), (3, 1), (4, 900)]]
    outs = [torch.full((db.n,), -7, dtype=torch.int32, device="cuda") for _ in qs]
    qo = np.concatenate([[0], np.cumsum([q.size for q in qs])])
    for step in range(nchunks):
        # each query starts at a different chunk
        chunks = [(i + step) % nchunks for i in range(len(qs))]
        gpu.sw_search_multi(np.concatenate(qs), qo, chunks, nchunks, D.handle, blosum, 10, 2, outs)
        torch.cuda.synchronize()
        if step == 0 and nchunks > 1:
            assert (outs[0].cpu().numpy() == -7).any()      # other chunks not written yet
    for q, o in zip(qs, outs):
        want = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
        assert (o.cpu().numpy() == want).all()
    D.close()


@pytest.mark.parametrize("lane_pack", [1, 2])
def test_server_results_alone_and_in_mix(gpu, blosum, lane_pack):
    """lane_pack 2: requests that share an iteration score the same chunk and
    share lanes two queries at a time."""
    from paper_2309_09609_amd.serve import GpuEngine, Server
    db = synth.small_db(seed=77, n=3000, lo=20, hi=1500, median=300)
    D = gpu.Database(db.residues, db.offsets, lane_pack=lane_pack)
    rng = np.random.default_rng(1)
    qs = [synth.small_query(seed=100 + i, m=int(m)) for i, m in enumerate(rng.integers(30, 700, 12))]
    arrivals = np.sort(rng.uniform(0, 0.002, len(qs)))   # close together: they share iterations
    eng = GpuEngine(D, blosum, 10, 2, k=10)
    mix = Server(eng, nchunks=4).run(qs, arrivals)
    assert mix.max_active > 1
    for i, q in enumerate(qs):
        alone = Server(GpuEngine(D, blosum, 10, 2, k=10), nchunks=4).run([q], [0.0])
        a_s, a_i = alone.results[0]
        m_s, m_i = mix.results[i]
        assert (a_s == m_s).all() and (a_i == m_i).all(), i
        ws, wi = oracle.topk(oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), 10)
        assert (m_s == ws).all() and (m_i == wi).all(), i
    D.close()


def test_server_under_tiny_memory_budget(gpu, blosum):
    from paper_2309_09609_amd.serve import GpuEngine, Server
    db = synth.small_db(seed=78, n=1000, lo=20, hi=800, median=300)
    D = gpu.Database(db.residues, db.offsets)
    qs = [synth.small_query(seed=200 + i, m=50 + 40 * i) for i in range(6)]
    eng = GpuEngine(D, blosum, 10, 2, k=5)
    srv = Server(eng, nchunks=3, mem_budget=2 * eng.slot_bytes)
    rep = srv.run(qs, np.zeros(len(qs)))
    assert srv.max_slots == 2 and rep.max_active == 2 and srv.allocated == 2
    for i, q in enumerate(qs):
        ws, wi = oracle.topk(oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), 5)
        assert (rep.results[i][0] == ws).all() and (rep.results[i][1] == wi).all()
    D.close()


def test_dynamic_batching_matches_the_oracle(gpu, blosum):
    from paper_2309_09609_amd.serve import batch_run
    db = synth.small_db(seed=79, n=2000, lo=20, hi=900, median=300)
    D = gpu.Database(db.residues, db.offsets, lane_pack=2)
    rng = np.random.default_rng(2)
    qs = [synth.small_query(seed=300 + i, m=int(m)) for i, m in enumerate(rng.integers(1, 600, 11))]
    arrivals = np.sort(rng.uniform(0, 0.02, len(qs)))
    rep = batch_run(D, qs, arrivals, blosum, 10, 2, k=10, max_batch=4)
    assert rep.iterations >= 3 and rep.max_active <= 4
    for i, q in enumerate(qs):
        ws, wi = oracle.topk(oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), 10)
        s, idx = rep.results[i]
        assert (s == ws).all() and (idx == wi).all(), i
    D.close()


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_paired_fifo_matches_the_oracle(gpu, blosum, depth):
    """Pairs of similar length share lanes (query pairs), singles run alone, up to `depth` units queued
    on the stream at once through one caller workspace: every top 10 equals the oracle's."""
    from paper_2309_09609_amd.serve import paired_run
    db = synth.small_db(seed=80 + depth, n=2000, lo=20, hi=900, median=300)
    D = gpu.Database(db.residues, db.offsets, memory="torch", lane_pack=2, force_lanes=2)
    rng = np.random.default_rng(3 + depth)
    lens = [int(m) for m in rng.integers(1, 700, 14)] + [300, 290, 0, 1, 1]
    qs = [synth.small_query(seed=400 + 20 * depth + i, m=m) for i, m in enumerate(lens)]
    arrivals = np.zeros(len(qs))            # all waiting at once: the pairs formed do not depend on timing
    print(f"paired FIFO depth {depth}: {len(qs)} requests, lengths {lens}", flush=True)
    rep = paired_run(D, qs, arrivals, blosum, 10, 2, k=10, ratio=0.75, depth=depth)
    assert rep.paired >= 2 and rep.iterations == len(qs) - rep.paired
    for i, q in enumerate(qs):
        ws, wi = oracle.topk(oracle.scores(q, db.residues, db.offsets, blosum, 10, 2), 10)
        s, idx = rep.results[i]
        assert (s == ws).all() and (idx == wi).all(), (i, lens[i])
    assert D.info()["device_bytes"] == 0
    D.close()
