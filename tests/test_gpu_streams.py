"""GPU: two handles searched on two non-default streams, every call queued without a wait in between
and the two streams interleaved (plain searches, top-k and the batched form, whose second call replays
its captured graph).  The library forks its side launches from the caller's stream and joins them back,
so every result equals the oracle's."""
import numpy as np
import pytest

import oracle
from inputs import synth

pytestmark = pytest.mark.gpu


def test_two_handles_on_two_streams(gpu, blosum):
    import torch
    dbs = [synth.small_db(seed=540 + i, n=1500, lo=0, hi=1200, median=300) for i in range(2)]
    # one handle on library memory, one on torch memory (caller workspaces)
    Ds = [gpu.Database(dbs[0].residues, dbs[0].offsets),
          gpu.Database(dbs[1].residues, dbs[1].offsets, memory="torch")]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    queries = [synth.small_query(seed=550 + i, m=m) for i, m in enumerate([144, 600, 37, 1000, 1])]
    want = [[oracle.scores(q, d.residues, d.offsets, blosum, 10, 2) for q in queries] for d in dbs]
    got = []
    for rep in range(2):
        for qi, q in enumerate(queries):
            for h in range(2):
                out = Ds[h].search(q, blosum, 10, 2, stream=streams[h])
                ts, ti = gpu.topk(out, 5, stream=streams[h])
                got.append((h, [qi], [out], ts[None], ti[None]))
        for h in range(2):
            scores, ts, ti = Ds[h].search_batch(queries, blosum, 10, 2, k=5, stream=streams[h])
            got.append((h, list(range(len(queries))), list(scores), ts, ti))
    torch.cuda.synchronize()
    for h, qis, rows, ts, ti in got:
        for r, qi in enumerate(qis):
            w = want[h][qi]
            row = rows[r].cpu().numpy()
            bad = np.nonzero(row != w)[0]
            assert bad.size == 0, f"handle {h} query {qi}: {bad.size} mismatches"
            ws_, wi_ = oracle.topk(w, 5)
            assert (ts[r].cpu().numpy() == ws_).all() and (ti[r].cpu().numpy() == wi_).all(), (h, qi)
    for D in Ds:
        D.close()
