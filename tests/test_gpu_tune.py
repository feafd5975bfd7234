"""GPU: the autotuner applies a parity-passing winner, and the scores it then
produces equal the oracle's (the knobs change speed only, Eq. 1-3 exactly)."""
import json

import numpy as np
import pytest

import oracle
from inputs import synth
from paper_2309_09609_amd import tune as tuner

pytestmark = pytest.mark.gpu


def test_tune_applies_an_oracle_checked_winner(gpu, blosum, tmp_path):
    import torch
    db = synth.small_db(seed=401, n=3000, lo=0, hi=1200, median=300)
    queries = [synth.small_query(seed=410 + i, m=m) for i, m in enumerate([60, 300, 310, 900, 45, 1200])]
    D = gpu.Database(db.residues, db.offsets)
    sample = tuner._sample(queries, 8)
    want = [oracle.scores(q, db.residues, db.offsets, blosum, 10, 2) for q in sample]
    verify = lambda i, row: np.array_equal(np.asarray(row, np.int64), want[i])  # noqa: E731
    path = str(tmp_path / "tune.json")
    tuner._memory_cache.clear()
    out = tuner.tune(D, queries, blosum, 10, 2, repeats=1, cache_path=path, verify=verify)
    assert all(t["parity"] for t in out["trials"]), out["trials"]
    assert out["key"] in json.load(open(path))
    scores, ts, ti = D.search_batch(queries, blosum, 10, 2, k=10)
    torch.cuda.synchronize()
    S = scores.cpu().numpy()
    for i, q in enumerate(queries):
        w = oracle.scores(q, db.residues, db.offsets, blosum, 10, 2)
        assert np.array_equal(S[i].astype(np.int64), w), i
        ws, wi = oracle.topk(w, 10)
        assert (ts[i].cpu().numpy() == ws).all() and (ti[i].cpu().numpy() == wi).all()
    # a second handle takes the cached knobs without trying candidates
    D2 = gpu.Database(db.residues, db.offsets)
    again = tuner.tune(D2, queries, blosum, 10, 2, cache_path=path)
    assert again["cached"] and again["knobs"] == out["knobs"]
    D.close()
    D2.close()
