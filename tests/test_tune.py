"""The autotuner's parity gate and cache, on the CPU with a stand-in database
whose searches come from the oracle (one candidate knob set is made wrong)."""
import json
import time

import numpy as np
import pytest

import oracle
from inputs import blosum62, synth
from paper_2309_09609_amd import tune as tuner

CANDS = [dict(rows_per_lane=16, lane_pack=1), dict(rows_per_lane=8, lane_pack=1), dict(rows_per_lane=16, lane_pack=2)]


class StandIn:
    """Database stand-in: exact scores from the oracle, except for ``bad`` knobs,
    whose scores are off by one on the subjects in ``wrong``; ``bad`` is also
    the fastest candidate, so only the gate keeps it from winning."""

    def __init__(self, db, bad, wrong):
        self.res, self.offsets, self.n = db.residues, db.offsets, db.n
        self.bad, self.wrong = bad, np.asarray(wrong, np.int64)
        self.knobs = {}
        self.applied = []

    def tune(self, **knobs):
        self.knobs = knobs
        self.applied.append(knobs)

    def search_batch(self, qs, subst, go, ge, k=0):
        S = np.stack([oracle.scores(q, self.res, self.offsets, subst, go, ge) for q in qs])
        if self.knobs == self.bad:
            S[:, self.wrong] += 1
        else:
            time.sleep(0.05)      # well above the noise of the oracle call itself
        return S, None, None

    def align_batch(self, qs, subjects, subst, go, ge):
        return [[{"score": oracle.pair(q, self.res[self.offsets[s]:self.offsets[s + 1]], subst, go, ge)} for s in sl]
                for q, sl in zip(qs, subjects)]


@pytest.fixture(scope="module")
def small():
    db = synth.small_db(seed=301, n=400, lo=0, hi=300)
    qs = [synth.small_query(seed=310 + i, m=m) for i, m in enumerate([40, 90, 150, 60])]
    return db, qs


def test_wrong_candidate_on_sampled_subjects_is_excluded(small, tmp_path):
    db, qs = small
    sm = blosum62()
    idx = tuner.sample_subjects(db.offsets, 48)
    fake = StandIn(db, CANDS[1], wrong=idx[:3])
    out = tuner.tune(fake, qs, sm, 10, 2, candidates=CANDS, repeats=1, cache_path=str(tmp_path / "t.json"))
    assert out["knobs"] != CANDS[1]
    bad = [t for t in out["trials"] if t["knobs"] == CANDS[1]][0]
    assert not bad["parity"] and bad["gcups"] == max(t["gcups"] for t in out["trials"])
    assert fake.knobs == out["knobs"]
    assert out["gate"]["subjects"] == idx.size


def test_verify_callback_catches_what_the_sample_misses(small):
    db, qs = small
    sm = blosum62()
    idx = set(tuner.sample_subjects(db.offsets, 48).tolist())
    outside = [k for k in range(db.n) if k not in idx][:2]
    fake = StandIn(db, CANDS[0], wrong=outside)
    want = [oracle.scores(q, db.residues, db.offsets, sm, 10, 2) for q in tuner._sample(qs, 8)]
    verify = lambda i, row: np.array_equal(np.asarray(row, np.int64), want[i])  # noqa: E731
    out = tuner.tune(fake, qs, sm, 10, 2, candidates=CANDS, repeats=1, use_cache=False, verify=verify)
    assert out["knobs"] != CANDS[0]
    assert [t["parity"] for t in out["trials"]] == [False, True, True]
    # without the callback the sampled gate alone lets it through (it is also the fastest)
    out2 = tuner.tune(StandIn(db, CANDS[0], wrong=outside), qs, sm, 10, 2, candidates=CANDS, repeats=1,
                      use_cache=False)
    assert out2["knobs"] == CANDS[0]


def test_no_passing_candidate_is_an_error(small):
    db, qs = small
    idx = tuner.sample_subjects(db.offsets, 48)

    class AllBad(StandIn):
        def search_batch(self, qs, subst, go, ge, k=0):
            S, _, _ = super().search_batch(qs, subst, go, ge, k)
            S[:, idx[0]] -= 1
            return S, None, None

    with pytest.raises(RuntimeError):
        tuner.tune(AllBad(db, None, []), qs, blosum62(), 10, 2, candidates=CANDS, repeats=1, use_cache=False)


def test_cache_is_keyed_by_scoring_setup(small, tmp_path):
    db, qs = small
    sm = blosum62()
    path = str(tmp_path / "sub" / "tune.json")
    tuner._memory_cache.clear()
    fake = StandIn(db, None, [])
    first = tuner.tune(fake, qs, sm, 10, 2, candidates=CANDS, repeats=1, cache_path=path)
    assert not first["cached"]
    doc = json.load(open(path))
    assert first["key"] in doc and "sm" in first["key"] and "g10/2" in first["key"]
    fake.applied.clear()
    again = tuner.tune(fake, qs, sm, 10, 2, candidates=CANDS, repeats=1, cache_path=path)
    assert again["cached"] and again["knobs"] == first["knobs"] and fake.applied == [first["knobs"]]
    other_gaps = tuner.tune(fake, qs, sm, 11, 1, candidates=CANDS, repeats=1, cache_path=path)
    assert not other_gaps["cached"]
    sm2 = sm.copy()
    sm2[0, 0] += 1
    assert tuner.shape_key("x", db.n, [q.size for q in qs], sm, 10, 2) != \
        tuner.shape_key("x", db.n, [q.size for q in qs], sm2, 10, 2)
