"""Seeded synthetic protein databases, queries and arrival traces.

The paper measures on the Env. NR 2021_04 database searched with 20 Swiss-Prot
queries of 144..5,478 residues (Sec. IV-A "Experimental Design").  Neither is
available here, so every workload is synthetic: residues are i.i.d. over the
20 amino acids with background frequencies, lengths are log-normal (or uniform)
with the sizes each workload names, and a few planted homologs and
overflow sentinels give the search something to find.  Nothing in this module
computes an alignment score: it only draws inputs.

Random streams: ``numpy.random.Generator(PCG64(SeedSequence(0,
spawn_key=(workload, stream))))`` with streams 0 = lengths, 1 = residues,
2 = queries, 3 = planted homologs, 4 = arrivals, 5 = sentinels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .blosum import ALPHABET, background_frequencies

LEN_SIGMA = 0.61          # log-normal shape: mean/median = 1.2047 as in a 570k-subject, 206M-residue DB
W_CODE = ALPHABET.index("W")


def rng_for(workload: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(0, spawn_key=(workload, stream))))


_LUT = None


def _residue_lut() -> np.ndarray:
    """2^16-entry table whose entry counts follow the background frequencies."""
    global _LUT
    if _LUT is None:
        f = background_frequencies()
        counts = np.floor(f * 65536).astype(np.int64)
        counts[np.argmax(f)] += 65536 - counts.sum()
        _LUT = np.repeat(np.arange(20, dtype=np.int8), counts)
        assert _LUT.size == 65536
    return _LUT


def background_residues(rng: np.random.Generator, count: int, chunk: int = 1 << 26) -> np.ndarray:
    """int8[count], i.i.d. residue codes with background frequencies."""
    lut = _residue_lut()
    out = np.empty(int(count), dtype=np.int8)
    for s in range(0, int(count), chunk):
        e = min(int(count), s + chunk)
        out[s:e] = lut[rng.integers(0, 65536, size=e - s, dtype=np.uint16)]
    return out


def lognormal_lengths(rng, count, median, lo, hi, sigma=LEN_SIGMA) -> np.ndarray:
    x = np.exp(rng.normal(np.log(median), sigma, size=int(count)))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def mutate(rng: np.random.Generator, seq: np.ndarray, sub_rate: float, indel_rate: float) -> np.ndarray:
    """A homolog of ``seq``: point substitutions and geometric-length indels."""
    lut = _residue_lut()
    s = seq.copy()
    hit = rng.random(s.size) < sub_rate
    s[hit] = lut[rng.integers(0, 65536, size=int(hit.sum()), dtype=np.uint16)]
    if indel_rate <= 0:
        return s
    out = []
    i = 0
    while i < s.size:
        if rng.random() < indel_rate:
            k = int(rng.geometric(0.5))
            if rng.random() < 0.5:   # insertion before position i
                out.append(lut[rng.integers(0, 65536, size=k, dtype=np.uint16)])
            else:                     # deletion of k residues
                i += k
                continue
        out.append(s[i:i + 1])
        i += 1
    return np.concatenate(out) if out else s[:0]


def w_rich_block(rng: np.random.Generator, length: int, w_frac: float = 0.9) -> np.ndarray:
    """A block mostly of tryptophan: its self-alignment scores far above 2^15."""
    b = background_residues(rng, length)
    b[rng.random(length) < w_frac] = W_CODE
    return b


@dataclass
class Database:
    residues: np.ndarray                 # int8, all subjects concatenated
    offsets: np.ndarray                  # int64[n + 1]
    planted: dict = field(default_factory=dict)   # query index -> int64 subject indices
    sentinels: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    name: str = ""

    @property
    def n(self) -> int:
        return self.offsets.size - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def subject(self, k: int) -> np.ndarray:
        return self.residues[self.offsets[k]:self.offsets[k + 1]]


def _assemble(workload, lengths, inserts, name) -> Database:
    """Background residues for every subject, then ``inserts`` (index -> seq) spliced in."""
    lengths = lengths.copy()
    for k, seq in inserts.items():
        lengths[k] = seq.size
    offsets = np.zeros(lengths.size + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    res = background_residues(rng_for(workload, 1), int(offsets[-1]))
    for k, seq in inserts.items():
        res[offsets[k]:offsets[k + 1]] = seq
    return Database(res, offsets, name=name)


def _plant(workload, queries, lengths, per_query, reserved=()) -> tuple[dict, dict]:
    """Choose subjects to replace with mutated copies of each query."""
    rng = rng_for(workload, 3)
    taken = set(int(x) for x in reserved)
    planted, inserts = {}, {}
    for qi, q in enumerate(queries):
        idx = []
        while len(idx) < per_query:
            k = int(rng.integers(0, lengths.size))
            if k in taken:
                continue
            taken.add(k)
            idx.append(k)
            inserts[k] = mutate(rng, q, float(rng.uniform(0.1, 0.7)), float(rng.uniform(0.0, 0.05)))
        planted[qi] = np.array(sorted(idx), dtype=np.int64)
    return planted, inserts


# ---------------------------------------------------------------- workload 1
def workload1():
    """1 query (m = 144) vs 2,000 subjects, log-normal lengths median 300 clipped to 20..1,000."""
    q = background_residues(rng_for(1, 2), 144)
    lengths = lognormal_lengths(rng_for(1, 0), 2000, 300, 20, 1000)
    planted, inserts = _plant(1, [q], lengths, per_query=5)
    db = _assemble(1, lengths, inserts, "2k")
    db.planted = planted
    return [q], db


# ---------------------------------------------------------- workloads 2 and 3
WL2_QLENS = [int(round(144 * (5478 / 144) ** (k / 19))) for k in range(20)]
SENTINEL_BLOCK = 3600


def _wl2_queries():
    rng = rng_for(2, 2)
    qs = [background_residues(rng, m) for m in WL2_QLENS]
    block = w_rich_block(rng_for(2, 5), SENTINEL_BLOCK)
    k = WL2_QLENS.index(3735)
    qs[k][60:60 + SENTINEL_BLOCK] = block
    return qs, block, k


def sp570k(n: int = 570_000):
    """Synthetic 570k-subject database (~2.06e8 residues), shared by workloads 2 and 3.

    Log-normal lengths median 300 clipped 20..35,000; the last 16 subjects get
    log-uniform lengths 5,000..35,000 with one exactly 35,000; 20 planted
    homologs per workload-2 query; three sentinel subjects carry the W-rich
    block of one query so their scores exceed the int16 range.
    ``n`` smaller than 570,000 gives a scaled-down database with the same recipe.
    """
    rng = rng_for(2, 0)
    lengths = lognormal_lengths(rng, n, 300, 20, 35_000)
    tail = min(16, n)
    lengths[n - tail:] = np.rint(np.exp(rng.uniform(np.log(5000), np.log(35000), size=tail))).astype(np.int64)
    lengths[n - 1] = 35_000
    qs, block, _ = _wl2_queries()
    srng = rng_for(2, 5)
    sentinels = []
    inserts = {}
    while len(sentinels) < min(3, n):
        k = int(srng.integers(0, max(1, n - tail)))
        if k in sentinels:
            continue
        sentinels.append(k)
        pre = background_residues(srng, int(srng.integers(20, 200)))
        post = background_residues(srng, int(srng.integers(20, 200)))
        inserts[k] = np.concatenate([pre, block, post])
    planted, pins = _plant(2, qs, lengths, per_query=20 if n >= 10_000 else 2, reserved=sentinels + list(range(n - tail, n)))
    inserts.update(pins)
    db = _assemble(2, lengths, inserts, f"sp{n // 1000}k")
    db.planted = planted
    db.sentinels = np.array(sorted(sentinels), dtype=np.int64)
    return db


def workload2_queries():
    """20 queries, lengths log-uniform over 144..5,478; one carries the W-rich sentinel block."""
    qs, _, _ = _wl2_queries()
    return qs


def workload3_queries(db: Database, nq: int = 256, with_sources: bool = False):
    """``nq`` queries with lengths uniform 50..5,000; each embeds a mutated DB subject
    (``with_sources``: also return those subjects' indices)."""
    rng = rng_for(3, 2)
    qs, sources = [], []
    _, block, _ = _wl2_queries()
    for i in range(nq):
        m = int(rng.integers(50, 5001))
        q = background_residues(rng, m)
        sources.append(int(rng.integers(0, db.n)))
        src = db.subject(sources[-1])
        hom = mutate(rng, src, float(rng.uniform(0.05, 0.4)), 0.01)[:m]
        at = int(rng.integers(0, m - hom.size + 1))
        q[at:at + hom.size] = hom
        qs.append(q)
    # the longest query carries the sentinel block so the int32 rerun path is exercised
    k = int(np.argmax([q.size for q in qs]))
    if qs[k].size >= SENTINEL_BLOCK + 20:
        qs[k][10:10 + SENTINEL_BLOCK] = block
    if with_sources:
        return qs, np.array(sources, dtype=np.int64)
    return qs


# ---------------------------------------------------------------- workload 4
def workload4(nq: int = 64, n: int = 10_000):
    """64 queries (500..5,000) vs 10,000 long subjects (3,000..35,000), uniform lengths."""
    rng = rng_for(4, 2)
    qs = [background_residues(rng, int(rng.integers(500, 5001))) for _ in range(nq)]
    lengths = rng_for(4, 0).integers(3000, 35_001, size=n).astype(np.int64)
    planted, inserts = _plant(4, qs, lengths, per_query=1)
    db = _assemble(4, lengths, inserts, f"long{n // 1000}k")
    db.planted = planted
    return qs, db


# ---------------------------------------------------------------- workload 5
def workload5_db(n: int = 10_000_000):
    """Serving database: log-normal lengths median 250 clipped 20..35,000, one subject of 35,000."""
    lengths = lognormal_lengths(rng_for(5, 0), n, 250, 20, 35_000)
    lengths[n - 1] = 35_000
    return _assemble(5, lengths, {}, f"serve{n // 1_000_000}M")


def workload5_queries(count: int):
    rng = rng_for(5, 2)
    ls = lognormal_lengths(rng, count, 350, 30, 5000)
    return [background_residues(rng, int(m)) for m in ls]


def poisson_arrivals(rate_per_s: float, count: int, workload: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    gaps = rng_for(workload, 4).exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps)


# ---------------------------------------------------------------- sampling
def parity_sample(db: Database, stride: int = 1000, long_threshold: int = 3000) -> np.ndarray:
    """Subjects whose scores the oracle recomputes at full size: every ``stride``-th
    subject, all planted homologs, all sentinels and every subject longer than
    ``long_threshold``."""
    idx = [np.arange(0, db.n, stride, dtype=np.int64), db.sentinels,
           np.nonzero(db.lengths > long_threshold)[0].astype(np.int64)]
    idx += list(db.planted.values())
    return np.unique(np.concatenate(idx))


def small_db(seed: int, n: int, lo: int, hi: int, median: float | None = None):
    """A small random database for parity tests (uniform or log-normal lengths)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(99, 0))))
    if median is None:
        lengths = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    else:
        lengths = lognormal_lengths(rng, n, median, lo, hi)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    res = background_residues(rng, int(offsets[-1]))
    return Database(res, offsets, name=f"small{seed}")


def small_query(seed: int, m: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(99, 1))))
    return background_residues(rng, m)
