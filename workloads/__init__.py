"""Seeded synthetic workloads shaped like the paper's (Sec. 5: text shingle
sets and bag-of-visual-words image sets, 100-query workloads, planted near
duplicates).  The paper's own datasets (a private proposal corpus and an
ImageNet/SIFT subset) are not available; these generators stand in for them.

This module holds no arithmetic of the method: it only draws sets, queries,
planted near-duplicates and the random permutation / hash coefficients that
the method consumes.  Both the GPU path and the oracle take its outputs as
inputs.  Every draw comes from numpy's PCG64 seeded explicitly.

A collection is CSR: ``ids`` uint32[nnz] and ``offsets`` uint64[n+1].
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

P31 = (1 << 31) - 1
P32P15 = (1 << 32) + 15
HASH_TABLE, HASH_MODP31, HASH_MODP32P15 = 0, 1, 2
LAYOUT_OPH, LAYOUT_HIER = 0, 1


@dataclass
class Collection:
    ids: np.ndarray                # uint32[nnz]
    offsets: np.ndarray            # uint64[n + 1]

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def set(self, i: int) -> np.ndarray:
        return self.ids[int(self.offsets[i]):int(self.offsets[i + 1])]

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))


@dataclass
class Workload:
    name: str
    collection: Collection
    queries: Collection
    universe: int
    hash_kind: int
    layout: int
    k: int
    kp: int
    ra: int = 1
    rb: int = 1
    T: Tuple[int, int] = (4, 5)
    eps: Tuple[int, int] = (1, 10000)
    perm: Optional[np.ndarray] = None
    ha: int = 0
    hb: int = 0
    planted: List[Tuple[int, int, float]] = field(default_factory=list)  # (query, set, exact J)

    @property
    def goph(self) -> bool:
        return self.layout == LAYOUT_OPH


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def csr_from_lists(sets) -> Collection:
    sizes = np.array([len(s) for s in sets], dtype=np.uint64)
    offsets = np.zeros(len(sets) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    ids = (np.concatenate([np.asarray(s, dtype=np.uint32) for s in sets])
           if len(sets) and offsets[-1] else np.zeros(0, dtype=np.uint32))
    return Collection(ids, offsets)


def perm_table(D: int, seed: int) -> np.ndarray:
    """A uniformly random permutation of [0, D) (Fisher-Yates by numpy)."""
    return np.random.default_rng(seed).permutation(D).astype(np.uint32)


def hash_coeffs(p: int, count: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """count pairs (a, b) with 1 <= a < p and 0 <= b < p."""
    rng = np.random.default_rng(seed)
    a = rng.integers(1, p, size=count, dtype=np.uint64)
    b = rng.integers(0, p, size=count, dtype=np.uint64)
    return a, b


# --------------------------------------------------------------------------
# Element samplers
# --------------------------------------------------------------------------
def _zipf_ranks(rng, n: int, count: int, s: float) -> np.ndarray:
    """Ranks in [0, n) with P(rank r) roughly proportional to (r+1)^-s, by
    inverting the continuous power law on [1, n+1)."""
    u = rng.random(count, dtype=np.float64)
    c = 1.0 - (n + 1.0) ** (1.0 - s)
    x = np.power(1.0 - u * c, 1.0 / (1.0 - s))
    r = np.floor(x).astype(np.int64) - 1
    np.clip(r, 0, n - 1, out=r)
    return r


def _splitmix64_finalize(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixer (Steele, Lea, Flood 2014) on uint64."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def _parallel_fill(total: int, seed: int, fn, dtype=np.uint32, chunk: int = 1 << 24) -> np.ndarray:
    """Fill uint32[total] chunk by chunk, each chunk from its own child seed."""
    out = np.empty(total, dtype=dtype)
    nchunks = max(1, (total + chunk - 1) // chunk)
    seeds = np.random.SeedSequence(seed).spawn(nchunks)

    def work(i):
        lo, hi = i * chunk, min(total, (i + 1) * chunk)
        if hi > lo:
            out[lo:hi] = fn(np.random.default_rng(seeds[i]), hi - lo)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nchunks)))
    return out


def _offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes.astype(np.uint64), out=off[1:])
    return off


# --------------------------------------------------------------------------
# Collections
# --------------------------------------------------------------------------
def uniform_distinct_sets(n: int, D: int, lo: int, hi: int, seed: int) -> Collection:
    """n sets of distinct uniform ids in [0, D), sizes uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=n)
    return csr_from_lists([np.sort(rng.choice(D, size=int(m), replace=False)) for m in sizes])


def zipf_sets(n: int, D: int, median: float, sigma: float, lo: int, hi: int, seed: int,
              s: float = 1.1) -> Collection:
    """Bag-of-visual-words-like sets: sizes round(LogNormal(ln median, sigma))
    clipped to [lo, hi]; codewords drawn with Zipf(s) frequencies over D
    codewords, frequent codewords scattered over the id space by a seeded
    permutation.  Repeated draws of a codeword inside a set are kept (a bag);
    the set is the distinct ids."""
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.rint(rng.lognormal(math.log(median), sigma, size=n)), lo, hi).astype(np.int64)
    cw = np.random.default_rng(seed + 7).permutation(D).astype(np.uint32)
    total = int(sizes.sum())
    ids = _parallel_fill(total, seed + 11, lambda g, m: cw[_zipf_ranks(g, D, m, s)])
    return Collection(ids, _offsets(sizes))


def shingle_sets(n: int, lo: int, hi: int, seed: int) -> Collection:
    """Text-shingle-like sets: uniform 64-bit shingle ids mixed to uint32 by
    the SplitMix64 finalizer; sizes uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=n)
    total = int(sizes.sum())

    def draw(g, m):
        z = g.integers(0, np.iinfo(np.uint64).max, size=m, dtype=np.uint64, endpoint=True)
        return (_splitmix64_finalize(z) & np.uint64(0xFFFFFFFF)).astype(np.uint32)

    ids = _parallel_fill(total, seed + 13, draw)
    return Collection(ids, _offsets(sizes))


def loguniform_sizes(rng, count: int, lo: int, hi: int) -> np.ndarray:
    return np.clip(np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))), lo, hi).astype(np.int64)


# --------------------------------------------------------------------------
# Planted near-duplicates
# --------------------------------------------------------------------------
def plant(coll: Collection, queries: Collection, per_query: int, j_lo: float, j_hi: float,
          fresh, seed: int) -> Tuple[Collection, List[Tuple[int, int, float]]]:
    """Overwrite per_query random collection slots per query with a near
    duplicate of that query: drop x of its m distinct ids and add x fresh ids,
    J = (m - x)/(m + x), J target uniform in [j_lo, j_hi].  fresh(rng, count)
    draws candidate ids.  Returns the new collection and (query, slot, J)."""
    rng = np.random.default_rng(seed)
    n = coll.n
    nq = queries.n
    slots = rng.choice(n, size=nq * per_query, replace=False)
    repl = {}
    truth = []
    for qi in range(nq):
        Q = np.unique(queries.set(qi))
        for r in range(per_query):
            J = rng.uniform(j_lo, j_hi)
            newset, Jx = _perturb(rng, Q, J, fresh)
            slot = int(slots[qi * per_query + r])
            repl[slot] = newset
            truth.append((qi, slot, Jx))
    return replace_sets(coll, repl), truth


def _perturb(rng, Q: np.ndarray, J: float, fresh) -> Tuple[np.ndarray, float]:
    """A set at Jaccard about J from the distinct ids Q: drop x of its m ids and
    add x fresh ones, x = round(m (1 - J) / (1 + J)); returns it (sorted) and its
    exact J = (m - x) / (m + x)."""
    m = len(Q)
    x = int(round(m * (1 - J) / (1 + J)))
    x = max(0, min(x, m - 1))
    keep = rng.choice(Q, size=m - x, replace=False)
    add = np.zeros(0, dtype=np.uint32)
    while len(add) < x:
        cand = np.unique(np.asarray(fresh(rng, 4 * x + 8), dtype=np.uint32))
        cand = cand[~np.isin(cand, Q)]
        add = np.unique(np.concatenate([add, cand]))
    add = rng.permutation(add)[:x]
    return np.sort(np.concatenate([keep, add]).astype(np.uint32)), (m - x) / (m + x)


def plant_queries(batches: List[Collection], source: Collection, frac: float, j_lo: float, j_hi: float,
                  fresh, seed: int, row_offset: int = 0):
    """Replace a fraction of the queries of each batch with near-duplicates of
    random sets of `source` (the collection, or a prefix of it) at J in
    [j_lo, j_hi].  Returns the new batches and (batch, query, source row +
    row_offset, exact J) per planted query."""
    rng = np.random.default_rng(seed)
    out, truth = [], []
    for bi, b in enumerate(batches):
        n_dup = int(rng.binomial(b.n, frac))
        if n_dup == 0:
            out.append(b)
            continue
        which = np.sort(rng.choice(b.n, size=n_dup, replace=False))
        sets = [b.set(i) for i in range(b.n)]
        for qi in which.tolist():
            row = int(rng.integers(0, source.n))
            J = rng.uniform(j_lo, j_hi)
            sets[qi], Jx = _perturb(rng, np.unique(source.set(row)), J, fresh)
            truth.append((bi, qi, row + row_offset, Jx))
        out.append(csr_from_lists(sets))
    return out, truth


def replace_sets(coll: Collection, repl: dict) -> Collection:
    """Collection with the sets at the given slots replaced."""
    if not repl:
        return coll
    sizes = coll.sizes().copy()
    for slot, s in repl.items():
        sizes[slot] = len(s)
    offsets = _offsets(sizes)
    ids = np.empty(int(offsets[-1]), dtype=np.uint32)
    # copy the untouched runs between replaced slots in bulk
    order = sorted(repl)
    prev = 0
    for slot in order + [coll.n]:
        if slot > prev:
            a, b = int(coll.offsets[prev]), int(coll.offsets[slot])
            ids[int(offsets[prev]):int(offsets[prev]) + (b - a)] = coll.ids[a:b]
        if slot < coll.n:
            ids[int(offsets[slot]):int(offsets[slot + 1])] = repl[slot]
        prev = slot + 1
    return Collection(ids, offsets)


# --------------------------------------------------------------------------
# The five workload shapes
# --------------------------------------------------------------------------
def tiny_goph(seed: int = 1805, n: int = 2000, n_q: int = 16, per_query: int = 10) -> Workload:
    """2,000 sets of 50-500 distinct ids over D = 2^16, explicit seeded
    permutation, OPH k = 128 in GOPH groups of 16, 16 queries with 10 planted
    near-duplicates each at J in [0.7, 0.95], T = 4/5."""
    D = 1 << 16
    coll = uniform_distinct_sets(n, D, 50, 500, seed)
    qs = uniform_distinct_sets(n_q, D, 50, 500, seed + 1)
    coll, truth = plant(coll, qs, per_query, 0.7, 0.95, lambda g, c: g.integers(0, D, size=c), seed + 2)
    return Workload("oph_goph_2k", coll, qs, D, HASH_TABLE, LAYOUT_OPH, 128, 16,
                    T=(4, 5), perm=perm_table(D, seed + 3), planted=truth)


def hoph_bovw(n: int = 1_000_000, n_q: int = 1024, seed: int = 1806, k: int = 512, kp: int = 32,
              ra: int = 1, rb: int = 1, planted_frac: float = 0.01, T=(4, 5)) -> Workload:
    """Bag-of-visual-words sets over D = 2^20 codewords (Zipf(1.1)), sizes
    log-normal with median 600 clipped to [100, 4000]; hash (a x + b) mod
    (2^31 - 1); HOPH a:b with k bins in groups of k'; 1% of the collection
    planted as near-duplicates of the queries at J in [0.5, 0.98]."""
    D = 1 << 20
    coll = zipf_sets(n, D, 600, 0.75, 100, 4000, seed)
    qs = zipf_sets(n_q, D, 600, 0.75, 100, 4000, seed + 1)
    per_q = max(1, int(round(planted_frac * n / max(1, n_q))))
    per_q = min(per_q, max(1, n // max(1, n_q)))
    cw = np.random.default_rng(seed + 7).permutation(D).astype(np.uint32)
    fresh = lambda g, c: cw[_zipf_ranks(g, D, c, 1.1)]
    coll, truth = plant(coll, qs, per_q, 0.5, 0.98, fresh, seed + 2)
    a, b = hash_coeffs(P31, 1, seed + 3)
    return Workload(f"hoph{ra}{rb}_bovw_{n}", coll, qs, D, HASH_MODP31, LAYOUT_HIER, k, kp,
                    ra=ra, rb=rb, T=T, ha=int(a[0]), hb=int(b[0]), planted=truth)


def hoph_shingles(n: int = 4_000_000, n_q: int = 4096, seed: int = 1807, k: int = 256, kp: int = 32,
                  ra: int = 1, rb: int = 2, per_query: int = 10, T=(7, 10)) -> Workload:
    """Text-shingle sets over D = 2^32 (64-bit shingles mixed to uint32),
    sizes uniform 20-2000; hash (a x + b) mod (2^32 + 15); HOPH a:b, k bins in
    groups of k'; about 10 planted near-duplicates per query at J in
    [0.5, 0.98]."""
    D = 1 << 32
    coll = shingle_sets(n, 20, 2000, seed)
    qs = shingle_sets(n_q, 20, 2000, seed + 1)
    per_q = min(per_query, max(1, n // max(1, n_q)))
    fresh = lambda g, c: g.integers(0, D, size=c, dtype=np.uint64).astype(np.uint32)
    coll, truth = plant(coll, qs, per_q, 0.5, 0.98, fresh, seed + 2)
    a, b = hash_coeffs(P32P15, 1, seed + 3)
    return Workload(f"hoph{ra}{rb}_shingles_{n}", coll, qs, D, HASH_MODP32P15, LAYOUT_HIER, k, kp,
                    ra=ra, rb=rb, T=T, ha=int(a[0]), hb=int(b[0]), planted=truth)


def query_batches(n_batches: int, seed: int, max_batch: int = 4096, lo: int = 10, hi: int = 10_000,
                  D: int = 1 << 20) -> List[Collection]:
    """Uneven query batches: batch size round(exp(U[0, ln max_batch])), query
    set sizes log-uniform in [lo, hi], Zipf(1.1) codewords."""
    rng = np.random.default_rng(seed)
    cw = np.random.default_rng(seed + 7).permutation(D).astype(np.uint32)
    out = []
    for _ in range(n_batches):
        bs = int(np.clip(np.rint(np.exp(rng.uniform(0, math.log(max_batch)))), 1, max_batch))
        sizes = loguniform_sizes(rng, bs, lo, hi)
        ids = cw[_zipf_ranks(rng, D, int(sizes.sum()), 1.1)]
        out.append(Collection(ids, _offsets(sizes)))
    return out


def poisson_arrivals(rate_qps: float, count: int, seed: int, median: float = 800, sigma: float = 0.75,
                     lo: int = 10, hi: int = 10_000, D: int = 1 << 20):
    """Arrival times (s) of a Poisson stream and the request sets (log-normal
    sizes, Zipf(1.1) codewords)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_qps, size=count))
    sizes = np.clip(np.rint(rng.lognormal(math.log(median), sigma, size=count)), lo, hi).astype(np.int64)
    cw = np.random.default_rng(seed + 7).permutation(D).astype(np.uint32)
    ids = cw[_zipf_ranks(rng, D, int(sizes.sum()), 1.1)]
    return t, Collection(ids, _offsets(sizes))
