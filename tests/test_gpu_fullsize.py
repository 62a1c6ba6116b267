"""Parity at full workload sizes, in the launch configuration bench.py times:
every signature of the 1,000,000-set bag-of-visual-words collection against the
oracle, and the candidate lists of a sample of queries (the GPU answers all
1,024, the oracle the sample); the self-join of that collection with its
queries in front (sampled rows, every j > i); the 500,000-set shingle collection (one GPU's
share of the 4,000,000-set workload over eight) with (1:2) HOPH, and sampled
MinWise signatures."""
from fractions import Fraction

import numpy as np
import pytest

import paper_1805_11254_amd as H
from oracle import scale
import workloads as W
from tests.hoph_testutil import dev_csr, oracle_sketch, params_of, to_u32

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _sample_queries(n_q, count, seed):
    rng = np.random.default_rng(seed)
    return sorted(set([0, n_q - 1] + rng.choice(n_q, size=count, replace=False).tolist()))


def _check_queries(w, sig_h, qsig_h, offs, ids, sample, policy=H.EMPTY_JOINT):
    oo, oi, _ = scale.query(sig_h, qsig_h[sample], goph=w.goph, kp=w.kp, T=Fraction(*w.T), eps=Fraction(*w.eps),
                            policy=policy, ra=w.ra, rb=w.rb)
    for j, q in enumerate(sample):
        got = ids[offs[q]:offs[q + 1]].tolist()
        want = oi[oo[j]:oo[j + 1]].tolist()
        assert got == want, (q, len(got), len(want))


def test_bovw_1M_full_signatures_and_sampled_queries():
    print("[case] bovw 1M", flush=True)
    w = W.hoph_bovw()                     # the bench workload: 1,000,000 sets, 1,024 queries
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    qids, qoffs = dev_csr(w.queries)
    sig = H.sketch_oph(p, ids, offs)
    qsig = H.sketch_oph(p, qids, qoffs)
    H.sync()
    idx = H.Index(p, sig[:0], capacity=w.collection.n)
    idx.append(sig)
    go, gi = H.query_hoph(idx, qsig, T=w.T, eps=w.eps)
    go, gi = go.cpu().numpy(), to_u32(gi)
    sig_h, qsig_h = to_u32(sig), to_u32(qsig)
    del sig, ids, offs
    osig = oracle_sketch(w, w.collection)
    bad = np.flatnonzero((osig != sig_h).any(axis=1))
    assert bad.size == 0, f"{bad.size} signatures differ, first sets {bad[:5].tolist()}"
    assert (oracle_sketch(w, w.queries) == qsig_h).all()
    _check_queries(w, osig, qsig_h, go, gi, _sample_queries(w.queries.n, 14, 1))
    idx.free()


def test_bovw_1M_self_join_sampled_rows():
    """Self-join of the bench's self-join collection (the 1,024 query sets in
    front of the 1,000,000 sets: 1,001,024 rows, 5·10^11 pairs), in the launch
    configuration bench.py times: every signature against the oracle, and for
    sampled rows i (query rows with planted copies among them) the full list
    of accepted j > i against the oracle's decisions over all j."""
    print("[case] bovw 1M self-join", flush=True)
    w = W.hoph_bovw()
    q, c = w.queries, w.collection
    coll = W.Collection(np.concatenate([q.ids, c.ids]).astype(np.uint32),
                        np.concatenate([q.offsets, c.offsets[1:] + q.offsets[-1]]).astype(np.uint64))
    n = coll.n
    p = params_of(w)
    ids, offs = dev_csr(coll)
    sig = H.sketch_oph(p, ids, offs)
    H.sync()
    idx = H.Index(p, sig)
    go, gi = H.self_join(idx, T=w.T, eps=w.eps)
    go, gi = go.cpu().numpy(), to_u32(gi)
    sig_h = to_u32(sig)
    del sig, ids, offs
    osig = oracle_sketch(w, coll)
    assert (osig == sig_h).all()
    rng = np.random.default_rng(5)
    sample = sorted(set([0, 1, q.n - 1, q.n, n - 2, n - 1] + rng.choice(q.n, size=6, replace=False).tolist()
                        + rng.choice(n, size=8, replace=False).tolist()))
    oo, oi, _ = scale.query(osig, osig[sample], goph=w.goph, kp=w.kp, T=Fraction(*w.T), eps=Fraction(*w.eps),
                            ra=w.ra, rb=w.rb)
    planted_rows = 0
    for j, i in enumerate(sample):
        want = [x for x in oi[oo[j]:oo[j + 1]].tolist() if x > i]
        got = gi[go[i]:go[i + 1]].tolist()
        assert got == want, (i, len(got), len(want))
        planted_rows += i < q.n and len(want) > 0
    assert planted_rows > 0
    idx.free()


def test_shingles_500k_hoph12_and_minwise_sample():
    import torch
    print("[case] shingles 500k", flush=True)
    w = W.hoph_shingles(n=500_000, n_q=512, seed=1807, ra=1, rb=2, T=(7, 10))
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    qids, qoffs = dev_csr(w.queries)
    sig = H.sketch_oph(p, ids, offs)
    qsig = H.sketch_oph(p, qids, qoffs)
    H.sync()
    idx = H.Index(p, sig)
    go, gi = H.query_hoph(idx, qsig, T=w.T, eps=w.eps)
    go, gi = go.cpu().numpy(), to_u32(gi)
    sig_h, qsig_h = to_u32(sig), to_u32(qsig)
    osig = oracle_sketch(w, w.collection)
    assert (osig == sig_h).all()
    _check_queries(w, osig, qsig_h, go, gi, _sample_queries(w.queries.n, 10, 2))
    idx.free()
    # MinWise with k = 512 independent hashes mod 2^32 + 15, on a sample of sets
    ha, hb = W.hash_coeffs(W.P32P15, 512, 99)
    mp = H.MinwiseParams(512, W.HASH_MODP32P15, 1 << 32, torch.from_numpy(ha.view(np.int64)).cuda(),
                         torch.from_numpy(hb.view(np.int64)).cuda())
    ms = H.minwise_sketch(mp, ids, offs).cpu().numpy().view(np.uint64)
    which = np.random.default_rng(3).choice(w.collection.n, size=150, replace=False).astype(np.uint64)
    om = scale.minwise_sketch(w.collection.ids, w.collection.offsets, hash_kind=W.HASH_MODP32P15, universe=1 << 32,
                              ha=ha, hb=hb, which=which)
    assert (ms[which.astype(np.int64)] == om).all()
