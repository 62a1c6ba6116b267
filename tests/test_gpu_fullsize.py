"""Parity at full workload sizes, in the launch configurations bench.py times,
every expected value from the oracle on its own signatures of the raw sets:

- the 1,000,000-set bag-of-visual-words collection: every signature and the
  candidate lists of all 1,024 queries; its self-join (sampled rows, every
  accepted j > i);
- the 4,000,000-set text-shingle collection over 2^32 ids, k = 256 in groups of
  32: every index row and every query signature for (1:2), (2:1) and (1:1) HOPH,
  and the candidate lists of sampled queries at T = 1/2, 7/10 and 9/10 (the GPU
  answers all 4,096); plain OPH over all 256 bins (sampled queries against every
  set) and MinWise with k = 512 (sampled sets and queries);
- batched plans (graph, tuned) on a 2,000,000-set index, uneven batches with
  query sets of up to 10,000 ids and planted near-duplicates;
- the serving loop on an 8,000,000-set k = 256 index, requests alone and in the
  mix, before and after 5% of the sets are inserted online.

Each test prints its case before the GPU runs it."""
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


def _oracle_lists(w, osig, oqsig, T=None, policy=H.EMPTY_JOINT, ra=None, rb=None):
    T = w.T if T is None else T
    oo, oi, _ = scale.query(osig, oqsig, goph=w.goph, kp=w.kp, T=Fraction(*T), eps=Fraction(*w.eps),
                            policy=policy, ra=w.ra if ra is None else ra, rb=w.rb if rb is None else rb)
    return [oi[oo[j]:oo[j + 1]].tolist() for j in range(len(oo) - 1)]


def _check_queries(w, osig, oqsig, offs, ids, sample, T=None, ra=None, rb=None):
    want = _oracle_lists(w, osig, oqsig[sample], T=T, ra=ra, rb=rb)
    for j, q in enumerate(sample):
        got = ids[offs[q]:offs[q + 1]].tolist()
        assert got == want[j], (q, len(got), len(want[j]))
    return sum(len(x) for x in want)


# ---------------------------------------------------------------------------
# 1,000,000 bag-of-visual-words sets, HOPH (1:1), k = 512
# ---------------------------------------------------------------------------
def test_bovw_1M_full_signatures_and_all_queries():
    import torch
    print("[case] bovw 1M, all 1,024 queries", flush=True)
    w = W.hoph_bovw()                     # the step's workload: 1,000,000 sets, 1,024 queries
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    qids, qoffs = dev_csr(w.queries)
    # the step's launch configuration: sketch straight into the index rows
    idx = H.Index(p, torch.empty((0, w.k), dtype=torch.int32, device="cuda"), capacity=w.collection.n)
    idx.append_sets(ids, offs)
    qsig = H.sketch_oph(p, qids, qoffs)
    H.sync()
    go, gi = H.query_hoph(idx, qsig, T=w.T, eps=w.eps)
    go, gi = go.cpu().numpy(), to_u32(gi)
    rows_h, qsig_h = to_u32(idx.rows()), to_u32(qsig)
    del ids, offs
    osig = oracle_sketch(w, w.collection)
    bad = np.flatnonzero((osig != rows_h).any(axis=1))
    assert bad.size == 0, f"{bad.size} index rows differ, first sets {bad[:5].tolist()}"
    oq = oracle_sketch(w, w.queries)
    assert (oq == qsig_h).all()
    found = _check_queries(w, osig, oq, go, gi, list(range(w.queries.n)))
    assert found > 1000
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


# ---------------------------------------------------------------------------
# 4,000,000 text-shingle sets over 2^32 ids, k = 256, HOPH (1:2), (2:1), (1:1)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def shingles_4M():
    print("[case] shingles 4M: generating", flush=True)
    w = W.hoph_shingles()                 # 4,000,000 sets, 4,096 queries, about 10 planted per query
    ids, offs = dev_csr(w.collection)
    qids, qoffs = dev_csr(w.queries)
    yield w, ids, offs, qids, qoffs
    del ids, offs, qids, qoffs


@pytest.mark.parametrize("ra,rb", [(1, 2), (2, 1), (1, 1)])
def test_shingles_4M_hoph_all_thresholds(shingles_4M, ra, rb):
    print(f"[case] shingles 4M HOPH {ra}:{rb}", flush=True)
    w, ids, offs, qids, qoffs = shingles_4M
    p = H.SketchParams(w.layout, w.k, w.kp, w.hash_kind, w.universe, ra, rb, w.ha, w.hb)
    qsig = H.sketch_oph(p, qids, qoffs)
    idx = H.Index(p, qsig[:0], capacity=w.collection.n)
    idx.append_sets(ids, offs)
    H.sync()
    results = {}
    for T in ((1, 2), (7, 10), (9, 10)):
        go, gi = H.query_hoph(idx, qsig, T=T, eps=w.eps)
        results[T] = (go.cpu().numpy(), to_u32(gi))
    rows_h, qsig_h = to_u32(idx.rows()), to_u32(qsig)
    idx.free()
    del qsig
    kw = dict(hash_kind=w.hash_kind, universe=w.universe, layout=w.layout, k=w.k, kp=w.kp, ra=ra, rb=rb,
              ha=w.ha, hb=w.hb)
    osig = scale.sketch(w.collection.ids, w.collection.offsets, **kw)
    bad = np.flatnonzero((osig != rows_h).any(axis=1))
    assert bad.size == 0, f"{bad.size} index rows differ, first sets {bad[:5].tolist()}"
    del rows_h
    oq = scale.sketch(w.queries.ids, w.queries.offsets, **kw)
    assert (oq == qsig_h).all()
    sample = _sample_queries(w.queries.n, 14, 7 + ra)
    for T, (go, gi) in results.items():
        found = _check_queries(w, osig, oq, go, gi, sample, T=T, ra=ra, rb=rb)
        assert found > 0, T


def test_shingles_4M_plain_oph_and_minwise(shingles_4M):
    """The comparators on the same collection: plain OPH (Eq. 6 over all 256
    bins, no early stop) for sampled queries against all 4,000,000 sets, and
    MinWise with k = 512 independent hashes mod 2^32 + 15 (every set sketched on
    the GPU; sampled sets' signatures, and sampled queries against the planted
    copies and 4,000 other sets)."""
    import torch
    print("[case] shingles 4M plain OPH and MinWise", flush=True)
    w, ids, offs, qids, qoffs = shingles_4M
    p = H.SketchParams(W.LAYOUT_OPH, w.k, w.kp, w.hash_kind, w.universe, 1, 1, w.ha, w.hb)
    sample = _sample_queries(w.queries.n, 14, 11)
    qsig = H.sketch_oph(p, qids, qoffs)
    sub = qsig[sample].contiguous()
    idx = H.Index(p, qsig[:0], capacity=w.collection.n)
    idx.append_sets(ids, offs)
    H.sync()
    for T in ((1, 2), (7, 10), (9, 10)):
        go, gi = H.query_oph_full(idx, sub, T=T)
        go, gi = go.cpu().numpy(), to_u32(gi)
        if T == (1, 2):
            kw = dict(hash_kind=w.hash_kind, universe=w.universe, layout=W.LAYOUT_OPH, k=w.k, kp=w.kp,
                      ha=w.ha, hb=w.hb)
            osig = scale.sketch(w.collection.ids, w.collection.offsets, **kw)
            oq = scale.sketch(w.queries.ids, w.queries.offsets, which=np.array(sample, dtype=np.uint64), **kw)
            assert (to_u32(sub) == oq).all()
        oo, oi = scale.query_oph_full(osig, oq, T=Fraction(*T))
        assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist(), T
    idx.free()
    del osig
    # MinWise, k = 512
    ha, hb = W.hash_coeffs(W.P32P15, 512, 99)
    mp = H.MinwiseParams(512, W.HASH_MODP32P15, 1 << 32, torch.from_numpy(ha.view(np.int64)).cuda(),
                         torch.from_numpy(hb.view(np.int64)).cuda())
    ms = H.minwise_sketch(mp, ids, offs)          # every set: 4,000,000 x 512 minima
    # a subset of rows: the planted copies of the sampled queries and random others
    rng = np.random.default_rng(3)
    rows = sorted(set([s for (q, s, J) in w.planted if q in set(sample)]
                      + rng.choice(w.collection.n, size=4000, replace=False).tolist()))
    rows_u = np.array(rows, dtype=np.uint64)
    om = scale.minwise_sketch(w.collection.ids, w.collection.offsets, hash_kind=W.HASH_MODP32P15, universe=1 << 32,
                              ha=ha, hb=hb, which=rows_u)
    ms_sub = ms[torch.as_tensor(rows_u.astype(np.int64), device="cuda")].contiguous()
    assert (ms_sub.cpu().numpy().view(np.uint64) == om).all()
    del ms
    omq = scale.minwise_sketch(w.queries.ids, w.queries.offsets, hash_kind=W.HASH_MODP32P15, universe=1 << 32,
                               ha=ha, hb=hb, which=np.array(sample, dtype=np.uint64))
    mq = H.minwise_sketch(mp, qids, qoffs)[sample].contiguous()
    assert (mq.cpu().numpy().view(np.uint64) == omq).all()
    found = 0
    for T in ((1, 2), (7, 10)):
        go, gi = H.minwise_query(mp, ms_sub, mq, T=T)
        oo, oi = scale.minwise_query(om, omq, T=Fraction(*T))
        assert go.cpu().numpy().tolist() == oo.tolist() and to_u32(gi).tolist() == oi.tolist(), T
        found += len(oi)
    assert found > 0


# ---------------------------------------------------------------------------
# Batched plans on a 2,000,000-set index (k = 512), uneven batches
# ---------------------------------------------------------------------------
def test_batched_2M_plan_sampled_batches():
    import torch
    print("[case] batched plan, 2M-set index", flush=True)
    N, chunk = 2_000_000, 1_000_000
    a, b = W.hash_coeffs(W.P31, 1, 1809)
    p = H.SketchParams(W.LAYOUT_HIER, 512, 32, W.HASH_MODP31, 1 << 20, 1, 1, int(a[0]), int(b[0]))
    w = W.Workload("batched", None, None, 1 << 20, W.HASH_MODP31, W.LAYOUT_HIER, 512, 32, ha=int(a[0]),
                   hb=int(b[0]))
    idx, osigs, first = None, [], None
    for c0 in range(0, N, chunk):
        coll = W.zipf_sets(chunk, 1 << 20, 600, 0.75, 100, 4000, 1806 + 1000 * (c0 // chunk))
        ids, offs = dev_csr(coll)
        if idx is None:
            idx = H.Index(p, torch.empty((0, 512), dtype=torch.int32, device="cuda"), capacity=N)
            first = coll
        idx.append_sets(ids, offs)
        torch.cuda.synchronize()
        osigs.append(oracle_sketch(w, coll))
        del ids, offs
    osig = np.concatenate(osigs)
    del osigs
    assert (to_u32(idx.rows(0, 4096)) == osig[:4096]).all() and (to_u32(idx.rows(N - 4096)) == osig[-4096:]).all()
    batches = W.query_batches(40, 1856)
    cw = np.random.default_rng(1806 + 7).permutation(1 << 20).astype(np.uint32)
    fresh = lambda g, c: cw[W._zipf_ranks(g, 1 << 20, c, 1.1)]
    batches, truth = W.plant_queries(batches, first, 0.05, 0.5, 0.98, fresh, 1857)
    del first
    # a small, a median and a large batch, and the batch with the longest query set
    sizes = np.array([bt.n for bt in batches])
    longest = int(np.argmax([bt.sizes().max() for bt in batches]))
    pick = sorted(set([int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes)),
                       longest]))
    assert max(batches[longest].sizes()) >= 9000
    max_ids = max(int(batches[i].ids.size) for i in pick)
    plan = H.Plan(idx, p, T=(4, 5), eps=(1, 10000), max_queries=4096, max_query_ids=max_ids, max_results=1 << 20,
                  use_graph=True, tune=True)
    planted_found = 0
    for bi in pick:
        bt = batches[bi]
        qi, qo = dev_csr(bt)
        plan.run(qi, qo)
        go, gi = plan.results()
        go, gi = go.cpu().numpy(), to_u32(gi)
        oq = oracle_sketch(w, bt)
        assert (to_u32(plan.query_sigs(512)) == oq).all(), bi
        # every query of a batch of up to 256; else the planted ones and 48 others
        planted = sorted(set(q for (b_, q, row, J) in truth if b_ == bi))
        check = list(range(bt.n)) if bt.n <= 256 else sorted(set(planted + _sample_queries(bt.n, 48, bi)))
        want = dict(zip(check, _oracle_lists(w, osig, oq[check])))
        for q in check:
            assert gi[go[q]:go[q + 1]].tolist() == want[q], (bi, q)
        planted_found += sum(1 for (b_, q, row, J) in truth if b_ == bi and row in set(want[q]))
    assert planted_found > 0
    assert plan.info()["graph"] == 1 and plan.info()["fallbacks"] == 0
    plan.free()
    idx.free()


# ---------------------------------------------------------------------------
# Serving on an 8,000,000-set k = 256 index with 5% inserted online
# ---------------------------------------------------------------------------
def test_serving_8M_with_inserts_sampled_requests():
    import torch
    print("[case] serving, 8M-set index with inserts", flush=True)
    N, chunk = 8_000_000, 1_000_000
    n_ins = N // 20
    a, b = W.hash_coeffs(W.P31, 1, 1809)
    p = H.SketchParams(W.LAYOUT_HIER, 256, 32, W.HASH_MODP31, 1 << 20, 1, 1, int(a[0]), int(b[0]))
    w = W.Workload("serving", None, None, 1 << 20, W.HASH_MODP31, W.LAYOUT_HIER, 256, 32, ha=int(a[0]),
                   hb=int(b[0]))
    cw = np.random.default_rng(1806 + 7).permutation(1 << 20).astype(np.uint32)
    fresh = lambda g, c: cw[W._zipf_ranks(g, 1 << 20, c, 1.1)]
    # requests: log-normal sizes (median 800); the first 8 have near-duplicates in
    # the first chunk, the next 8 among the inserted sets
    t_arr, req = W.poisson_arrivals(50_000, 32, 1877)
    req8 = W.Collection(req.ids[:int(req.offsets[8])], req.offsets[:9])
    req16 = W.Collection(req.ids[int(req.offsets[8]):int(req.offsets[16])], req.offsets[8:17] - req.offsets[8])
    idx, osigs = None, []
    for c0 in range(0, N, chunk):
        coll = W.zipf_sets(chunk, 1 << 20, 600, 0.75, 100, 4000, 1806 + 1000 * (c0 // chunk))
        if c0 == 0:
            coll, _ = W.plant(coll, req8, 3, 0.6, 0.98, fresh, 1878)
        ids, offs = dev_csr(coll)
        if idx is None:
            idx = H.Index(p, torch.empty((0, 256), dtype=torch.int32, device="cuda"), capacity=N + n_ins)
        idx.append_sets(ids, offs)
        torch.cuda.synchronize()
        osigs.append(oracle_sketch(w, coll))
        del ids, offs, coll
    osig = np.concatenate(osigs)
    del osigs
    assert (to_u32(idx.rows(N - 4096)) == osig[-4096:]).all()
    oq = oracle_sketch(w, req)
    srv = H.Server(idx, p, T=(4, 5), eps=(1, 10000), slots=4, max_batch_queries=256, max_batch_ids=1 << 20,
                   max_batch_results=1 << 16, use_graph=True, tune=True)

    def served(arrivals):
        ro, ri = srv.replay(req.ids, req.offsets, arrivals, keep_results=True)
        return [ri[ro[j]:ro[j + 1]].tolist() for j in range(req.n)]

    want = _oracle_lists(w, osig, oq)
    assert sum(len(x) > 0 for x in want[:8]) >= 6
    alone = [srv.wait(srv.submit(req.set(j))).tolist() for j in range(req.n)]
    assert alone == want
    assert served(t_arr - t_arr[0]) == want             # Poisson arrivals at 50k q/s
    assert served(np.zeros(req.n)) == want              # all at once
    # 5% more sets inserted online, near-duplicates of requests 8..15 among them
    extra = W.zipf_sets(n_ins, 1 << 20, 600, 0.75, 100, 4000, 1896)
    extra, _ = W.plant(extra, req16, 3, 0.6, 0.98, fresh, 1897)
    for lo in range(0, n_ins, n_ins // 4):
        hi = min(n_ins, lo + n_ins // 4)
        o = extra.offsets[lo:hi + 1]
        srv.insert(extra.ids[int(o[0]):int(o[-1])], o - o[0])
    assert len(idx) == N + n_ins
    osig = np.concatenate([osig, oracle_sketch(w, extra)])
    want2 = _oracle_lists(w, osig, oq)
    assert sum(any(x >= N for x in want2[j]) for j in range(8, 16)) >= 6
    assert served(t_arr - t_arr[0]) == want2
    assert [srv.wait(srv.submit(req.set(j))).tolist() for j in range(req.n)] == want2
    assert srv.stats()["inserted_sets"] == n_ins
    srv.close()
    idx.free()
