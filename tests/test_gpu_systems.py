"""Batched execution (hoph_plan_*): persistent kernels that read the batch
size from device memory, one captured hipGraph replayed per batch, tile shapes
tuned on the first batch; and the serving loop (hoph_server_*).  Every expected
value comes from the oracle on its own signatures of the raw sets (collection,
query sets of 3 to 10,000 ids, online inserts): the plan's query signatures (the
chunked sketch) and every result list must equal the oracle's bit for bit, for
every batch size, with and without the graph, tuned or not, across graph
replays interleaved with other device work, and for each served request alone
and in the mix."""
from fractions import Fraction

import numpy as np
import pytest

import paper_1805_11254_amd as H
from oracle import scale
import workloads as W
from tests.hoph_testutil import dev_csr, oracle_sketch, params_of, to_u32

pytestmark = pytest.mark.gpu


def _batch(coll: W.Collection, rows):
    return W.csr_from_lists([coll.set(i) for i in rows])


def _host_path(w, p, idx, qc):
    ids, offs = dev_csr(qc)
    qsig = H.sketch_oph(p, ids, offs)
    fn = H.query_goph if w.goph else H.query_hoph
    o, i = fn(idx, qsig, T=w.T, eps=w.eps)
    return o.cpu().numpy().tolist(), to_u32(i).tolist(), to_u32(qsig)


def _plan_path(plan, qc):
    ids, offs = dev_csr(qc)
    plan.run(ids, offs)
    o, i = plan.results()
    return o.cpu().numpy().tolist(), to_u32(i).tolist()


def _oracle_csr(w, osig, oqsig):
    """The oracle's CSR (offsets, ids) for its own query signatures against its
    own collection signatures."""
    oo, oi, _ = scale.query(osig, oqsig, goph=w.goph, kp=w.kp, T=Fraction(*w.T), eps=Fraction(*w.eps),
                            ra=w.ra, rb=w.rb)
    return oo.tolist(), oi.tolist()


def _oracle_lists(w, osig, oqsig):
    o, i = _oracle_csr(w, osig, oqsig)
    return [i[o[j]:o[j + 1]] for j in range(len(o) - 1)]


@pytest.fixture(scope="module")
def bovw():
    w = W.hoph_bovw(n=30_011, n_q=300, seed=31, planted_frac=0.05)
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    sig = H.sketch_oph(p, ids, offs)
    idx = H.Index(p, sig)
    # query sets of very uneven sizes: the workload's queries plus long and short ones
    rng = np.random.default_rng(4)
    extra = [rng.choice(1 << 20, size=n, replace=False).astype(np.uint32) for n in (10, 12, 9000, 10_000, 3)]
    qsets = [w.queries.set(i) for i in range(w.queries.n)] + extra
    qc = W.csr_from_lists(qsets)
    # the oracle's own signatures of the raw sets
    osig = oracle_sketch(w, w.collection)
    oq = oracle_sketch(w, qc)
    assert (to_u32(sig) == osig).all()
    yield w, p, idx, sig, qc, osig, oq
    idx.free()


def test_oracle_covers_long_query_sets(bovw):
    """The 9,000- and 10,000-id query sets: the host path's sketch against the
    oracle's."""
    print("[case] long query sets", flush=True)
    w, p, idx, sig, qc, osig, oq = bovw
    rows = [300, 301, 302, 303, 304]
    assert max(qc.sizes()[rows]) == 10_000
    ids, offs = dev_csr(_batch(qc, rows))
    assert (to_u32(H.sketch_oph(p, ids, offs)) == oq[rows]).all()


@pytest.mark.parametrize("use_graph,tune", [(False, False), (True, False), (True, True)])
def test_plan_equals_host_path_and_oracle(bovw, use_graph, tune):
    print(f"[case] plan graph={use_graph} tune={tune}", flush=True)
    w, p, idx, sig, qc, osig, oq = bovw
    plan = H.Plan(idx, p, T=w.T, eps=w.eps, max_queries=256, max_query_ids=400_000, max_results=1 << 16,
                  use_graph=use_graph, tune=tune)
    for rows in ([0], list(range(7)), list(range(150, 278)), list(range(299, 305)), [303, 304, 1, 2],
                 list(range(256))):
        sub = _batch(qc, rows)
        want_o, want_i = _oracle_csr(w, osig, oq[rows])
        host_o, host_i, qsig_h = _host_path(w, p, idx, sub)
        assert (qsig_h == oq[rows]).all(), rows[:5]
        assert (host_o, host_i) == (want_o, want_i), rows[:5]
        got_o, got_i = _plan_path(plan, sub)
        # the chunked sketch of the plan against the oracle's signatures
        assert (to_u32(plan.query_sigs(w.k)) == oq[rows]).all(), rows[:5]
        assert (got_o, got_i) == (want_o, want_i), rows[:5]
    info = plan.info()
    assert info["graph"] == (1 if use_graph else 0) and info["tuned"] == (1 if tune else 0)
    assert info["fallbacks"] == 0
    plan.free()


def test_graph_replays_interleaved_with_eager_work(bovw):
    import torch
    print("[case] graph replays", flush=True)
    w, p, idx, sig, qc, osig, oq = bovw
    eager = H.Plan(idx, p, T=w.T, eps=w.eps, max_queries=128, max_query_ids=400_000, max_results=1 << 15,
                   use_graph=False)
    graph = H.Plan(idx, p, T=w.T, eps=w.eps, max_queries=128, max_query_ids=400_000, max_results=1 << 15,
                   use_graph=True)
    rng = np.random.default_rng(8)
    for rep in range(6):
        rows = sorted(rng.choice(qc.n, size=int(rng.integers(1, 128)), replace=False).tolist())
        sub = _batch(qc, rows)
        want = _plan_path(eager, sub)
        # unrelated device work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        torch.cuda.synchronize()
        got = _plan_path(graph, sub)
        assert got == want, rep
        assert got == _oracle_csr(w, osig, oq[rows]), rep
    assert graph.info()["graph"] == 1
    eager.free()
    graph.free()


def test_plan_capacity_and_fallbacks(bovw):
    print("[case] plan fallbacks", flush=True)
    w, p, idx, sig, qc, osig, oq = bovw
    sub = _batch(qc, list(range(40)))
    want_o, want_i = _oracle_csr(w, osig, oq[:40])
    need = len(want_i)
    assert need >= 2
    small = H.Plan(idx, p, T=w.T, eps=w.eps, max_queries=64, max_query_ids=100_000, max_results=need - 1)
    ids, offs = dev_csr(sub)
    small.run(ids, offs)
    with pytest.raises(H.HophError) as ei:
        small.results()
    assert ei.value.status == H.HOPH_E_CAPACITY and ei.value.needed == need
    # a batch larger than the plan is refused before any launch
    with pytest.raises(H.HophError) as ei:
        big = _batch(qc, list(range(65)))
        bi, bo = dev_csr(big)
        small.run(bi, bo)
    assert ei.value.status == H.HOPH_E_CAPACITY
    small.free()


def test_plan_query_with_many_results_falls_back_exactly():
    """Near-identical collection: one query accepts more than 4096 sets, which
    the per-query LDS sort does not take; the plan redoes the batch exactly."""
    print("[case] plan big segment", flush=True)
    rng = np.random.default_rng(6)
    base = rng.choice(1 << 20, size=200, replace=False)
    sets = []
    for i in range(9000):
        s = base.copy()
        s[rng.integers(0, 200, size=3)] = rng.integers(0, 1 << 20, size=3)
        sets.append(s)
    coll = W.csr_from_lists(sets)
    w = W.Workload("same", coll, coll, 1 << 20, W.HASH_MODP31, W.LAYOUT_HIER, 256, 32, ha=1234567, hb=89)
    p = params_of(w)
    ids, offs = dev_csr(coll)
    sig = H.sketch_oph(p, ids, offs)
    idx = H.Index(p, sig)
    q = _batch(coll, [0, 1, 2])
    osig = oracle_sketch(w, coll)
    assert (to_u32(sig) == osig).all()
    want_o, want_i = _oracle_csr(w, osig, osig[:3])
    assert max(np.diff(want_o)) > 4096
    assert _host_path(w, p, idx, q)[:2] == (want_o, want_i)
    plan = H.Plan(idx, p, T=w.T, eps=w.eps, max_queries=4, max_query_ids=10_000, max_results=1 << 16)
    got = _plan_path(plan, q)
    assert got == (want_o, want_i)
    assert plan.info()["fallbacks"] == 1 and plan.info()["fallback_causes"] == 4   # the per-query sort's limit
    plan.free()
    idx.free()


def test_goph_plan_matches_oracle():
    print("[case] goph plan", flush=True)
    w = W.tiny_goph()
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    sig = H.sketch_oph(p, ids, offs)
    idx = H.Index(p, sig)
    plan = H.Plan(idx, p, T=w.T, eps=w.eps, max_queries=16, max_query_ids=20_000, max_results=4096, tune=True)
    got_o, got_i = _plan_path(plan, w.queries)
    osig, oq = oracle_sketch(w, w.collection), oracle_sketch(w, w.queries)
    assert (to_u32(sig) == osig).all()
    assert (to_u32(plan.query_sigs(w.k)) == oq).all()
    assert (got_o, got_i) == _oracle_csr(w, osig, oq)
    plan.free()
    idx.free()


# ---------------------------------------------------------------------------
# Serving loop
# ---------------------------------------------------------------------------
def test_server_results_same_alone_and_in_the_mix(bovw):
    print("[case] server alone vs mix", flush=True)
    w, p, idx, sig, qc, osig, oq = bovw
    srv = H.Server(idx, p, T=w.T, eps=w.eps, slots=3, max_batch_queries=64, max_batch_ids=200_000,
                   max_batch_results=1 << 15)
    rows = list(range(0, 300, 3)) + [300, 301, 302, 303, 304]
    sub = _batch(qc, rows)
    want = _oracle_lists(w, osig, oq[rows])
    # alone: one request in flight at a time
    alone = []
    for j in range(sub.n):
        t = srv.submit(sub.set(j))
        alone.append(srv.wait(t).tolist())
    st = srv.stats()
    assert st["completed"] == sub.n and st["mean_batch_queries"] == 1.0
    # in the mix: all requests arrive within a few hundred microseconds
    srv.reset_stats()
    arrivals = np.sort(np.random.default_rng(1).uniform(0, 3e-4, size=sub.n))
    ro, ri = srv.replay(sub.ids, sub.offsets, arrivals, keep_results=True)
    mix = [ri[ro[j]:ro[j + 1]].tolist() for j in range(sub.n)]
    st = srv.stats()
    assert st["completed"] == sub.n and st["mean_batch_queries"] > 1.0, st
    assert alone == want
    assert mix == want
    assert st["p99_ms"] >= st["p50_ms"] > 0
    srv.close()


def test_server_online_inserts_are_visible_and_exact():
    print("[case] server inserts", flush=True)
    w = W.hoph_bovw(n=8_000, n_q=20, seed=41, planted_frac=0.01)
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    sig = H.sketch_oph(p, ids, offs)
    idx = H.Index(p, sig, capacity=w.collection.n + 500)
    osig, oq = oracle_sketch(w, w.collection), oracle_sketch(w, w.queries)
    assert (to_u32(sig) == osig).all()
    srv = H.Server(idx, p, T=w.T, eps=w.eps, slots=2, max_batch_queries=32, max_batch_ids=100_000,
                   max_batch_results=1 << 14)
    # new near-duplicates of query 0
    Q0 = np.unique(w.queries.set(0))
    rng = np.random.default_rng(2)
    new_sets = [np.sort(np.concatenate([Q0[:-2], rng.integers(0, 1 << 20, size=2).astype(np.uint32)]))
                for _ in range(5)] + [rng.integers(0, 1 << 20, size=300).astype(np.uint32) for _ in range(40)]
    before = srv.wait(srv.submit(w.queries.set(0))).tolist()
    assert before == _oracle_lists(w, osig, oq[:1])[0]
    new = W.csr_from_lists(new_sets)
    srv.insert(new.ids, new.offsets)
    assert len(idx) == w.collection.n + len(new_sets)
    # the grown collection as the oracle sketches it
    osig2 = np.concatenate([osig, oracle_sketch(w, new)])
    after = srv.wait(srv.submit(w.queries.set(0))).tolist()
    added = [x for x in after if x >= w.collection.n]
    assert before == [x for x in after if x < w.collection.n]
    assert added == list(range(w.collection.n, w.collection.n + 5))
    assert after == _oracle_lists(w, osig2, oq[:1])[0]
    # the whole query batch against the grown index
    want = _oracle_lists(w, osig2, oq)
    ro, ri = srv.replay(w.queries.ids, w.queries.offsets, np.zeros(w.queries.n), keep_results=True)
    assert [ri[ro[j]:ro[j + 1]].tolist() for j in range(w.queries.n)] == want
    assert srv.stats()["inserted_sets"] == len(new_sets)
    # past the index capacity
    big = W.csr_from_lists([rng.integers(0, 1 << 20, size=50).astype(np.uint32) for _ in range(600)])
    with pytest.raises(H.HophError) as ei:
        srv.insert(big.ids, big.offsets)
    assert ei.value.status == H.HOPH_E_CAPACITY
    srv.close()
    idx.free()


def test_server_admission_by_memory(bovw):
    print("[case] server admission", flush=True)
    w, p, idx, sig, qc, osig, oq = bovw
    one = H.Server(idx, p, T=w.T, eps=w.eps, slots=4, max_batch_queries=16, max_batch_ids=20_000,
                   max_batch_results=4096, device_mem_budget=1)
    st = one.stats()
    assert st["slots"] == 1 and st["slot_bytes"] > 0
    # a query set larger than a batch is refused, the server keeps serving
    with pytest.raises(H.HophError) as ei:
        one.submit(np.arange(20_001, dtype=np.uint32))
    assert ei.value.status == H.HOPH_E_CAPACITY
    r = one.wait(one.submit(qc.set(0))).tolist()
    assert r == _oracle_lists(w, osig, oq[:1])[0]
    assert one.stats()["rejected"] == 1
    one.close()
    two = H.Server(idx, p, T=w.T, eps=w.eps, slots=4, max_batch_queries=16, max_batch_ids=20_000,
                   max_batch_results=4096, device_mem_budget=2 * st["slot_bytes"] + 1)
    assert two.stats()["slots"] == 2
    two.close()


def test_coarse_plan_report():
    """hoph_coarse_plan follows the last call on the index: nothing before any
    query and after an empty batch, the first-group code kernels for a
    first-group pass (the light one for a self-join with one plane word), the
    word pass with COARSE_WORDS, the plain OPH comparator's pass, and the
    same shape from hoph_scan_timing as from the query it times."""
    w = W.hoph_bovw(n=3_000, n_q=40, seed=71, planted_frac=0.05)
    p = params_of(w)
    ids, offs = dev_csr(w.collection)
    qids, qoffs = dev_csr(w.queries)
    idx = H.Index(p, H.sketch_oph(p, ids, offs))
    qsig = H.sketch_oph(p, qids, qoffs)
    assert idx.last_coarse_plan() == (0, "none", 0, 0)
    H.query_hoph(idx, qsig, T=w.T, eps=w.eps)
    depth, kernel, planes, tiles = idx.last_coarse_plan()
    assert depth == 1 and kernel in ("first_group", "first_group_light") and tiles >= 1, (depth, kernel)
    assert H.scan_timing(idx, qsig, T=w.T, eps=w.eps, reps=2) > 0
    assert idx.last_coarse_plan() == (depth, kernel, planes, tiles)
    H.query_hoph(idx, qsig, T=w.T, eps=w.eps, coarse=H.COARSE_WORDS)
    assert idx.last_coarse_plan()[1] == "words"
    H.query_oph_full(idx, qsig, T=w.T)
    assert idx.last_coarse_plan()[:2] == (0, "oph_full")
    H.self_join(idx, T=w.T, eps=w.eps)
    depth, kernel, planes, tiles = idx.last_coarse_plan()
    assert depth == 1 and (kernel == "first_group_light" or (kernel == "first_group" and planes == 0)), kernel
    H.query_hoph(idx, qsig[:0], T=w.T, eps=w.eps)
    assert idx.last_coarse_plan() == (0, "none", 0, 0)
    idx.free()
