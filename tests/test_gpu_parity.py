"""GPU parity: the HIP path against the oracle, element by element, on seeded
inputs of the paper's workload shapes (scaled so the oracle finishes in
seconds, spanning many 64-set tiles with a ragged tail), plus edge cases.
Everything is exact integer work, so the bar is bit-exact equality."""
from fractions import Fraction

import numpy as np
import pytest

import paper_1805_11254_amd as H
from oracle import scale, tiny
import workloads as W
from tests.hoph_testutil import (csr_lists, dev_csr, gpu_query, gpu_sketch, oracle_query, oracle_sketch, params_of,
                                 to_u32)

pytestmark = pytest.mark.gpu


def _print_case(name):
    print(f"[case] {name}", flush=True)


SMALL = {
    "goph_tiny": lambda: W.tiny_goph(),
    "hoph11_bovw": lambda: W.hoph_bovw(n=20_003, n_q=48, seed=11, planted_frac=0.02),
    "hoph12_shingles": lambda: W.hoph_shingles(n=12_345, n_q=40, seed=12, ra=1, rb=2, T=(7, 10)),
    "hoph21_shingles": lambda: W.hoph_shingles(n=9_999, n_q=33, seed=13, ra=2, rb=1, T=(1, 2)),
    "goph_bovw_512": lambda: _goph_bovw(),
}


def _goph_bovw():
    w = W.hoph_bovw(n=8_191, n_q=24, seed=14, planted_frac=0.03)
    w.layout = W.LAYOUT_OPH
    w.name = "goph_bovw_512"
    return w


_cache = {}


def workload(name):
    if name not in _cache:
        _cache[name] = SMALL[name]()
    return _cache[name]


@pytest.mark.parametrize("name", list(SMALL))
def test_sketch_bit_exact(name):
    _print_case(f"sketch {name}")
    w = workload(name)
    g = to_u32(gpu_sketch(w, w.collection))
    H.sync()
    o = oracle_sketch(w, w.collection)
    assert g.shape == o.shape
    bad = np.argwhere(g != o)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:5].tolist()}"
    gq = to_u32(gpu_sketch(w, w.queries))
    assert (gq == oracle_sketch(w, w.queries)).all()


@pytest.mark.parametrize("name", list(SMALL))
def test_pair_counts_match_oracle(name):
    import torch
    _print_case(f"pair_counts {name}")
    w = workload(name)
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    idx = H.Index(p, sig)
    rng = np.random.default_rng(3)
    pairs = [(q, s) for (q, s, _) in w.planted[:200]]
    pairs += [(int(rng.integers(w.queries.n)), int(rng.integers(w.collection.n))) for _ in range(300)]
    pairs += [(0, w.collection.n - 1), (w.queries.n - 1, 0)]
    P = torch.tensor(pairs, dtype=torch.int32, device="cuda")
    sh, qh = to_u32(sig), to_u32(qsig)
    for policy in (H.EMPTY_JOINT, H.EMPTY_EITHER, H.EMPTY_LITERAL):
        m, e = H.pair_counts(idx, qsig, P, policy)
        m, e = m.cpu().numpy(), e.cpu().numpy()
        for i, (q, s) in enumerate(pairs):
            om, oe = scale.pair_counts(qh[q], sh[s], w.kp, policy)
            assert m[i].tolist() == om.tolist() and e[i].tolist() == oe.tolist(), (policy, q, s)
    idx.free()


QUERY_GRID = [((4, 5), (1, 10_000)), ((1, 2), (1, 100)), ((9, 10), (0, 1)), ((7, 10), (1, 1000))]


@pytest.mark.parametrize("name", list(SMALL))
def test_query_candidates_bit_exact(name):
    _print_case(f"query {name}")
    w = workload(name)
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    idx = H.Index(p, sig)
    sh, qh = to_u32(sig), to_u32(qsig)
    kind = "goph" if w.goph else "hoph"
    for T, eps in QUERY_GRID:
        for policy in (H.EMPTY_JOINT, H.EMPTY_EITHER, H.EMPTY_LITERAL):
            oo, oi = oracle_query(w, sh, qh, T, eps, policy)
            for coarse in (H.COARSE_CODES, H.COARSE_WORDS):
                go, gi = gpu_query(kind, idx, qsig, T, eps, policy, coarse=coarse)
                assert go.tolist() == oo.tolist(), (T, eps, policy, coarse)
                assert gi.tolist() == oi.tolist(), (T, eps, policy, coarse)
    idx.free()


@pytest.mark.parametrize("name", ["goph_tiny", "hoph11_bovw", "goph_bovw_512"])
def test_results_do_not_depend_on_coarse_depth(name):
    _print_case(f"depth {name}")
    w = workload(name)
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    idx = H.Index(p, sig)
    kind = "goph" if w.goph else "hoph"
    for policy in (H.EMPTY_JOINT, H.EMPTY_EITHER):
        ref = None
        for coarse in (H.COARSE_CODES, H.COARSE_WORDS):
            for depth in (0, 1, 2, 3, 4):
                out = gpu_query(kind, idx, qsig, (4, 5), (1, 10_000), policy, coarse_depth=depth, coarse=coarse)
                cur = (out[0].tolist(), out[1].tolist())
                ref = cur if ref is None else ref
                assert cur == ref, (policy, coarse, depth)
    idx.free()


@pytest.mark.parametrize("ra,rb", [(1, 2), (2, 1), (1, 1)])
def test_multi_group_code_pass_matches_oracle(ra, rb):
    """The coarse pass over 2-4 groups of 32 bins on codes (its state bounded
    per group from the query's own empty count) at the library's depth and at
    depths 2, 3 and 4, for JOINT and LITERAL, at thresholds whose first reject
    cutoff comes at the first or a later group; collections of large sets and of
    sets of 20-60 ids (most bins empty), with planted near-duplicates."""
    _print_case(f"multi-group code pass {ra}:{rb}")
    big = W.hoph_shingles(n=6_007, n_q=24, seed=21 + ra, ra=ra, rb=rb)
    small = W.hoph_shingles(n=3_001, n_q=16, seed=31 + ra, ra=ra, rb=rb)
    small.collection = W.csr_from_lists([big.collection.set(i)[:20 + i % 41] for i in range(3_001)])
    small.queries = W.csr_from_lists([small.collection.set(i * 7) for i in range(16)])
    for w in (big, small):
        p = params_of(w)
        sig = gpu_sketch(w, w.collection, p)
        qsig = gpu_sketch(w, w.queries, p)
        idx = H.Index(p, sig)
        sh, qh = to_u32(sig), to_u32(qsig)
        found = 0
        for T in ((1, 2), (3, 5), (7, 10)):
            for policy in (H.EMPTY_JOINT, H.EMPTY_LITERAL):
                oo, oi = oracle_query(w, sh, qh, T, (1, 10_000), policy)
                found += len(oi)
                for depth in (0, 2, 3, 4):
                    go, gi = gpu_query("hoph", idx, qsig, T, (1, 10_000), policy, coarse_depth=depth)
                    assert go.tolist() == oo.tolist(), (T, policy, depth)
                    assert gi.tolist() == oi.tolist(), (T, policy, depth)
        assert found > 0
        idx.free()


@pytest.mark.parametrize("ra,rb,Ts", [(1, 2, [(63, 100), (67, 100), (71, 100), (73, 100), (81, 100), (87, 100)]),
                                      (2, 1, [(30, 100), (37, 100), (45, 100), (52, 100), (60, 100)]),
                                      (1, 1, [(51, 100), (46, 100)])])
def test_first_group_plane_splits_match_oracle(ra, rb, Ts):
    """The first-group code pass at thresholds whose reject cutoff on differing
    bins takes each first-phase plane count (2 to 6 planes before the rest of
    the chain; the kernel that keeps only those planes in registers), and the
    two-group pass, for JOINT and LITERAL, on large shingle sets with planted
    near-duplicates: results equal to the oracle's."""
    _print_case(f"first-group plane splits {ra}:{rb}")
    w = W.hoph_shingles(n=6_007, n_q=40, seed=41 + ra + 3 * rb, ra=ra, rb=rb)   # >= 32: both kernels
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    idx = H.Index(p, sig)
    sh, qh = to_u32(sig), to_u32(qsig)
    found, shapes = 0, set()
    for T in Ts:
        for policy in (H.EMPTY_JOINT, H.EMPTY_LITERAL):
            oo, oi = oracle_query(w, sh, qh, T, (1, 10_000), policy)
            found += len(oi)
            go, gi = gpu_query("hoph", idx, qsig, T, (1, 10_000), policy)
            assert go.tolist() == oo.tolist(), (T, policy)
            assert gi.tolist() == oi.tolist(), (T, policy)
            surv, acc = idx.last_query_counts()
            assert acc == len(oi) and surv >= acc, (T, policy, surv, acc)
            depth, kernel, planes, _ = idx.last_coarse_plan()
            shapes.add((depth, kernel, planes))
    assert len(shapes) >= 2, shapes      # the thresholds take different pass shapes
    assert found > 0
    idx.free()


@pytest.mark.parametrize("copies", [2_047, 2_048, 2_049, 4_100])
def test_output_stage_around_its_one_workgroup_limit(copies):
    """Batches whose accepted pairs fall just below, at and above the 2,048 keys
    the one-workgroup output stage sorts (above it the general stage runs):
    collections holding `copies` copies of two query sets among other sets, one
    and two queries per batch, CSR lists equal to the oracle's, through
    query_hoph and through a batched plan (eager and graph-captured); with too
    small a result capacity the call reports the count it needs."""
    _print_case(f"output stage, {copies} copies")
    rng = np.random.default_rng(copies)
    qa = np.sort(rng.choice(1 << 20, size=60, replace=False)).astype(np.uint32)
    qb = np.sort(rng.choice(1 << 20, size=90, replace=False)).astype(np.uint32)
    sets = []
    for i in range(copies):
        sets.append(qa if i % 2 == 0 else qb)
        if i % 3 == 0:
            sets.append(np.sort(rng.choice(1 << 20, size=int(rng.integers(20, 200)), replace=False)).astype(np.uint32))
    coll = W.csr_from_lists(sets)
    a, b = W.hash_coeffs(W.P31, 1, 77)
    for qsets in ([qa], [qa, qb]):
        qs = W.csr_from_lists(qsets)
        w = W.Workload("copies", coll, qs, 1 << 20, W.HASH_MODP31, W.LAYOUT_HIER, 256, 32, ha=int(a[0]), hb=int(b[0]))
        p = params_of(w)
        sig = gpu_sketch(w, coll, p)
        qsig = gpu_sketch(w, qs, p)
        idx = H.Index(p, sig)
        oo, oi = oracle_query(w, oracle_sketch(w, coll), oracle_sketch(w, qs), w.T, w.eps, H.EMPTY_JOINT)
        go, gi = gpu_query("hoph", idx, qsig, w.T, w.eps, H.EMPTY_JOINT)
        assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist(), (copies, len(qsets))
        assert len(oi) >= copies // 2
        with pytest.raises(H.HophError) as e:
            H.query_hoph(idx, qsig, T=w.T, eps=w.eps, capacity=len(oi) - 1)
        assert e.value.status == H.HOPH_E_CAPACITY and e.value.needed == len(oi)
        _, exact = H.query_hoph(idx, qsig, T=w.T, eps=w.eps, capacity=len(oi))
        assert exact.tolist() == oi.tolist()
        # a batched plan (eager and graph-captured): the same lists, and no batch
        # redone on the host path (the general stage follows within the plan)
        qi, qo = dev_csr(qs)
        for graph in (False, True):
            plan = H.Plan(idx, p, T=w.T, eps=w.eps, max_queries=4, max_query_ids=1_000, max_results=1 << 13,
                          use_graph=graph)
            for _ in range(2):
                plan.run(qi, qo)
                po, pi = plan.results()
                assert po.cpu().numpy().tolist() == oo.tolist() and to_u32(pi).tolist() == oi.tolist(), graph
            assert plan.info()["fallbacks"] == 0
            plan.free()
        idx.free()


def test_modp32_top_of_range_signatures():
    """Sets whose ids hash to the top of the (a x + b) mod (2^32 + 15) range
    (2^32 - 3 .. 2^32 + 14, the values the sketch's 32-bit view clamps): every
    signature against the oracle's, for plain OPH and the 1:1, 1:2 and 2:1
    hierarchies, in the host path and the chunked sketch of a plan."""
    _print_case("modp32 top of range")
    P = tiny.P32P15
    a, bb = 2_654_435_761, 97
    inv = pow(a, -1, P)
    top = [((v - bb) * inv) % P for v in range((1 << 32) - 3, P)]
    top = [x for x in top if x < (1 << 32)]
    assert any((a * x + bb) % P >= (1 << 32) for x in top)
    rng = np.random.default_rng(33)
    sets = []
    for i in range(300):
        s = rng.integers(0, 1 << 32, size=int(rng.integers(1, 400)), dtype=np.uint64)
        s = np.concatenate([s, np.array(top[: 1 + i % len(top)], dtype=np.uint64)]) if i % 3 else s
        sets.append(np.unique(s).astype(np.uint32))
    sets.append(np.array(top[:1], dtype=np.uint32))                  # a set of one top id
    coll = W.csr_from_lists(sets)
    for layout, ra, rb in [(W.LAYOUT_OPH, 1, 1), (W.LAYOUT_HIER, 1, 1), (W.LAYOUT_HIER, 1, 2), (W.LAYOUT_HIER, 2, 1)]:
        w = W.Workload("top", coll, coll, 1 << 32, W.HASH_MODP32P15, layout, 256, 32, ra=ra, rb=rb, ha=a, hb=bb)
        p = params_of(w)
        osig = oracle_sketch(w, coll)
        assert (to_u32(gpu_sketch(w, coll, p)) == osig).all(), (layout, ra, rb)
        if layout == W.LAYOUT_HIER:
            idx = H.Index(p, gpu_sketch(w, coll, p))
            plan = H.Plan(idx, p, max_queries=512, max_query_ids=200_000, max_results=1 << 16, use_graph=False)
            ids, offs = dev_csr(coll)
            plan.run(ids, offs)
            plan.results()
            assert (to_u32(plan.query_sigs(256)) == osig).all(), (ra, rb)
            plan.free()
            idx.free()


# The library's 8-bit bin code (a multiplicative mix scaled into 255 values,
# EMPTY apart), restated here only to build adversarial inputs: bins whose
# values differ from a query's but whose codes are equal.
def _code8(v):
    v = np.asarray(v, dtype=np.uint64)
    return np.where(v == tiny.EMPTY, 255, (((v * 0x9E3779B1) & 0xFFFFFFFF) * 255) >> 32).astype(np.uint64)


def _colliding_value(v, rng):
    """A value != v (and != EMPTY) with the same code as v."""
    target = int(_code8(v))
    while True:
        cand = rng.integers(0, 1 << 32, size=4096, dtype=np.uint64)
        hit = cand[(_code8(cand) == target) & (cand != v) & (cand != tiny.EMPTY)]
        if hit.size:
            return int(hit[0])


def _policies_that_fit(p, T, eps):
    """Empty policies whose exact tables fit 64 bits for these parameters
    (lcm(1..k') does not for k' above 42; LITERAL needs no lcm)."""
    out = []
    for policy in (H.EMPTY_JOINT, H.EMPTY_EITHER, H.EMPTY_LITERAL):
        try:
            H.decision_tables(p, T, eps, policy)
            out.append(policy)
        except H.HophError as e:
            assert e.status == H.HOPH_E_UNSUPPORTED
    assert H.EMPTY_LITERAL in out
    return out


@pytest.mark.parametrize("k,kp", [(512, 32), (320, 40), (512, 64)])
def test_code_collisions_match_oracle(k, kp):
    """Index sets whose bins carry a query's codes but not its values (in a
    fraction of the bins that would make the code count look like a near-
    duplicate): the coarse pass on codes cannot reject them, every such pair
    goes to the exact per-pair pass, and the result must equal the oracle's."""
    import torch
    _print_case(f"code collisions kp={kp}")
    w = W.hoph_bovw(n=6_000, n_q=12, seed=21, k=k, kp=kp, planted_frac=0.01)
    p = params_of(w)
    sig = to_u32(gpu_sketch(w, w.collection, p)).copy()
    qsig = to_u32(gpu_sketch(w, w.queries, p)).copy()
    rng = np.random.default_rng(22)
    table = {}
    for s_ in range(0, w.collection.n, 2):
        q = s_ % 4                      # queries 0..3 meet half of the collection this way
        frac = (0.55, 0.7, 0.85, 1.0)[q]
        for g in range(min(4, w.k // kp)):
            bins = np.arange(g * kp, (g + 1) * kp)
            chosen = bins[rng.random(kp) < frac]
            for b in chosen:
                v = int(qsig[q, b])
                if v == tiny.EMPTY:
                    continue
                key = (v, int(rng.integers(4)))
                if key not in table:
                    table[key] = _colliding_value(v, rng)
                sig[s_, b] = table[key]
    dsig = torch.from_numpy(sig.view(np.int32)).to("cuda")
    dq = torch.from_numpy(qsig.view(np.int32)).to("cuda")
    idx = H.Index(p, dsig)
    # T = 4/5, 7/10 and 1/2 take the code pass's three plane splits (2, 4, all 8 first)
    for T, eps in (((4, 5), (1, 10_000)), ((7, 10), (1, 10_000)), ((1, 2), (1, 100))):
        for policy in _policies_that_fit(p, T, eps):
            oo, oi = oracle_query(w, sig, qsig, T, eps, policy)
            for depth in (0, 1, 3):
                go, gi = gpu_query("hoph", idx, dq, T, eps, policy, coarse_depth=depth)
                assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist(), (T, eps, policy, depth)
    idx.free()


@pytest.mark.parametrize("layout,k,kp", [(W.LAYOUT_HIER, 128, 8), (W.LAYOUT_HIER, 192, 12), (W.LAYOUT_HIER, 320, 20),
                                         (W.LAYOUT_OPH, 120, 12), (W.LAYOUT_HIER, 320, 40), (W.LAYOUT_OPH, 448, 64),
                                         (W.LAYOUT_OPH, 160, 8), (W.LAYOUT_OPH, 160, 5)])
def test_group_sizes_match_oracle(layout, k, kp):
    """Group sizes other than 16 and 32: code planes of one or two words per
    plane, index stores through the word path, both coarse filters."""
    _print_case(f"group size layout={layout} k={k} kp={kp}")
    w = W.hoph_bovw(n=3_001, n_q=10, seed=23 + kp, k=k, kp=kp, planted_frac=0.02)
    w.layout = layout
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    sh, qh = to_u32(sig), to_u32(qsig)
    assert (sh == oracle_sketch(w, w.collection)).all()
    idx = H.Index(p, sig)
    kind = "goph" if w.goph else "hoph"
    for T, eps in (((4, 5), (1, 10_000)), ((1, 2), (1, 100))):
        for policy in _policies_that_fit(p, T, eps):
            oo, oi = oracle_query(w, sh, qh, T, eps, policy)
            for coarse in (H.COARSE_CODES, H.COARSE_WORDS):
                go, gi = gpu_query(kind, idx, qsig, T, eps, policy, coarse=coarse)
                assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist(), (T, eps, policy, coarse)
    idx.free()


def test_oph_full_comparator_bit_exact():
    _print_case("oph_full")
    for name in ("goph_tiny", "hoph11_bovw"):
        w = workload(name)
        p = params_of(w)
        sig = gpu_sketch(w, w.collection, p)
        qsig = gpu_sketch(w, w.queries, p)
        idx = H.Index(p, sig)
        sh, qh = to_u32(sig), to_u32(qsig)
        for T in ((1, 2), (4, 5)):
            for policy in (H.EMPTY_JOINT, H.EMPTY_EITHER, H.EMPTY_LITERAL):
                go, gi = H.query_oph_full(idx, qsig, T=T, policy=policy)
                oo, oi = scale.query_oph_full(sh, qh, T=Fraction(*T), policy=policy)
                assert go.cpu().numpy().tolist() == oo.tolist()
                assert to_u32(gi).tolist() == oi.tolist()
        idx.free()


def test_minwise_bit_exact():
    import torch
    _print_case("minwise")
    for kind, p in ((W.HASH_MODP31, W.P31), (W.HASH_MODP32P15, W.P32P15)):
        coll = W.zipf_sets(3_001, 1 << 20, 80, 0.5, 5, 400, seed=21)
        qs = W.zipf_sets(7, 1 << 20, 80, 0.5, 5, 400, seed=22)
        repl = {5: qs.set(0), 77: np.concatenate([qs.set(1)[:-3], np.array([5, 6, 7], dtype=np.uint32)])}
        coll = W.replace_sets(coll, repl)
        ha, hb = W.hash_coeffs(p, 200, 23)
        mp = H.MinwiseParams(200, kind, 1 << 20, torch.from_numpy(ha.view(np.int64)).cuda(),
                             torch.from_numpy(hb.view(np.int64)).cuda())
        ids, offs = dev_csr(coll)
        qids, qoffs = dev_csr(qs)
        g = H.minwise_sketch(mp, ids, offs)
        gq = H.minwise_sketch(mp, qids, qoffs)
        o = scale.minwise_sketch(coll.ids, coll.offsets, hash_kind=kind, universe=1 << 20, ha=ha, hb=hb)
        oq = scale.minwise_sketch(qs.ids, qs.offsets, hash_kind=kind, universe=1 << 20, ha=ha, hb=hb)
        assert (g.cpu().numpy().view(np.uint64) == o).all()
        assert (gq.cpu().numpy().view(np.uint64) == oq).all()
        for T in ((1, 2), (3, 10)):
            go, gi = H.minwise_query(mp, g, gq, T=T)
            oo, oi = scale.minwise_query(o, oq, T=Fraction(*T))
            assert go.cpu().numpy().tolist() == oo.tolist()
            assert to_u32(gi).tolist() == oi.tolist()


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------
def test_edge_tiny_and_degenerate_inputs():
    import torch
    _print_case("edges")
    D = 1 << 12
    perm = W.perm_table(D, 9)
    sets = [[5], [5], [0], [D - 1], list(range(0, D, 3)), list(range(D)), [7, 7, 7, 7], [1, 2, 3], [3, 2, 1]]
    coll = W.csr_from_lists(sets)
    for layout, k, kp in ((W.LAYOUT_OPH, 64, 16), (W.LAYOUT_HIER, 24, 8), (W.LAYOUT_OPH, 10, 5), (W.LAYOUT_HIER, 14, 2)):
        w = W.Workload("edge", coll, coll, D, W.HASH_TABLE, layout, k, kp, perm=perm)
        g = to_u32(gpu_sketch(w, coll))
        assert (g == oracle_sketch(w, coll)).all()
        p = params_of(w)
        sig = gpu_sketch(w, coll, p)
        idx = H.Index(p, sig, capacity=100)
        for T, eps in ((1, 1), (1, 10_000)), ((1, 2), (1, 10)), ((1, 10), (0, 1)):
            for policy in (0, 1, 2):
                go, gi = gpu_query("goph" if w.goph else "hoph", idx, sig, T, eps, policy)
                oo, oi = oracle_query(w, g, g, T, eps, policy)
                assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist()
        # no queries
        go, gi = gpu_query("goph" if w.goph else "hoph", idx, sig[:0], (4, 5), (1, 10_000), 0)
        assert go.tolist() == [0] and gi.size == 0
        idx.free()


def test_empty_index_and_append():
    import torch
    _print_case("append")
    w = workload("hoph11_bovw")
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    idx = H.Index(p, sig[:0], capacity=w.collection.n)
    go, gi = gpu_query("hoph", idx, qsig, (4, 5), (1, 10_000), 0)
    assert go.tolist() == [0] * (w.queries.n + 1) and gi.size == 0
    # append in ragged pieces
    cuts = [0, 1, 63, 64, 65, 1000, 7777, w.collection.n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        idx.append(sig[a:b].contiguous())
    assert len(idx) == w.collection.n
    with pytest.raises(H.HophError) as ei:
        idx.append(sig[:1].contiguous())
    assert ei.value.status == H.HOPH_E_CAPACITY
    go, gi = gpu_query("hoph", idx, qsig, (4, 5), (1, 10_000), 0)
    oo, oi = oracle_query(w, to_u32(sig), to_u32(qsig), (4, 5), (1, 10_000), 0)
    assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist()
    idx.free()


def test_results_capacity_reports_needed():
    _print_case("capacity")
    w = workload("goph_tiny")
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    idx = H.Index(p, sig)
    _, full = H.query_goph(idx, qsig, T=(1, 2), eps=(1, 10_000))
    need = full.numel()
    assert need > 2
    with pytest.raises(H.HophError) as ei:
        H.query_goph(idx, qsig, T=(1, 2), eps=(1, 10_000), capacity=need - 1)
    assert ei.value.status == H.HOPH_E_CAPACITY and ei.value.needed == need
    _, exact = H.query_goph(idx, qsig, T=(1, 2), eps=(1, 10_000), capacity=need)
    assert exact.numel() == need
    with pytest.raises(H.HophError) as ei:
        H.query_goph(idx, qsig, T=(1, 2), eps=(1, 10_000), coarse=7)
    assert ei.value.status == H.HOPH_E_INVAL
    idx.free()


@pytest.mark.parametrize("layout,k,kp,kind,depth", [(W.LAYOUT_HIER, 256, 32, "hoph", 1),
                                                     (W.LAYOUT_HIER, 256, 32, "hoph", 4),
                                                     (W.LAYOUT_OPH, 320, 10, "goph", 27),
                                                     (W.LAYOUT_HIER, 256, 32, "hoph", 0),
                                                     (W.LAYOUT_OPH, 320, 10, "goph", 0)])
def test_survivor_overflow_path_matches_oracle(layout, k, kp, kind, depth):
    """Near-identical collection: every pair survives the coarse pass, more
    survivors than the survivor buffer holds, so the batch is re-run in
    sub-batches; the result must still be exact.  The first-group pass, the
    register-resident pass over 4 groups and the LDS-staged deep pass (GOPH,
    27 groups of 10 bins in 9 code units) each append through their
    wavefront's batch; at the library's own depth (0) the overflowing batch
    is first re-run at the deepest depth, then split."""
    _print_case(f"survivor overflow layout={layout} k={k} kp={kp} depth={depth}")
    rng = np.random.default_rng(5)
    base = rng.choice(1 << 20, size=300, replace=False)
    sets = []
    for i in range(40_000):
        s = base.copy()
        s[rng.integers(0, 300, size=2)] = rng.integers(0, 1 << 20, size=2)
        sets.append(s)
    coll = W.csr_from_lists(sets)
    qs = W.csr_from_lists(sets[:30])
    w = W.Workload("same", coll, qs, 1 << 20, W.HASH_MODP31, layout, k, kp, ha=99991, hb=5)
    p = params_of(w)
    sig = gpu_sketch(w, coll, p)
    qsig = gpu_sketch(w, qs, p)
    idx = H.Index(p, sig)
    go, gi = gpu_query(kind, idx, qsig, (99, 100), (1, 10 ** 6), 0, coarse_depth=depth)
    oo, oi = oracle_query(w, to_u32(sig), to_u32(qsig), (99, 100), (1, 10 ** 6), 0)
    assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist()
    idx.free()


def test_device_error_flags():
    import torch
    _print_case("error flags")
    p = H.SketchParams(H.LAYOUT_OPH, 64, 16, H.HASH_MODP31, 1000, hash_a=7, hash_b=1)
    ids = torch.tensor([1, 2, 5000, 3], dtype=torch.int32, device="cuda")
    offs = torch.tensor([0, 2, 4], dtype=torch.int64, device="cuda")
    H.sync()
    H.sketch_oph(p, ids, offs)
    with pytest.raises(H.HophError) as ei:
        H.sync()
    assert ei.value.status == H.HOPH_E_RANGE
    H.sync()      # cleared
    offs2 = torch.tensor([0, 2, 2, 4], dtype=torch.int64, device="cuda")
    ids2 = torch.tensor([1, 2, 3, 4], dtype=torch.int32, device="cuda")
    out = H.sketch_oph(p, ids2, offs2)
    with pytest.raises(H.HophError) as ei:
        H.sync()
    assert ei.value.status == H.HOPH_E_INVAL
    assert (to_u32(out)[1] == tiny.EMPTY).all()


def _append_sets_check(w, cuts):
    import torch
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    two_step = H.Index(p, sig)
    fused = H.Index(p, sig[:0], capacity=w.collection.n)
    ids, offs = dev_csr(w.collection)
    offs_h = w.collection.offsets.astype(np.int64)
    for a, b in zip(cuts[:-1], cuts[1:]):
        lo = int(offs_h[a])
        piece_offs = torch.from_numpy((offs_h[a:b + 1] - lo).copy()).to("cuda")
        fused.append_sets(ids[lo:int(offs_h[b])].contiguous(), piece_offs)
    H.sync()
    assert len(fused) == w.collection.n
    sh, qh = to_u32(sig), to_u32(qsig)
    kind = "goph" if w.goph else "hoph"
    T, eps = (4, 5), (1, 10_000)
    policies = _policies_that_fit(p, T, eps)
    for policy in policies:
        oo, oi = oracle_query(w, sh, qh, T, eps, policy)
        for coarse in (H.COARSE_CODES, H.COARSE_WORDS):
            go, gi = gpu_query(kind, fused, qsig, T, eps, policy, coarse=coarse)
            assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist(), (policy, coarse)
    rng = np.random.default_rng(31)
    pairs = [(int(rng.integers(w.queries.n)), int(rng.integers(w.collection.n))) for _ in range(400)]
    pairs += [(0, 0), (w.queries.n - 1, w.collection.n - 1)]
    P = torch.tensor(pairs, dtype=torch.int32, device="cuda")
    for policy in policies:
        m1, e1 = H.pair_counts(two_step, qsig, P, policy)
        m2, e2 = H.pair_counts(fused, qsig, P, policy)
        assert torch.equal(m1, m2) and torch.equal(e1, e2), policy
    # the code planes written after sketching into the rows are the ones the
    # index store writes from given signatures, word for word
    n = w.collection.n
    ca, cb = two_step.code_planes(), fused.code_planes()
    assert ca.shape == cb.shape
    cu, tiles, _, pw = ca.shape
    ra, rb = ca.reshape(cu, tiles * 64, pw)[:, :n], cb.reshape(cu, tiles * 64, pw)[:, :n]
    assert torch.equal(ra, rb)
    two_step.free()
    fused.free()
    return sh, ra.cpu().numpy().view(np.uint32)


def _planes_from_rows(sh, kp, cu):
    """Code planes restated from signature rows: groups of k' <= 16 bins share a
    code unit, pk = min(32 // k', L) whole groups (else one group per unit);
    bit i of word p W + w of (row, unit u) is bit p of the code of bin 32 w + i
    of the unit."""
    n, k = sh.shape
    L = k // kp
    pk = min(32 // kp, L) if kp <= 16 else 1
    ub = pk * kp
    W_ = 1 if ub <= 32 else 2
    out = np.zeros((cu, n, 8 * W_), dtype=np.uint64)
    for u in range(cu):
        codes = _code8(sh[:, u * ub:(u + 1) * ub])               # n x ub
        for i in range(ub):
            for pl in range(8):
                out[u, :, pl * W_ + i // 32] |= ((codes[:, i] >> np.uint64(pl)) & np.uint64(1)) << np.uint64(i % 32)
    return out.astype(np.uint32)


@pytest.mark.parametrize("name", list(SMALL))
def test_append_sets_matches_oracle(name):
    """Sketching straight into the index (ragged appends that start and end
    inside tiles) gives the index that sketch_oph + index_append gives."""
    _print_case(f"append_sets {name}")
    w = workload(name)
    n = w.collection.n
    cuts = sorted(set([0, 1, 63, 64, 65, 130, n // 3, n // 3 + 7, n - 1, n]))
    _append_sets_check(w, cuts)


@pytest.mark.parametrize("layout,k,kp", [(W.LAYOUT_HIER, 192, 12), (W.LAYOUT_OPH, 120, 10), (W.LAYOUT_HIER, 320, 40),
                                         (W.LAYOUT_HIER, 320, 20), (W.LAYOUT_OPH, 320, 40), (W.LAYOUT_OPH, 160, 5),
                                         (W.LAYOUT_HIER, 512, 32), (W.LAYOUT_OPH, 512, 64), (W.LAYOUT_OPH, 270, 9),
                                         (W.LAYOUT_OPH, 24, 8), (W.LAYOUT_HIER, 256, 16)])
def test_append_sets_group_sizes(layout, k, kp):
    """Group sizes of one and two plane words, code units of several small
    groups (odd and even unit widths, a unit that spans the whole row), odd and
    even counts of units, every sketch lookup; the planes also against a
    restatement from the rows."""
    _print_case(f"append_sets group size layout={layout} k={k} kp={kp}")
    w = W.hoph_bovw(n=2_345, n_q=8, seed=41 + kp, k=k, kp=kp, planted_frac=0.02)
    w.layout = layout
    sh, planes = _append_sets_check(w, [0, 100, 1000, 2_345])
    cu = planes.shape[0]
    assert (planes == _planes_from_rows(sh, kp, cu)).all()


def test_append_sets_reports_range_and_empty_sets():
    import torch
    _print_case("append_sets errors")
    p = H.SketchParams(H.LAYOUT_OPH, 64, 16, H.HASH_MODP31, 1000, hash_a=7, hash_b=1)
    idx = H.Index(p, torch.empty((0, 64), dtype=torch.int32, device="cuda"), capacity=10)
    H.sync()
    idx.append_sets(torch.tensor([1, 2, 5000, 3], dtype=torch.int32, device="cuda"),
                    torch.tensor([0, 2, 4], dtype=torch.int64, device="cuda"))
    with pytest.raises(H.HophError) as ei:
        H.sync()
    assert ei.value.status == H.HOPH_E_RANGE
    H.sync()
    idx.append_sets(torch.tensor([1, 2], dtype=torch.int32, device="cuda"),
                    torch.tensor([0, 2, 2], dtype=torch.int64, device="cuda"))
    with pytest.raises(H.HophError) as ei:
        H.sync()
    assert ei.value.status == H.HOPH_E_INVAL
    with pytest.raises(H.HophError) as ei:
        idx.append_sets(torch.tensor([1] * 7, dtype=torch.int32, device="cuda"),
                        torch.arange(8, dtype=torch.int64, device="cuda"))
    assert ei.value.status == H.HOPH_E_CAPACITY
    idx.free()


@pytest.mark.parametrize("name", list(SMALL))
def test_pair_estimates_match_oracle(name):
    """Whole-signature estimate (Lemma 3 / group mean, exact), Eq. 6 counts and
    the Eq. 8 plug-in variance for accepted and random pairs."""
    import torch
    _print_case(f"pair_estimates {name}")
    w = workload(name)
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    idx = H.Index(p, sig)
    sh, qh = to_u32(sig), to_u32(qsig)
    kind = "goph" if w.goph else "hoph"
    lay = tiny.Layout(w.layout, tiny.hash_range(w.hash_kind, w.universe), w.k, w.kp, w.ra, w.rb)
    go, gi = H.query_goph(idx, qsig) if w.goph else H.query_hoph(idx, qsig)
    acc = H.result_pairs(go, gi)
    rng = np.random.default_rng(7)
    rnd = torch.tensor([(int(rng.integers(w.queries.n)), int(rng.integers(w.collection.n))) for _ in range(300)]
                       + [(w.queries.n, 0), (0, w.collection.n)], dtype=torch.int32, device="cuda")
    pairs = torch.cat([acc, rnd]).contiguous()
    ph = pairs.cpu().numpy()
    unions = torch.tensor([float(2 + (i % 5000)) for i in range(ph.shape[0])], dtype=torch.float64, device="cuda")
    for policy in _policies_that_fit(p, (4, 5), (1, 10_000)):
        for u in (None, unions):
            r = H.pair_estimates(idx, qsig, pairs, policy, unions=u)
            est, mb, eb, var = (r["est"].cpu().numpy(), r["mb"].cpu().numpy().view(np.uint32),
                                r["eb"].cpu().numpy().view(np.uint32), r["var"].cpu().numpy())
            den = r["denominator"]
            for i, (q, s) in enumerate(ph.tolist()):
                if q >= w.queries.n or s >= w.collection.n:
                    assert est[i] == -1 and mb[i] == 0xFFFFFFFF and np.isnan(var[i])
                    continue
                g = None if u is None else int(unions[i].item())
                R, m, e, v = tiny.pair_report(qh[q].tolist(), sh[s].tolist(), lay, w.goph, policy, g)
                assert Fraction(int(est[i]), den) == R, (policy, q, s)
                assert (int(mb[i]), int(eb[i])) == (m, e), (policy, q, s)
                assert abs(var[i] - float(v)) <= 1e-12 * max(1.0, abs(float(v))), (policy, q, s, var[i], float(v))
    idx.free()


def _with_queries_inside(w):
    """The workload's query sets placed in front of its collection, so that the
    planted near-duplicates are pairs inside one collection."""
    q, c = w.queries, w.collection
    ids = np.concatenate([q.ids, c.ids]).astype(np.uint32)
    offs = np.concatenate([q.offsets, c.offsets[1:] + q.offsets[-1]]).astype(np.uint64)
    return W.Collection(ids, offs)


SELF_JOIN = {
    "goph_tiny": lambda: W.tiny_goph(n=1500),
    "hoph11_bovw": lambda: W.hoph_bovw(n=3_000, n_q=40, seed=51, planted_frac=0.05),
    "hoph12_shingles": lambda: W.hoph_shingles(n=2_500, n_q=30, seed=52, ra=1, rb=2, T=(7, 10)),
}


@pytest.mark.parametrize("name", list(SELF_JOIN))
def test_self_join_matches_oracle(name):
    """Every accepted pair i < j inside the collection, as the oracle's full
    pair matrix restricted to j > i (the decision is symmetric)."""
    _print_case(f"self_join {name}")
    w = SELF_JOIN[name]()
    coll = _with_queries_inside(w)
    p = params_of(w)
    sig = gpu_sketch(w, coll, p)
    sh = to_u32(sig)
    idx = H.Index(p, sig)
    n = coll.n
    for T, eps in (((4, 5), (1, 10_000)), ((1, 2), (1, 100))):
        for policy in (H.EMPTY_JOINT, H.EMPTY_EITHER):
            oo, oi = oracle_query(w, sh, sh, T, eps, policy)
            want = [[j for j in row if j > i] for i, row in enumerate(csr_lists(oo, oi))]
            assert sum(len(r) for r in want) > 0
            for coarse in (H.COARSE_CODES, H.COARSE_WORDS):
                go, gi = H.self_join(idx, T=T, eps=eps, policy=policy, coarse=coarse)
                got = csr_lists(go.cpu().numpy(), to_u32(gi))
                assert len(got) == n and got == want, (T, eps, policy, coarse)
    idx.free()


@pytest.mark.parametrize("ra,rb,Ts", [(1, 2, [(63, 100), (71, 100), (81, 100), (87, 100)]),
                                      (2, 1, [(30, 100), (45, 100), (60, 100)]),
                                      (1, 1, [(4, 5), (51, 100)])])
def test_self_join_plane_splits_match_oracle(ra, rb, Ts):
    """The self-join's first-group pass at thresholds that take different
    first-phase plane counts and both first-group kernels (the upper-triangle
    item walk and the i < j filter of each), for JOINT and LITERAL, on shingle
    sets with planted near-duplicates: every accepted pair i < j equal to the
    oracle's."""
    _print_case(f"self-join plane splits {ra}:{rb}")
    w = W.hoph_shingles(n=1_777, n_q=24, seed=61 + ra + 3 * rb, ra=ra, rb=rb)
    coll = _with_queries_inside(w)
    p = params_of(w)
    sig = gpu_sketch(w, coll, p)
    sh = to_u32(sig)
    idx = H.Index(p, sig)
    found = 0
    for T in Ts:
        for policy in (H.EMPTY_JOINT, H.EMPTY_LITERAL):
            oo, oi = oracle_query(w, sh, sh, T, (1, 10_000), policy)
            want = [[j for j in row if j > i] for i, row in enumerate(csr_lists(oo, oi))]
            found += sum(len(r) for r in want)
            go, gi = H.self_join(idx, T=T, eps=(1, 10_000), policy=policy)
            got = csr_lists(go.cpu().numpy(), to_u32(gi))
            assert got == want, (T, policy)
            surv, acc = idx.last_query_counts()
            assert acc == sum(len(r) for r in want) and surv >= acc, (T, policy, surv, acc)
            depth, kernel, planes, tiles = idx.last_coarse_plan()
            if depth == 1:      # one plane word: the light kernel, else one phase over all planes
                assert kernel == "first_group_light" or (kernel == "first_group" and planes == 0), \
                    (T, policy, kernel, planes)
                if kernel == "first_group_light":
                    assert tiles == (16 if planes <= 3 else 8), (T, policy, planes, tiles)
    assert found > 0
    idx.free()


def _code_groups(kp, L, hier=False):
    """Groups that carry codes in the index and groups per code unit: units of
    pk = min(32 // k', L) whole groups when k' <= 16 (else 1); at least 4 units,
    about 128 bins for HOPH and 256 for GOPH, at most 24 units (12 when
    k' > 32), none past the row."""
    pk = min(32 // kp, L) if kp <= 16 else 1
    units = min(L // pk, max(4, min(12 if kp > 32 else 24, -(-(128 if hier else 256) // (pk * kp)))))
    return units * pk, pk


@pytest.mark.parametrize("k,kp", [(160, 8), (160, 5), (320, 10), (320, 20), (320, 40), (270, 9), (150, 3), (24, 8)])
def test_deep_code_pass_matches_oracle(k, kp):
    """GOPH with small groups: the coarse pass on codes at every depth from 1
    to the number of groups that carry codes, across the boundaries of code
    units (several small groups per unit) and of the register-resident units
    (past 4 units it stages a tile's planes in LDS), for queries and the
    self-join."""
    _print_case(f"deep code pass k={k} kp={kp}")
    w = W.hoph_bovw(n=2_500, n_q=12, seed=61 + kp, k=k, kp=kp, planted_frac=0.03, T=(7, 10))
    w.layout = W.LAYOUT_OPH
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    sh, qh = to_u32(sig), to_u32(qsig)
    idx = H.Index(p, sig)
    cg, pk = _code_groups(kp, k // kp)
    assert idx.code_planes().shape[0] * pk == cg
    depths = sorted(d for d in {1, 2, 3, 4, 5, pk, pk + 1, 4 * pk, 4 * pk + 1, cg // 2 + 1, cg} if 1 <= d <= cg)
    for T, eps in (((7, 10), (1, 10_000)), ((1, 2), (1, 1000))):
        for policy in _policies_that_fit(p, T, eps):
            oo, oi = oracle_query(w, sh, qh, T, eps, policy)
            for depth in depths:
                go, gi = gpu_query("goph", idx, qsig, T, eps, policy, coarse_depth=depth)
                assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist(), (T, eps, policy, depth)
    T, eps = (7, 10), (1, 10_000)
    oo, oi = oracle_query(w, sh, sh, T, eps, H.EMPTY_JOINT)
    want = [[j for j in row if j > i] for i, row in enumerate(csr_lists(oo, oi))]
    for depth in (0, cg):
        go, gi = H.self_join(idx, T=T, eps=eps, coarse_depth=depth)
        assert csr_lists(go.cpu().numpy(), to_u32(gi)) == want, depth
    # persistent plan kernels (eager and graph-replayed) on the same deep pass
    oo, oi = oracle_query(w, sh, qh, T, eps, H.EMPTY_JOINT)
    qids, qoffs = dev_csr(w.queries)
    for use_graph in (False, True):
        plan = H.Plan(idx, p, T=T, eps=eps, max_queries=16, max_query_ids=int(w.queries.ids.size) + 16,
                      max_results=1 << 16, use_graph=use_graph, tune=True)
        for rep in range(3):
            plan.run(qids, qoffs)
            po, pi = plan.results()
            assert po.cpu().numpy().tolist() == oo.tolist() and to_u32(pi).tolist() == oi.tolist(), (use_graph, rep)
        plan.free()
    idx.free()


@pytest.mark.parametrize("k,kp,ra,rb", [(256, 16, 1, 2), (256, 16, 2, 1), (128, 8, 1, 2), (96, 12, 2, 1)])
def test_hoph_ratios_with_code_units(k, kp, ra, rb):
    """HOPH with unequal weights (1:2, 2:1) and groups small enough to share
    plane words (code units of 2-4 groups): every depth across the unit
    boundaries and the library's own, for each empty policy whose tables fit,
    against the oracle; also the self-join."""
    _print_case(f"hoph ratios with code units k={k} kp={kp} {ra}:{rb}")
    w = W.hoph_bovw(n=2_000, n_q=10, seed=71 + kp + ra, k=k, kp=kp, planted_frac=0.03, T=(7, 10))
    w.layout, w.ra, w.rb = W.LAYOUT_HIER, ra, rb
    p = params_of(w)
    sig = gpu_sketch(w, w.collection, p)
    qsig = gpu_sketch(w, w.queries, p)
    sh, qh = to_u32(sig), to_u32(qsig)
    idx = H.Index(p, sig)
    cg, pk = _code_groups(kp, k // kp, hier=True)
    assert pk > 1 and idx.code_planes().shape[0] * pk == cg
    depths = sorted(d for d in {0, 1, 2, pk, pk + 1, cg} if 0 <= d <= cg)
    for T, eps in (((7, 10), (1, 10_000)), ((1, 2), (1, 1000))):
        for policy in _policies_that_fit(p, T, eps):
            oo, oi = oracle_query(w, sh, qh, T, eps, policy)
            for depth in depths:
                go, gi = gpu_query("hoph", idx, qsig, T, eps, policy, coarse_depth=depth)
                assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist(), (T, eps, policy, depth)
    T, eps = (7, 10), (1, 10_000)
    oo, oi = oracle_query(w, sh, sh, T, eps, H.EMPTY_LITERAL)
    want = [[j for j in row if j > i] for i, row in enumerate(csr_lists(oo, oi))]
    go, gi = H.self_join(idx, T=T, eps=eps, policy=H.EMPTY_LITERAL)
    assert csr_lists(go.cpu().numpy(), to_u32(gi)) == want
    idx.free()


def _default_depth(p, T, eps, kp, cg, pk):
    """The documented default coarse depth: the first group alone when it
    rejects at least 1/8 of its match counts, else one group past the first
    step with a reject cutoff, rounded up to whole code units, at most cg."""
    t = H.decision_tables(p, T, eps)
    unit0 = t["W"][0] * t["dmul"][0]
    m0 = t["rej"][0] // unit0 if t["rej"][0] >= 0 else -1
    if m0 >= 0 and 8 * m0 >= kp:
        return 1
    g1 = next((l + 1 for l, r in enumerate(t["rej"]) if r >= 0), None)
    return cg if g1 is None else min(cg, -(-(g1 + 1) // pk) * pk)


@pytest.mark.parametrize("layout,k,kp,ra,rb,T,want", [(W.LAYOUT_OPH, 320, 32, 1, 1, (7, 10), 4),
                                                      (W.LAYOUT_OPH, 320, 10, 1, 1, (7, 10), 12),
                                                      (W.LAYOUT_OPH, 320, 10, 1, 1, (1, 2), 18),
                                                      (W.LAYOUT_HIER, 512, 32, 1, 1, (4, 5), 1),
                                                      (W.LAYOUT_HIER, 256, 16, 1, 2, (1, 2), None)])
def test_default_coarse_depth(layout, k, kp, ra, rb, T, want):
    """The plan reports the depth the library picked when the caller leaves it
    open, which is the documented rule (worked values: GOPH k' = 32 at T = 0.7
    first rejects at group 3, so 4; k' = 10 at group 10, so 11, rounded up to
    the 3-group code unit: 12)."""
    _print_case(f"default depth layout={layout} k={k} kp={kp} {ra}:{rb} T={T}")
    w = W.hoph_bovw(n=500, n_q=4, seed=7, k=k, kp=kp)
    w.layout, w.ra, w.rb = layout, ra, rb
    p = params_of(w)
    idx = H.Index(p, gpu_sketch(w, w.collection, p))
    cg, pk = _code_groups(kp, k // kp, hier=layout == W.LAYOUT_HIER)
    expect = _default_depth(p, T, (1, 10_000), kp, cg, pk)
    if want is not None:
        assert expect == want
    plan = H.Plan(idx, p, T=T, eps=(1, 10_000), max_queries=8, max_query_ids=1 << 16, use_graph=False)
    assert plan.info()["depth"] == expect
    plan.free()
    idx.free()


@pytest.mark.parametrize("n_sets", [9_000, 20_000])
def test_queries_with_thousands_of_results_match_oracle(n_sets):
    """Near-identical collections: each query accepts thousands of sets, sorted
    in LDS per query up to 16384 ids, by the global sort beyond."""
    _print_case(f"big segments n={n_sets}")
    rng = np.random.default_rng(n_sets)
    base = rng.choice(1 << 20, size=200, replace=False)
    sets = []
    for _ in range(n_sets):
        s = base.copy()
        s[rng.integers(0, 200, size=3)] = rng.integers(0, 1 << 20, size=3)
        sets.append(s)
    coll = W.csr_from_lists(sets)
    w = W.Workload("same", coll, coll, 1 << 20, W.HASH_MODP31, W.LAYOUT_HIER, 256, 32, ha=1234567, hb=89)
    p = params_of(w)
    sig = gpu_sketch(w, coll, p)
    sh = to_u32(sig)
    idx = H.Index(p, sig)
    qsig = sig[[0, 1, n_sets - 1]].contiguous()
    qh = to_u32(qsig)
    oo, oi = oracle_query(w, sh, qh, w.T, w.eps, H.EMPTY_JOINT)
    assert max(np.diff(oo)) > (4096 if n_sets < 16384 else 16384)
    go, gi = gpu_query("hoph", idx, qsig, w.T, w.eps, H.EMPTY_JOINT)
    assert go.tolist() == oo.tolist() and gi.tolist() == oi.tolist()
    idx.free()
