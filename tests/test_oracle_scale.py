"""The C oracle (oracle/oph_oracle.c) against the exact Python oracle on small
random inputs: signatures, per-pair decisions and stop steps, the plain-OPH
and MinWise comparators; plus the seed-mean convergence of the estimator to
Jaccard under the universal hash family."""
import random
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import scale, tiny
import workloads as W


def _family(rng, D, n, base_size=40):
    """n sets around a few base sets, so that similarities spread over [0, 1]."""
    bases = [rng.sample(range(D), base_size) for _ in range(3)]
    sets = []
    for i in range(n):
        b = list(bases[i % 3])
        keep = rng.randint(base_size // 3, base_size)
        s = set(rng.sample(b, keep))
        s |= set(rng.randrange(D) for _ in range(rng.randint(0, base_size // 2)))
        sets.append(sorted(s))
    return sets


CASES = [
    # (hash kind, universe, layout, k, kp, a, b)
    (tiny.HASH_TABLE, 4096, tiny.LAYOUT_OPH, 32, 8, 1, 1),
    (tiny.HASH_TABLE, 1000, tiny.LAYOUT_HIER, 24, 4, 1, 1),
    (tiny.HASH_MODP31, 10 ** 6, tiny.LAYOUT_OPH, 64, 16, 1, 1),
    (tiny.HASH_MODP31, 1 << 20, tiny.LAYOUT_HIER, 64, 16, 1, 2),
    (tiny.HASH_MODP32P15, 1 << 32, tiny.LAYOUT_HIER, 64, 8, 2, 1),
    (tiny.HASH_MODP32P15, 1 << 32, tiny.LAYOUT_OPH, 96, 32, 1, 1),
]


@pytest.mark.parametrize("case", CASES)
def test_c_oracle_matches_python_oracle(case):
    kind, U, layout, k, kp, a, b = case
    rng = random.Random(hash(case) & 0xFFFF)
    D = min(U, 1 << 16) if kind == tiny.HASH_TABLE else U
    sets = _family(rng, min(D, 1 << 30), 30)
    qsets = _family(rng, min(D, 1 << 30), 4)
    perm = W.perm_table(D, 5) if kind == tiny.HASH_TABLE else None
    if kind == tiny.HASH_MODP31:
        ha, hb = rng.randrange(1, tiny.P31), rng.randrange(tiny.P31)
    elif kind == tiny.HASH_MODP32P15:
        ha, hb = rng.randrange(1, tiny.P32P15), rng.randrange(tiny.P32P15)
    else:
        ha = hb = 0
    lay = tiny.Layout(layout, tiny.hash_range(kind, D), k, kp, a, b)
    coll = W.csr_from_lists(sets)
    qcoll = W.csr_from_lists(qsets)
    kw = dict(hash_kind=kind, universe=D, layout=layout, k=k, kp=kp, ra=a, rb=b, ha=ha, hb=hb, perm=perm)
    sig_c = scale.sketch(coll.ids, coll.offsets, **kw)
    q_c = scale.sketch(qcoll.ids, qcoll.offsets, **kw)
    sig_p = [tiny.sketch(s, lay, kind, perm, ha, hb) for s in sets]
    q_p = [tiny.sketch(s, lay, kind, perm, ha, hb) for s in qsets]
    assert sig_c.tolist() == sig_p
    assert q_c.tolist() == q_p
    # bin starts agree
    assert scale.layout_starts(kind, D, layout, k, kp, a, b).tolist()[:-1] == lay.starts
    goph = layout == tiny.LAYOUT_OPH
    for policy in (tiny.EMPTY_JOINT, tiny.EMPTY_EITHER, tiny.EMPTY_LITERAL):
        for T, eps in [(F(1, 2), F(1, 10000)), (F(4, 5), F(1, 100)), (F(7, 10), F(0))]:
            offs, ids, steps, dd, ds = scale.query(sig_c, q_c, goph=goph, kp=kp, T=T, eps=eps,
                                                   policy=policy, ra=a, rb=b, dense=True)
            for qi, q in enumerate(q_p):
                for si, s in enumerate(sig_p):
                    d, st = tiny.decide(q, s, lay, goph, T, eps, policy)
                    assert dd[qi, si] == int(d) and ds[qi, si] == st, (qi, si, policy, T, eps)
            for qi in range(len(q_p)):
                acc = [si for si in range(len(sig_p)) if dd[qi, si]]
                assert ids[offs[qi]:offs[qi + 1]].tolist() == acc
        offs, ids = scale.query_oph_full(sig_c, q_c, T=F(3, 5), policy=policy)
        for qi, q in enumerate(q_p):
            acc = [si for si, s in enumerate(sig_p) if tiny.oph_full_decide(q, s, F(3, 5), policy)]
            assert ids[offs[qi]:offs[qi + 1]].tolist() == acc


def test_minwise_c_matches_python():
    rng = random.Random(3)
    sets = _family(rng, 1 << 20, 25)
    qsets = _family(rng, 1 << 20, 3)
    for kind, p in [(tiny.HASH_MODP31, tiny.P31), (tiny.HASH_MODP32P15, tiny.P32P15)]:
        ha, hb = W.hash_coeffs(p, 48, 9)
        coeffs = list(zip(ha.tolist(), hb.tolist()))
        coll, qcoll = W.csr_from_lists(sets), W.csr_from_lists(qsets)
        sc = scale.minwise_sketch(coll.ids, coll.offsets, hash_kind=kind, universe=1 << 20, ha=ha, hb=hb)
        qc = scale.minwise_sketch(qcoll.ids, qcoll.offsets, hash_kind=kind, universe=1 << 20, ha=ha, hb=hb)
        sp = [tiny.minwise_sketch(s, kind, coeffs) for s in sets]
        qp = [tiny.minwise_sketch(s, kind, coeffs) for s in qsets]
        assert sc.tolist() == sp and qc.tolist() == qp
        offs, ids = scale.minwise_query(sc, qc, T=F(1, 2))
        for qi, q in enumerate(qp):
            assert ids[offs[qi]:offs[qi + 1]].tolist() == [i for i, s in enumerate(sp) if tiny.minwise_decide(q, s, F(1, 2))]


def test_sketch_subset_and_errors():
    rng = random.Random(4)
    sets = _family(rng, 5000, 12)
    coll = W.csr_from_lists(sets)
    kw = dict(hash_kind=tiny.HASH_MODP31, universe=5000, layout=tiny.LAYOUT_OPH, k=16, kp=4, ha=12345, hb=777)
    full = scale.sketch(coll.ids, coll.offsets, **kw)
    sub = scale.sketch(coll.ids, coll.offsets, which=np.array([7, 2, 2]), **kw)
    assert (sub == full[[7, 2, 2]]).all()
    bad = coll.ids.copy()
    bad[3] = 5000
    with pytest.raises(scale.OracleError):
        scale.sketch(bad, coll.offsets, **kw)
    empty = W.csr_from_lists([[1, 2], [], [3]])
    with pytest.raises(scale.OracleError):
        scale.sketch(empty.ids, empty.offsets, **kw)
    e = scale.sketch(empty.ids, empty.offsets, allow_empty=True, **kw)
    assert (e[1] == tiny.EMPTY).all()


def test_seed_mean_converges_to_jaccard():
    """Eq. 7 under the universal hash family: the mean JOINT estimate over many
    (a, b) seeds lies within 4.5 standard errors of the exact Jaccard."""
    rng = random.Random(11)
    D = 1 << 20
    A = set(rng.sample(range(D), 300))
    common = rng.sample(sorted(A), 180)
    B = set(common) | set(rng.sample(range(D), 150))
    J = float(tiny.jaccard(A, B))
    coll = W.csr_from_lists([sorted(A), sorted(B)])
    ests = []
    ha, hb = W.hash_coeffs(tiny.P31, 1500, 21)
    for a, b in zip(ha.tolist(), hb.tolist()):
        s = scale.sketch(coll.ids, coll.offsets, hash_kind=tiny.HASH_MODP31, universe=D,
                         layout=tiny.LAYOUT_OPH, k=64, kp=64, ha=a, hb=b)
        m, e = scale.pair_counts(s[0], s[1], 64, tiny.EMPTY_JOINT)
        ests.append(m[0] / (64 - e[0]))
    ests = np.array(ests)
    se = ests.std(ddof=1) / np.sqrt(len(ests))
    assert abs(ests.mean() - J) < 4.5 * se, (ests.mean(), J, se)
