"""Pins of the exact oracle (oracle/tiny.py) to values fixed by the paper and by
mathematics: the printed worked examples, Table 2, Examples 1 and 2, the
exhaustive mean and variance of the OPH estimator (Eqs. 7-8), the MinWise
collision probability, and invariants.  The functions named ``pin_*`` are
also run against deliberately broken copies of the oracle in
test_oracle_mutations.py, to show that each plausible mistake fails a pin."""
import itertools
import random
import json
import os
from fractions import Fraction as F

import pytest

from oracle import tiny

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EX = json.load(open(os.path.join(GOLD, "worked_examples.json")))


def _none_to_empty(v):
    if isinstance(v, list):
        return [_none_to_empty(x) for x in v]
    return tiny.EMPTY if v is None else v


def _flat(v):
    return [x for g in v for x in g] if v and isinstance(v[0], list) else v


def _printed_close(value: float, printed: str) -> bool:
    """value agrees with the printed decimal to its last printed digit."""
    s = printed.lower()
    mant, _, exp = s.partition("e")
    digits = mant.replace("-", "").replace(".", "").lstrip("0")
    exp10 = int(exp) if exp else 0
    frac_digits = len(mant.split(".")[1]) if "." in mant else 0
    ulp = 10.0 ** (exp10 - frac_digits)
    return abs(value - float(printed)) <= 0.5 * ulp * (1 + 1e-9) or (digits == "1" and abs(value - 1) < 1e-9)


# ---------------------------------------------------------------------------
# Worked examples, Sec. 3.2 (OPH) and Sec. 4.1 (1:1 HOPH)
# ---------------------------------------------------------------------------
def pin_oph_example():
    ex = EX["oph"]
    lay = tiny.Layout(tiny.LAYOUT_OPH, EX["D"], ex["k"], ex["k"])
    ident = list(range(EX["D"]))
    sig = {n: tiny.sketch(s, lay, tiny.HASH_TABLE, ident) for n, s in EX["sets"].items()}
    for n in ("D1", "D2", "D3"):
        assert sig[n] == _none_to_empty(ex["representation"][n])
        samples = [tiny.EMPTY if v == tiny.EMPTY else v + lay.starts[b] for b, v in enumerate(sig[n])]
        assert samples == _none_to_empty(ex["samples"][n])
    for pol in (tiny.EMPTY_JOINT, tiny.EMPTY_EITHER, tiny.EMPTY_LITERAL):
        assert float(tiny.oph_estimate(sig["D1"], sig["D2"], pol)) == ex["estimate_D1_D2"]
    # 0.333 is reproduced when a bin empty in either signature is excluded
    assert round(float(tiny.oph_estimate(sig["D1"], sig["D3"], tiny.EMPTY_EITHER)), 3) == ex["estimate_D1_D3"]
    assert float(tiny.jaccard(EX["sets"]["D1"], EX["sets"]["D2"])) == ex["exact_D1_D2"]
    assert float(tiny.jaccard(EX["sets"]["D1"], EX["sets"]["D3"])) == ex["exact_D1_D3"]


def pin_hoph_example():
    ex = EX["hoph_1_1"]
    kp, L = ex["kp"], ex["groups"]
    lay = tiny.Layout(tiny.LAYOUT_HIER, EX["D"], kp * L, kp, 1, 1)
    ident = list(range(EX["D"]))
    sig = {n: tiny.sketch(s, lay, tiny.HASH_TABLE, ident) for n, s in EX["sets"].items()}
    for n in ("D1", "D2", "D3"):
        samples = [tiny.EMPTY if v == tiny.EMPTY else v + lay.starts[b] for b, v in enumerate(sig[n])]
        assert samples == _none_to_empty(_flat(ex["samples"][n]))
    for n in ("D1", "D2"):
        assert sig[n] == _none_to_empty(_flat(ex["representation"][n]))
    est = lambda a, b, pol: float(tiny.hoph_estimate(sig[a], sig[b], lay, False, pol))
    assert est("D1", "D2", tiny.EMPTY_JOINT) == ex["estimate_D1_D2"]
    assert est("D1", "D2", tiny.EMPTY_EITHER) == ex["estimate_D1_D2"]
    assert est("D1", "D3", tiny.EMPTY_EITHER) == ex["estimate_D1_D3"]
    # the paper's stop rule allows exactly three groups here
    with pytest.raises(ValueError):
        tiny.Layout(tiny.LAYOUT_HIER, EX["D"], kp * (L + 1), kp, 1, 1)


def test_oph_example():
    pin_oph_example()


def test_hoph_example():
    pin_hoph_example()


# ---------------------------------------------------------------------------
# Table 2 and Examples 1-2 (Sec. 3.3, Sec. 4.1)
# ---------------------------------------------------------------------------
def _table2():
    rows = []
    for line in open(os.path.join(GOLD, "table2_binomial_tails.txt")):
        if line.strip() and not line.startswith("#"):
            X, lt, ge = line.split()
            rows.append((int(X), lt, ge))
    return rows


def pin_table2():
    rows = _table2()
    assert len(rows) == 20
    for X, lt, ge in rows:
        assert _printed_close(float(tiny.tail_below(100, F(3, 5), X)), lt), (X, lt)
        assert _printed_close(float(tiny.tail_at_or_above(100, F(3, 5), X)), ge), (X, ge)


def _ex1_pair():
    ex = EX["example1_goph"]
    kp, n = ex["kp"], ex["n"]
    q = [0] * (kp * n)
    s = [1] * (kp * n)
    for g, mm in enumerate(ex["matches_per_group"]):
        for i in range(mm):
            s[g * kp + i] = 0
    return q, s, kp, n


def pin_example1():
    ex = EX["example1_goph"]
    q, s, kp, n = _ex1_pair()
    lay = tiny.Layout(tiny.LAYOUT_OPH, 10 ** 6, kp * n, kp)
    d, step, tr = tiny.decide_trace(q, s, lay, True, F(*ex["T"]), F(*ex["eps"]), tiny.EMPTY_LITERAL)
    assert d is tiny.REJECT and step == 4
    for (m, e, S, Pr, x, tail), printed in zip(tr, ex["M_ra_printed"]):
        # the printed M_ra values are truncated to the shown digits
        ndig = len(printed.split(".")[1]) if "." in printed else 0
        assert abs(float(x) - float(printed)) < 10.0 ** -ndig, (x, printed)
    assert _printed_close(float(tr[3][5]), "5.0732E-08")
    # M_a = k' T = 60: the first step is case i, the next three case ii
    assert tr[0][3] < F(3, 5) and all(t[3] >= F(3, 5) for t in tr[1:4])


def pin_example2():
    ex = EX["example2_hoph_1_1"]
    kp, n = ex["kp"], ex["n"]
    q = [0] * (kp * n)
    s = [1] * (kp * n)
    for i in range(ex["matches_group1"]):
        s[i] = 0
    lay = tiny.Layout(tiny.LAYOUT_HIER, 10 ** 9, kp * n, kp, 1, 1)
    d, step, tr = tiny.decide_trace(q, s, lay, False, F(*ex["T"]), F(*ex["eps"]), tiny.EMPTY_LITERAL)
    assert d is tiny.REJECT and step == ex["step"]
    assert tr[0][3] == F(4, 5) and tr[0][4] == 80
    assert _printed_close(float(tr[0][5]), "1.64119E-05")


def test_table2():
    pin_table2()


def test_example1():
    pin_example1()


def test_example2():
    pin_example2()


def test_tail_integers_match_scipy():
    """j_lo / j_hi against scipy's binomial cdf/sf where the float value is
    not within rounding of eps."""
    stats = pytest.importorskip("scipy.stats")
    for kp, T, eps in [(16, F(4, 5), F(1, 10000)), (32, F(4, 5), F(1, 10000)), (32, F(1, 2), F(1, 10000)),
                       (32, F(7, 10), F(1, 1000)), (32, F(9, 10), F(1, 100000)), (64, F(3, 5), F(1, 10000)),
                       (100, F(3, 5), F(1, 10000))]:
        j_lo, j_hi = tiny.tail_integers(kp, T, eps)
        lo = max([j for j in range(-1, kp + 1) if j < 0 or stats.binom.cdf(j, kp, float(T)) <= float(eps)])
        hi = min([j for j in range(0, kp + 2) if j > kp or stats.binom.sf(j - 1, kp, float(T)) <= float(eps)])
        assert (j_lo, j_hi) == (lo, hi)


# ---------------------------------------------------------------------------
# Eq. 7 (unbiasedness) and Eq. 8 (variance), exhaustively over all D! permutations
# ---------------------------------------------------------------------------
PAIRS_D8 = [({0, 1, 2, 3}, {2, 3, 4, 5, 6, 7}), ({0, 1, 5}, {1, 2, 3, 4, 6, 7}), ({0, 1, 2, 3, 4}, {2, 3, 4, 5, 6})]


def _exhaustive_estimates(A, B, D, k):
    lay = tiny.Layout(tiny.LAYOUT_OPH, D, k, k)
    out = []
    for perm in itertools.permutations(range(D)):
        qa = tiny.sketch(A, lay, tiny.HASH_TABLE, perm)
        qb = tiny.sketch(B, lay, tiny.HASH_TABLE, perm)
        m, e, aj = tiny.group_counts(qa, qb, tiny.EMPTY_JOINT)
        out.append((tiny.group_rate(m, e, k, aj, tiny.EMPTY_JOINT), e))
    return out


def pin_unbiased_and_variance(D=8, ks=(2, 4), pairs=PAIRS_D8):
    for A, B in pairs:
        J = tiny.jaccard(A, B)
        g = len(A | B)
        for k in ks:
            est = _exhaustive_estimates(A, B, D, k)
            n = len(est)
            mean = sum(r for r, _ in est) / n
            assert mean == J, (A, B, k, mean, J)                       # Eq. 7
            var = sum((r - J) ** 2 for r, _ in est) / n
            e_inv = sum(F(1, k - e) for _, e in est) / n
            formula = J * (1 - J) * (e_inv * (1 + F(1, g - 1)) - F(1, g - 1))
            assert var == formula, (A, B, k, var, formula)              # Eq. 8


def test_eq7_eq8_exhaustive():
    pin_unbiased_and_variance()


def pin_minwise_collision(D=7):
    """Over every permutation, min psi(A) == min psi(B) with probability J."""
    for A, B in [({0, 1, 2}, {1, 2, 3, 4}), ({0, 6}, {1, 2, 6}), ({3}, {3})]:
        hits = tot = 0
        for perm in itertools.permutations(range(D)):
            hits += min(perm[x] for x in A) == min(perm[x] for x in B)
            tot += 1
        assert F(hits, tot) == tiny.jaccard(A, B)


def test_minwise_collision_exhaustive():
    pin_minwise_collision()


MINWISE_PAIRS_D7 = [({0, 1, 2}, {1, 2, 3, 4}), ({0, 6}, {1, 2, 6}), ({3}, {3}), ({0, 1}, {5, 6})]


def pin_minwise_oracle(D=7, pairs=MINWISE_PAIRS_D7):
    """The oracle's MinWise comparator (Sec. 1-2), with all D! permutations of
    [0, D) as its k = D! independent permutations: the fraction of equal
    minima is exactly J (the min-wise collision probability), the decision is
    accept iff that fraction reaches T, and a single known permutation gives
    the smallest permuted element."""
    perms = list(itertools.permutations(range(D)))
    ident = tuple(range(D))
    rev = tuple(range(D - 1, -1, -1))
    shift = tuple((x + 1) % D for x in range(D))        # not its own inverse
    for A, B in pairs:
        J = tiny.jaccard(A, B)
        qa = tiny.minwise_sketch(sorted(A), tiny.HASH_TABLE, perms)
        qb = tiny.minwise_sketch(sorted(B), tiny.HASH_TABLE, perms)
        assert len(qa) == len(perms)
        eq = sum(1 for a, b in zip(qa, qb) if a == b)
        assert F(eq, len(perms)) == J, (A, B)
        assert tiny.minwise_decide(qa, qb, J)                       # inclusive at T = J
        if J < 1:
            assert not tiny.minwise_decide(qa, qb, J + F(1, 10 ** 6))
        if J > 0:
            assert tiny.minwise_decide(qa, qb, J - F(1, 10 ** 6))
        for S in (A, B):
            assert tiny.minwise_sketch(sorted(S), tiny.HASH_TABLE, [ident]) == [min(S)]
            assert tiny.minwise_sketch(sorted(S), tiny.HASH_TABLE, [rev]) == [D - 1 - max(S)]
            assert tiny.minwise_sketch(sorted(S), tiny.HASH_TABLE, [shift]) == [min((x + 1) % D for x in S)]
    assert tiny.minwise_sketch([], tiny.HASH_TABLE, [ident]) == [(1 << 64) - 1]


def test_minwise_oracle_exhaustive():
    pin_minwise_oracle()


def pin_goph_whole_estimate(seed=5, rounds=200):
    """The whole-signature estimate reported with a GOPH pair (the mean of its
    group rates) against what it reduces to: under LITERAL it is the matched
    bins over all k bins, Alg. 1's accumulated matches over n k'; under JOINT
    with no jointly empty bin it is Eq. 6 over all k bins; and over every
    permutation of a universe of D = k ids (each bin then holds exactly one id)
    its mean is J, as Eq. 7 states for one group."""
    rng = random.Random(seed)
    for _ in range(rounds):
        kp = rng.choice([1, 2, 3, 4, 8])
        L = rng.choice([1, 2, 3, 5])
        k = kp * L
        lay = tiny.Layout(tiny.LAYOUT_OPH, 1 << 12, k, kp)
        vals = [tiny.EMPTY, 0, 1, 2]
        q = [rng.choice(vals) for _ in range(k)]
        s = [rng.choice(vals) for _ in range(k)]
        m = sum(1 for a, b in zip(q, s) if a == b and a != tiny.EMPTY)
        est, mb, eb, _ = tiny.pair_report(q, s, lay, True, tiny.EMPTY_LITERAL)
        assert est == F(m, k) and mb == m and eb == 0
        s_full = [b if b != tiny.EMPTY or a != tiny.EMPTY else 3 for a, b in zip(q, s)]   # no joint empties
        m2 = sum(1 for a, b in zip(q, s_full) if a == b and a != tiny.EMPTY)
        est2, _, eb2, _ = tiny.pair_report(q, s_full, lay, True, tiny.EMPTY_JOINT)
        assert eb2 == 0 and est2 == F(m2, k) == tiny.oph_estimate(q, s_full, tiny.EMPTY_JOINT)
    D, kp = 6, 2
    lay = tiny.Layout(tiny.LAYOUT_OPH, D, D, kp)
    for A, B in [({0, 1, 2, 3}, {2, 3, 4, 5}), ({0, 1, 2, 3, 4, 5}, {0, 1, 2, 3, 4, 5}), ({0, 1, 2}, {3, 4, 5})]:
        assert A | B == set(range(D))
        tot = F(0)
        n = 0
        for perm in itertools.permutations(range(D)):
            qa = tiny.sketch(sorted(A), lay, tiny.HASH_TABLE, perm)
            qb = tiny.sketch(sorted(B), lay, tiny.HASH_TABLE, perm)
            tot += tiny.pair_report(qa, qb, lay, True, tiny.EMPTY_JOINT)[0]
            n += 1
        assert tot / n == tiny.jaccard(A, B)


def test_goph_whole_estimate():
    pin_goph_whole_estimate()


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
def _rand_layout(rng, R):
    if rng.random() < 0.5:
        kp = rng.choice([1, 2, 4, 8])
        L = rng.choice([1, 2, 4])
        return tiny.Layout(tiny.LAYOUT_OPH, R, kp * L, kp), True
    kp = rng.choice([2, 4])
    a, b = rng.choice([(1, 1), (1, 2), (2, 1)])
    for L in (4, 3, 2, 1):
        try:
            return tiny.Layout(tiny.LAYOUT_HIER, R, kp * L, kp, a, b), False
        except ValueError:
            continue
    raise AssertionError


def pin_invariants(seed=0, rounds=60):
    import random
    rng = random.Random(seed)
    for _ in range(rounds):
        D = rng.choice([64, 100, 257])
        perm = list(range(D))
        rng.shuffle(perm)
        lay, goph = _rand_layout(rng, D)
        A = rng.sample(range(D), rng.randint(1, 30))
        B = rng.sample(range(D), rng.randint(1, 30))
        sA = tiny.sketch(A, lay, tiny.HASH_TABLE, perm)
        sB = tiny.sketch(B, lay, tiny.HASH_TABLE, perm)
        T = F(rng.choice([1, 2, 3, 4, 7, 9]), 10)
        eps = F(1, rng.choice([10, 100, 10000]))
        # order and duplicates do not matter
        assert tiny.sketch(list(reversed(A)) + A[:3], lay, tiny.HASH_TABLE, perm) == sA
        # mergeability: sketch(A u B) is the elementwise min
        assert tiny.sketch(A + B, lay, tiny.HASH_TABLE, perm) == [min(x, y) for x, y in zip(sA, sB)]
        # identical sets: identical signatures, accepted for every T <= 1
        assert tiny.decide(sA, list(sA), lay, goph, T, eps)[0] is tiny.ACCEPT
        # disjoint sets: no non-empty matches
        C = [x for x in range(D) if x not in set(A)][:20]
        sC = tiny.sketch(C, lay, tiny.HASH_TABLE, perm)
        assert sum(1 for x, y in zip(sA, sC) if x == y != tiny.EMPTY) == 0
        # eps = 0: no early decision differs from the full weighted estimate
        full = tiny.hoph_estimate(sA, sB, lay, goph) >= T
        assert tiny.decide(sA, sB, lay, goph, T, F(0))[0] == full
        # one group: plain OPH
        one = tiny.Layout(tiny.LAYOUT_OPH, D, lay.k, lay.k)
        sA1 = tiny.sketch(A, one, tiny.HASH_TABLE, perm)
        sB1 = tiny.sketch(B, one, tiny.HASH_TABLE, perm)
        assert tiny.decide(sA1, sB1, one, True, T, eps)[0] == tiny.oph_full_decide(sA1, sB1, T)
        # monotone in matches: turning a mismatched non-empty bin into a match never
        # turns an accept into a reject
        d0 = tiny.decide(sA, sB, lay, goph, T, eps)[0]
        mism = [i for i, (x, y) in enumerate(zip(sA, sB)) if x != y and x != tiny.EMPTY and y != tiny.EMPTY]
        if mism and d0:
            sB2 = list(sB)
            sB2[mism[0]] = sA[mism[0]]
            assert tiny.decide(sA, sB2, lay, goph, T, eps)[0] is tiny.ACCEPT


def test_invariants():
    pin_invariants()


def test_weights_sum_to_one():
    for (a, b) in [(1, 1), (1, 2), (2, 1), (3, 5)]:
        lay = tiny.Layout(tiny.LAYOUT_HIER, 1 << 31, 32 * 6, 32, a, b)
        w = lay.weights(False)
        assert sum(w) == 1 and w[0] == F(a, a + b)
    assert tiny.Layout(tiny.LAYOUT_HIER, 16, 6, 2).weights(False) == [F(1, 2), F(1, 4), F(1, 4)]


def pin_hoph_weights_are_range_fractions():
    """Lemma 3 weights each group by the share of the permuted range it covers
    (r^j of the space; the a:b split of Sec. 4.1).  Where the recursive split
    is exact -- R a multiple of (a+b)^(L-1) -- the weights the oracle applies
    must equal each region's size over R, which the layout computes by a
    different route (repeated floor splits), for any a:b, not only 1:1.  Each
    region must also hold exactly k' bins of near-equal width, and with k' | a
    region the bins are equal (Sec. 4.1's k' equal-sized bins per group)."""
    for (a, b) in [(1, 1), (1, 2), (2, 1), (1, 3), (3, 1), (2, 3), (3, 5)]:
        for L in (2, 3, 4, 5):
            kp = 4
            R = (a + b) ** (L - 1) * kp * 11
            lay = tiny.Layout(tiny.LAYOUT_HIER, R, kp * L, kp, a, b)
            w = lay.weights(False)
            sizes = [e - s_ for (s_, e) in lay.groups]
            assert sum(sizes) == R
            assert w == [F(z, R) for z in sizes], (a, b, L)
            ends = lay.starts[1:] + [R]
            for j in range(L):
                widths = [ends[i] - lay.starts[i] for i in range(j * kp, (j + 1) * kp)]
                assert sum(widths) == sizes[j] and max(widths) - min(widths) <= 1
                if sizes[j] % kp == 0:
                    assert len(set(widths)) == 1
    # the GOPH weights are the equal shares of the n groups of an OPH layout
    lay = tiny.Layout(tiny.LAYOUT_OPH, 1 << 12, 32, 8)
    assert lay.weights(True) == [F(e - s_, lay.R) for (s_, e) in lay.groups]


def test_hoph_weights_are_range_fractions():
    pin_hoph_weights_are_range_fractions()


def _is_prime(n):
    if n < 2:
        return False
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1) or a % n == 0:
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_hash_moduli_are_prime():
    assert _is_prime(tiny.P31) and _is_prime(tiny.P32P15)
    assert all(not _is_prime((1 << 32) + d) for d in range(1, 15))


def test_layout_bins_partition_range():
    """Every value of a small range falls in exactly one bin and the bins are
    contiguous and ordered (both layouts)."""
    for lay in [tiny.Layout(tiny.LAYOUT_OPH, 1000, 24, 8), tiny.Layout(tiny.LAYOUT_HIER, 1000, 24, 8, 1, 2),
                tiny.Layout(tiny.LAYOUT_HIER, 997, 20, 4, 2, 1)]:
        ends = lay.starts[1:] + [lay.R]
        counts = [0] * lay.k
        for v in range(lay.R):
            b = lay.bin_of(v)
            assert lay.starts[b] <= v < ends[b]
            counts[b] += 1
        assert all(c > 0 for c in counts)
        for j, (s, e) in enumerate(lay.groups):
            assert lay.starts[j * lay.kp] == s


# ---------------------------------------------------------------------------
# Eq. 8 as reported per accepted pair (observed 1/(k - N_eb) for its expectation)
# ---------------------------------------------------------------------------
def pin_eq8_plugin():
    # where every bin always holds an element of the union (A u B = the whole
    # universe), N_eb = 0 for every permutation, so the observed 1/k is the
    # expectation and the plug-in must equal the exhaustive variance of Eq. 8
    D = 8
    for A, B in [({0, 1, 2, 3}, {2, 3, 4, 5, 6, 7}), ({0, 1, 2, 3, 4, 5}, {4, 5, 6, 7})]:
        assert A | B == set(range(D))
        J, g = tiny.jaccard(A, B), len(A | B)
        for k in (2, 4, 8):
            est = _exhaustive_estimates(A, B, D, k)
            assert all(e == 0 for _, e in est)
            var = sum((r - J) ** 2 for r, _ in est) / len(est)
            assert tiny.eq8_plugin(J, k, g) == var, (A, B, k)
    # the limit of large g is the binomial variance; no variance at R = 0 or 1
    for R, n in [(F(1, 3), 7), (F(5, 8), 32), (F(0), 5), (F(1), 9)]:
        assert tiny.eq8_plugin(R, n, None) == R * (1 - R) / n
        assert abs(float(tiny.eq8_plugin(R, n, 10 ** 12)) - float(R * (1 - R) / n)) < 1e-9
    assert tiny.eq8_plugin(F(0), 4, 10) == 0 and tiny.eq8_plugin(F(1), 4, 10) == 0


def test_eq8_plugin():
    pin_eq8_plugin()
