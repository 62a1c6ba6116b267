"""Exact, slow reference for one-permutation hashing (OPH), grouped OPH (GOPH)
and (a:b) hierarchical OPH (HOPH), after Zhang, Lin, Zhu, Yuan, Long and Huang,
"Hierarchical One Permutation Hashing: Efficient Multimedia Near Duplicate
Detection" (arXiv 1805.11254).

TEST INFRASTRUCTURE ONLY.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of bench.py may import this module.  The GPU library never
imports, links or calls anything under ``oracle/``, and this module imports
nothing from the library.

Everything here is plain Python integers and ``fractions.Fraction``: every
probability, weight, rate and decision is exact.  Loops are written in the
order the paper describes the method, for small inputs only.

Conventions fixed where the paper is silent, ambiguous or garbled (each is
listed with its reason in the design notes of the repository):

* ids live in [0, D); the permutation is a bijection table or a universal hash
  (a*x + b) mod p with p prime and p >= D (Sec. 3.2 asks for one random
  permutation psi; a hash mod a prime is injective on [0, D)).
* OPH bins (Sec. 3.2): the permuted range [0, R) is cut into k contiguous bins,
  bin b = floor(v*k/R); a bin keeps the minimum of its values, re-indexed to the
  offset from the bin start ("smallest possible representation"); an empty bin
  is EMPTY = 0xFFFFFFFF.
* HOPH regions (Sec. 4.1): the range is split a:b, the first part is a
  "permutation group" of k' equal bins, the second part is split again; split
  sizes are floors; L = k/k' groups; every split must leave both parts larger
  than k' (the paper's stop rule).
* per-group counts (Eqs. 1-4): m = bins equal and non-empty; e depends on the
  empty-bin policy: JOINT (both empty, Eq. 4), EITHER (either empty, the
  reading that reproduces the worked examples' 0.333 and 0.375) or LITERAL
  (no empty correction, Alg. 1/2 as printed).
* per-group rate (Eq. 6 / Lemma 3): m/(k'-e); 0/0 is 1 when every bin of the
  group is empty in both signatures, else 0; LITERAL uses m/k'.
* weights: GOPH 1/L each; HOPH w_j = r(1-r)^(j-1) for j < L and (1-r)^(L-1)
  for the last group, r = a/(a+b) (the fraction of the range each group covers).
* decision (Alg. 1/2, Def. 1, Ex. 1/2): after group l, S = sum w_j r_j,
  U = sum w_j, P_r = (T - S)/(1 - U), x = k' P_r, X ~ Bin(k', T).
  If P_r < T and P(X < x) <= eps: accept.  If P_r >= T and P(X >= x) <= eps:
  reject.  After the last group: accept iff S >= T.
"""
from __future__ import annotations

from bisect import bisect_right
from fractions import Fraction
from functools import lru_cache
from math import comb
from typing import Iterable, List, Optional, Sequence, Tuple

EMPTY = 0xFFFFFFFF
P31 = (1 << 31) - 1          # Mersenne prime 2^31 - 1
P32P15 = (1 << 32) + 15      # smallest prime above 2^32

HASH_TABLE, HASH_MODP31, HASH_MODP32P15 = 0, 1, 2
LAYOUT_OPH, LAYOUT_HIER = 0, 1
EMPTY_JOINT, EMPTY_LITERAL, EMPTY_EITHER = 0, 1, 2

ACCEPT, REJECT = True, False


# --------------------------------------------------------------------------
# Permutation (Sec. 3.2: one random permutation psi of the vocabulary)
# --------------------------------------------------------------------------
def hash_range(kind: int, universe: int) -> int:
    """Size R of the permuted range."""
    if kind == HASH_TABLE:
        return universe
    if kind == HASH_MODP31:
        return P31
    if kind == HASH_MODP32P15:
        return P32P15
    raise ValueError("unknown hash kind")


def permute(x: int, kind: int, perm: Optional[Sequence[int]] = None,
            ha: int = 0, hb: int = 0) -> int:
    """psi(x): a table lookup, or (a*x + b) mod p."""
    if kind == HASH_TABLE:
        return int(perm[x])
    p = P31 if kind == HASH_MODP31 else P32P15
    return (ha * x + hb) % p


# --------------------------------------------------------------------------
# Bin layout (Sec. 3.2 for OPH, Sec. 4.1 for (a:b) HOPH)
# --------------------------------------------------------------------------
class Layout:
    """The k contiguous bins that cut [0, R), and the L groups of k' bins."""

    def __init__(self, layout: int, R: int, k: int, kp: int,
                 ra: int = 1, rb: int = 1):
        if k <= 0 or kp <= 0 or k % kp:
            raise ValueError("k must be a positive multiple of k'")
        self.layout, self.R, self.k, self.kp = layout, R, k, kp
        self.L = k // kp
        self.ra, self.rb = ra, rb
        starts: List[int] = []
        if layout == LAYOUT_OPH:
            if k > R:
                raise ValueError("more bins than values")
            # bin b holds v with floor(v*k/R) == b, i.e. v >= ceil(b*R/k)
            starts = [-(-b * R // k) for b in range(k)]
            self.groups = [(starts[g * kp], starts[(g + 1) * kp] if g + 1 < self.L else R)
                           for g in range(self.L)]
        elif layout == LAYOUT_HIER:
            if ra <= 0 or rb <= 0:
                raise ValueError("a and b must be positive")
            regions = []
            lo = 0
            for _ in range(self.L - 1):
                size = (R - lo) * ra // (ra + rb)       # permutation group
                rest = R - lo - size                    # division group
                if size <= kp or rest <= kp:            # the paper's stop rule
                    raise ValueError("hierarchy deeper than the stop rule allows")
                regions.append((lo, lo + size))
                lo += size
            regions.append((lo, R))
            if R - lo < kp:
                raise ValueError("last group smaller than k'")
            self.groups = regions
            for (s, e) in regions:
                size = e - s
                starts += [s + (-(-t * size // kp)) for t in range(kp)]
        else:
            raise ValueError("unknown layout")
        self.starts = starts
        ends = starts[1:] + [R]
        if max(e - s for s, e in zip(starts, ends)) > EMPTY:
            raise ValueError("a bin is wider than 2^32-1 values")

    def bin_of(self, v: int) -> int:
        """The bin whose contiguous range holds v."""
        assert 0 <= v < self.R
        return bisect_right(self.starts, v) - 1

    def weights(self, goph: bool) -> List[Fraction]:
        """Group weights: 1/L for GOPH, the covered range fraction for HOPH."""
        if goph:
            return [Fraction(1, self.L)] * self.L
        r = Fraction(self.ra, self.ra + self.rb)
        w = [r * (1 - r) ** (j - 1) for j in range(1, self.L)]
        w.append((1 - r) ** (self.L - 1))
        return w


def sketch(elements: Iterable[int], lay: Layout, kind: int,
           perm: Optional[Sequence[int]] = None, ha: int = 0, hb: int = 0) -> List[int]:
    """OPH signature (Sec. 3.2 / Sec. 4.1): per bin, the smallest permuted
    value minus the bin start; EMPTY where the bin got nothing."""
    sig = [EMPTY] * lay.k
    for x in elements:
        v = permute(int(x), kind, perm, ha, hb)
        b = lay.bin_of(v)
        off = v - lay.starts[b]
        if off < sig[b]:
            sig[b] = off
    return sig


# --------------------------------------------------------------------------
# Matched and empty bins (Eqs. 1-4) and the per-group rate (Eq. 6, Lemma 3)
# --------------------------------------------------------------------------
def group_counts(q: Sequence[int], s: Sequence[int], policy: int) -> Tuple[int, int, bool]:
    """(m, e, all_joint_empty) over one group of bins."""
    m = sum(1 for a, b in zip(q, s) if a == b and a != EMPTY)
    joint = sum(1 for a, b in zip(q, s) if a == EMPTY and b == EMPTY)
    either = sum(1 for a, b in zip(q, s) if a == EMPTY or b == EMPTY)
    if policy == EMPTY_JOINT:
        e = joint
    elif policy == EMPTY_EITHER:
        e = either
    elif policy == EMPTY_LITERAL:
        e = 0
    else:
        raise ValueError("unknown empty policy")
    return m, e, joint == len(q)


def group_rate(m: int, e: int, nbins: int, all_joint_empty: bool, policy: int) -> Fraction:
    """Matched bins over non-empty bins; 0/0 is 1 when the group is empty in
    both signatures, else 0; LITERAL divides by every bin."""
    if policy == EMPTY_LITERAL:
        return Fraction(m, nbins)
    if nbins - e == 0:
        return Fraction(1) if all_joint_empty else Fraction(0)
    return Fraction(m, nbins - e)


def oph_estimate(q: Sequence[int], s: Sequence[int], policy: int = EMPTY_JOINT) -> Fraction:
    """Eq. 6 over every bin of two signatures."""
    m, e, aj = group_counts(q, s, policy)
    return group_rate(m, e, len(q), aj, policy)


def hoph_estimate(q: Sequence[int], s: Sequence[int], lay: Layout, goph: bool,
                  policy: int = EMPTY_JOINT) -> Fraction:
    """Lemma 3: the weighted sum of per-group rates."""
    w = lay.weights(goph)
    total = Fraction(0)
    for j in range(lay.L):
        sl = slice(j * lay.kp, (j + 1) * lay.kp)
        m, e, aj = group_counts(q[sl], s[sl], policy)
        total += w[j] * group_rate(m, e, lay.kp, aj, policy)
    return total


def eq8_plugin(R, nonempty: int, g: Optional[int]) -> Fraction:
    """Eq. 8 with the expectation of 1/(k - N_eb) replaced by the observed
    1/nonempty (nonempty = k - N_eb > 0); g = |D1 u D2|, None for the limit of
    large g, R(1 - R)/nonempty.  Returns 0 for g <= 1."""
    R = Fraction(R)
    inv = Fraction(1, nonempty)
    if g is None:
        return R * (1 - R) * inv
    if g <= 1:
        return Fraction(0)
    return R * (1 - R) * (inv * (1 + Fraction(1, g - 1)) - Fraction(1, g - 1))


def pair_report(q: Sequence[int], s: Sequence[int], lay: Layout, goph: bool, policy: int = EMPTY_JOINT,
                g: Optional[int] = None):
    """What is reported with an accepted pair: the whole-signature estimate
    (Lemma 3 for HOPH, the mean of group rates for GOPH), the matched and empty
    bins over all k bins (Eq. 1-4), and Eq. 8 with the observed 1/(k - N_eb)
    at R = the Eq. 6 estimate."""
    m, e, aj = group_counts(q, s, policy)
    k = len(q)
    R6 = group_rate(m, e, k, aj, policy)
    nonempty = k if policy == EMPTY_LITERAL else k - e
    var = eq8_plugin(R6, nonempty, g) if nonempty > 0 else Fraction(0)
    return hoph_estimate(q, s, lay, goph, policy), m, e, var


# --------------------------------------------------------------------------
# Binomial tails (Eq. 10, Table 2) and the small-probability event (Def. 1)
# --------------------------------------------------------------------------
def binom_pmf(n: int, p: Fraction, j: int) -> Fraction:
    return comb(n, j) * p ** j * (1 - p) ** (n - j)


def tail_below(n: int, p: Fraction, x) -> Fraction:
    """P(X < x) for X ~ Bin(n, p) and any real x (Table 2's F(x < X))."""
    return sum((binom_pmf(n, p, j) for j in range(n + 1) if j < x), Fraction(0))


def tail_at_or_above(n: int, p: Fraction, x) -> Fraction:
    """P(X >= x) for X ~ Bin(n, p) and any real x (Table 2's F(x >= X))."""
    return sum((binom_pmf(n, p, j) for j in range(n + 1) if j >= x), Fraction(0))


@lru_cache(maxsize=None)
def _below_at_ceil(n: int, p: Fraction, c: int) -> Fraction:
    return tail_below(n, p, c)


@lru_cache(maxsize=None)
def _above_at_ceil(n: int, p: Fraction, c: int) -> Fraction:
    return tail_at_or_above(n, p, c)


def _ceil(x: Fraction) -> int:
    return -((-x.numerator) // x.denominator)


def tail_integers(n: int, p: Fraction, eps: Fraction) -> Tuple[int, int]:
    """(j_lo, j_hi): j_lo = max{j >= -1 : P(X <= j) <= eps},
    j_hi = min{j <= n+1 : P(X >= j) <= eps}.  P(X < x) <= eps iff
    ceil(x) - 1 <= j_lo, and P(X >= x) <= eps iff ceil(x) >= j_hi."""
    j_lo = -1
    for j in range(0, n + 1):
        if tail_below(n, p, j + 1) <= eps:
            j_lo = j
    j_hi = n + 1
    for j in range(n, -1, -1):
        if tail_at_or_above(n, p, j) <= eps:
            j_hi = j
    return j_lo, j_hi


# --------------------------------------------------------------------------
# Sequential comparison (Alg. 1 for GOPH, Alg. 2 for (a:b) HOPH)
# --------------------------------------------------------------------------
def decide_trace(q: Sequence[int], s: Sequence[int], lay: Layout, goph: bool,
                 T: Fraction, eps: Fraction, policy: int = EMPTY_JOINT):
    """Walk the groups in order; return (decision, step, trace) where trace
    holds, per step, (m, e, S, P_r, x, tail) with tail the probability tested
    against eps (None at the last step)."""
    T, eps = Fraction(T), Fraction(eps)
    w = lay.weights(goph)
    kp = lay.kp
    S = Fraction(0)
    U = Fraction(0)
    trace = []
    for l in range(1, lay.L + 1):
        sl = slice((l - 1) * kp, l * kp)
        m, e, aj = group_counts(q[sl], s[sl], policy)
        S += w[l - 1] * group_rate(m, e, kp, aj, policy)
        U += w[l - 1]
        if l == lay.L:
            trace.append((m, e, S, None, None, None))
            return (S >= T), l, trace
        Pr = (T - S) / (1 - U)
        x = kp * Pr
        if Pr < T:
            # case i: the remaining groups need less than the average rate
            tail = _below_at_ceil(kp, T, _ceil(x))     # P(X < x)
            trace.append((m, e, S, Pr, x, tail))
            if tail <= eps:
                return ACCEPT, l, trace
        else:
            # case ii: they need at least the average rate
            tail = _above_at_ceil(kp, T, _ceil(x))     # P(X >= x)
            trace.append((m, e, S, Pr, x, tail))
            if tail <= eps:
                return REJECT, l, trace
    raise AssertionError("unreachable")


def decide(q, s, lay, goph, T, eps, policy=EMPTY_JOINT) -> Tuple[bool, int]:
    d, step, _ = decide_trace(q, s, lay, goph, T, eps, policy)
    return d, step


def oph_full_decide(q, s, T, policy=EMPTY_JOINT) -> bool:
    """Plain OPH comparator: Eq. 6 over all k bins, accept iff >= T."""
    return oph_estimate(q, s, policy) >= Fraction(T)


# --------------------------------------------------------------------------
# MinWise comparator (Sec. 1/2: k independent permutations, compare all k)
# --------------------------------------------------------------------------
def minwise_sketch(elements: Iterable[int], kind: int, coeffs: Sequence) -> List[int]:
    """k independent random permutations, each applied to every element; keep
    each permutation's minimum (2^64 - 1 for an empty set).  With kind
    HASH_TABLE, coeffs holds the k permutation tables of [0, D); otherwise the
    k pairs (a_i, b_i) of the hashes (a_i*x + b_i) mod p."""
    els = [int(x) for x in elements]
    out = []
    for c in coeffs:
        if kind == HASH_TABLE:
            vals = (permute(x, kind, c) for x in els)
        else:
            a, b = c
            vals = (permute(x, kind, None, a, b) for x in els)
        out.append(min(vals, default=(1 << 64) - 1))
    return out


def minwise_decide(q: Sequence[int], s: Sequence[int], T) -> bool:
    """Accept iff the fraction of equal minima reaches T."""
    eq = sum(1 for a, b in zip(q, s) if a == b)
    return Fraction(eq, len(q)) >= Fraction(T)


# --------------------------------------------------------------------------
# Ground truth (Sec. 3.1): Jaccard similarity
# --------------------------------------------------------------------------
def jaccard(a: Iterable[int], b: Iterable[int]) -> Fraction:
    A, B = set(int(x) for x in a), set(int(x) for x in b)
    if not A and not B:
        return Fraction(1)
    return Fraction(len(A & B), len(A | B))


def query_all(qsigs, ssigs, lay: Layout, goph: bool, T, eps, policy=EMPTY_JOINT):
    """For every query, the ascending ids of the accepted sets."""
    return [[i for i, s in enumerate(ssigs) if decide(q, s, lay, goph, T, eps, policy)[0]]
            for q in qsigs]
