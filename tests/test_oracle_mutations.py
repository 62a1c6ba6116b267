"""Plant plausible mistakes in the exact oracle (on the CPU) and check that at
least one pin fails for each: a pin set that let any of these through would
not be pinning the oracle to the paper."""
from fractions import Fraction

import pytest

from oracle import tiny
import tests.test_oracle_pins as P

PINS = [P.pin_oph_example, P.pin_hoph_example, P.pin_table2, P.pin_example1, P.pin_example2,
        P.pin_unbiased_and_variance, P.pin_invariants, P.pin_minwise_oracle, P.pin_goph_whole_estimate,
        P.pin_hoph_weights_are_range_fractions]


def _any_pin_fails():
    failed = []
    for pin in PINS:
        try:
            if pin is P.pin_unbiased_and_variance:
                pin(D=7, ks=(2, 4), pairs=[({0, 1, 2}, {2, 3, 4, 5}), ({0, 5}, {1, 5, 6})])
            else:
                pin()
        except Exception:
            failed.append(pin.__name__)
    return failed


def _orig(name):
    return getattr(tiny, name)


def mut_no_empty_correction(mp):
    f = _orig("group_counts")
    mp.setattr(tiny, "group_counts", lambda q, s, pol: (f(q, s, pol)[0], 0, f(q, s, pol)[2]))


def mut_uniform_hoph_weights(mp):
    mp.setattr(tiny.Layout, "weights", lambda self, goph: [Fraction(1, self.L)] * self.L)


def mut_lower_tail_inclusive(mp):
    mp.setattr(tiny, "tail_below", lambda n, p, x: sum((tiny.binom_pmf(n, p, j) for j in range(n + 1) if j <= x), Fraction(0)))
    tiny._below_at_ceil.cache_clear()


def mut_upper_tail_exclusive(mp):
    mp.setattr(tiny, "tail_at_or_above", lambda n, p, x: sum((tiny.binom_pmf(n, p, j) for j in range(n + 1) if j > x), Fraction(0)))
    tiny._above_at_ceil.cache_clear()


def mut_success_prob_flipped(mp):
    f = _orig("binom_pmf")
    mp.setattr(tiny, "binom_pmf", lambda n, p, j: f(n, 1 - p, j))
    tiny._below_at_ceil.cache_clear()
    tiny._above_at_ceil.cache_clear()


def mut_offset_from_group_start(mp):
    def sketch(elements, lay, kind, perm=None, ha=0, hb=0):
        sig = [tiny.EMPTY] * lay.k
        for x in elements:
            v = tiny.permute(int(x), kind, perm, ha, hb)
            b = lay.bin_of(v)
            off = v - lay.starts[(b // lay.kp) * lay.kp]
            sig[b] = min(sig[b], off)
        return sig
    mp.setattr(tiny, "sketch", sketch)


def mut_max_instead_of_min(mp):
    def sketch(elements, lay, kind, perm=None, ha=0, hb=0):
        sig = [None] * lay.k
        for x in elements:
            v = tiny.permute(int(x), kind, perm, ha, hb)
            b = lay.bin_of(v)
            off = v - lay.starts[b]
            sig[b] = off if sig[b] is None else max(sig[b], off)
        return [tiny.EMPTY if v is None else v for v in sig]
    mp.setattr(tiny, "sketch", sketch)


def mut_remaining_fraction_off_by_one(mp):
    """Alg. 1 read literally: the remaining-group divisor is one group short."""
    def decide_trace(q, s, lay, goph, T, eps, policy=tiny.EMPTY_JOINT):
        T, eps = Fraction(T), Fraction(eps)
        w = lay.weights(goph)
        kp = lay.kp
        S = Fraction(0)
        trace = []
        for l in range(1, lay.L + 1):
            sl = slice((l - 1) * kp, l * kp)
            m, e, aj = tiny.group_counts(q[sl], s[sl], policy)
            S += w[l - 1] * tiny.group_rate(m, e, kp, aj, policy)
            if l >= lay.L - 1:
                trace.append((m, e, S, None, None, None))
                return S >= T, l, trace
            U = sum(w[:l + 1])
            Pr = (T - S) / (1 - U)
            x = kp * Pr
            tail = tiny.tail_below(kp, T, x) if Pr < T else tiny.tail_at_or_above(kp, T, x)
            trace.append((m, e, S, Pr, x, tail))
            if tail <= eps:
                return (Pr < T), l, trace
    mp.setattr(tiny, "decide_trace", decide_trace)


def mut_cases_swapped(mp):
    def decide_trace(q, s, lay, goph, T, eps, policy=tiny.EMPTY_JOINT):
        T, eps = Fraction(T), Fraction(eps)
        w = lay.weights(goph)
        kp = lay.kp
        S = U = Fraction(0)
        trace = []
        for l in range(1, lay.L + 1):
            sl = slice((l - 1) * kp, l * kp)
            m, e, aj = tiny.group_counts(q[sl], s[sl], policy)
            S += w[l - 1] * tiny.group_rate(m, e, kp, aj, policy)
            U += w[l - 1]
            if l == lay.L:
                trace.append((m, e, S, None, None, None))
                return S >= T, l, trace
            Pr = (T - S) / (1 - U)
            x = kp * Pr
            tail = tiny.tail_at_or_above(kp, T, x) if Pr < T else tiny.tail_below(kp, T, x)
            trace.append((m, e, S, Pr, x, tail))
            if tail <= eps:
                return (Pr < T), l, trace
    mp.setattr(tiny, "decide_trace", decide_trace)


def mut_sign_of_remaining_rate(mp):
    def decide_trace(q, s, lay, goph, T, eps, policy=tiny.EMPTY_JOINT):
        T, eps = Fraction(T), Fraction(eps)
        w = lay.weights(goph)
        kp = lay.kp
        S = U = Fraction(0)
        trace = []
        for l in range(1, lay.L + 1):
            sl = slice((l - 1) * kp, l * kp)
            m, e, aj = tiny.group_counts(q[sl], s[sl], policy)
            S += w[l - 1] * tiny.group_rate(m, e, kp, aj, policy)
            U += w[l - 1]
            if l == lay.L:
                trace.append((m, e, S, None, None, None))
                return S >= T, l, trace
            Pr = (S - T) / (1 - U)
            x = kp * Pr
            tail = tiny.tail_below(kp, T, x) if Pr < T else tiny.tail_at_or_above(kp, T, x)
            trace.append((m, e, S, Pr, x, tail))
            if tail <= eps:
                return (Pr < T), l, trace
    mp.setattr(tiny, "decide_trace", decide_trace)


def mut_either_counts_joint_only(mp):
    f = _orig("group_counts")

    def gc(q, s, pol):
        if pol == tiny.EMPTY_EITHER:
            pol = tiny.EMPTY_JOINT
        return f(q, s, pol)
    mp.setattr(tiny, "group_counts", gc)


def mut_transposed_bin_formula(mp):
    """Bins numbered from the top of the range instead of the bottom."""
    orig_init = tiny.Layout.__init__

    def init(self, *a, **kw):
        orig_init(self, *a, **kw)
        self._rev = True
    mp.setattr(tiny.Layout, "__init__", init)
    orig_bin = tiny.Layout.bin_of
    mp.setattr(tiny.Layout, "bin_of", lambda self, v: orig_bin(self, self.R - 1 - v))


def mut_minwise_max(mp):
    def mw(elements, kind, coeffs):
        els = [int(x) for x in elements]
        return [max((tiny.permute(x, kind, c) if kind == tiny.HASH_TABLE else tiny.permute(x, kind, None, *c)
                     for x in els), default=(1 << 64) - 1) for c in coeffs]
    mp.setattr(tiny, "minwise_sketch", mw)


def mut_minwise_inverse_permutation(mp):
    f = _orig("minwise_sketch")

    def mw(elements, kind, coeffs):
        if kind != tiny.HASH_TABLE:
            return f(elements, kind, coeffs)
        inv = [tuple(sorted(range(len(c)), key=lambda x: c[x])) for c in coeffs]
        return f(elements, kind, inv)
    mp.setattr(tiny, "minwise_sketch", mw)


def mut_minwise_threshold_exclusive(mp):
    mp.setattr(tiny, "minwise_decide",
               lambda q, s, T: Fraction(sum(1 for a, b in zip(q, s) if a == b), len(q)) > Fraction(T))


def mut_hoph_weights_swapped_ratio(mp):
    """a:b read as b:a in the weights only (the layout still splits a:b)."""
    f = tiny.Layout.weights

    def weights(self, goph):
        if goph:
            return f(self, goph)
        self.ra, self.rb = self.rb, self.ra
        try:
            return f(self, goph)
        finally:
            self.ra, self.rb = self.rb, self.ra
    mp.setattr(tiny.Layout, "weights", weights)


def mut_goph_estimate_sum_of_rates(mp):
    f = _orig("hoph_estimate")

    def est(q, s, lay, goph, policy=tiny.EMPTY_JOINT):
        return f(q, s, lay, goph, policy) * (lay.L if goph else 1)
    mp.setattr(tiny, "hoph_estimate", est)


MUTATIONS = [mut_no_empty_correction, mut_uniform_hoph_weights, mut_lower_tail_inclusive,
             mut_upper_tail_exclusive, mut_success_prob_flipped, mut_offset_from_group_start,
             mut_max_instead_of_min, mut_remaining_fraction_off_by_one, mut_cases_swapped,
             mut_sign_of_remaining_rate, mut_either_counts_joint_only, mut_transposed_bin_formula,
             mut_minwise_max, mut_minwise_inverse_permutation, mut_minwise_threshold_exclusive,
             mut_goph_estimate_sum_of_rates, mut_hoph_weights_swapped_ratio]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=lambda m: m.__name__)
def test_pins_catch_mutation(mutation, monkeypatch):
    tiny._below_at_ceil.cache_clear()
    tiny._above_at_ceil.cache_clear()
    with monkeypatch.context() as mp:
        mutation(mp)
        failed = _any_pin_fails()
    tiny._below_at_ceil.cache_clear()
    tiny._above_at_ceil.cache_clear()
    assert failed, f"{mutation.__name__} passed every pin"


def test_unmutated_oracle_passes_every_pin():
    assert _any_pin_fails() == []
