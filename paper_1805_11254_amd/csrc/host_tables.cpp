// Host side of libhoph: layout validation (Sec. 3.2, Sec. 4.1), the exact
// binomial tail integers (Eq. 10, Def. 1) and the integer cutoff tables that
// turn the sequential comparison of Alg. 1 / Alg. 2 into comparisons of an
// exact 64-bit state.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "hoph_internal.h"

namespace hoph {

typedef __int128 i128;
typedef unsigned __int128 u128;

// ---------------------------------------------------------------------------
// Layout
// ---------------------------------------------------------------------------
static uint64_t range_of(const hoph_sketch_params &p) {
    if (p.hash == HOPH_HASH_TABLE) return p.universe;
    if (p.hash == HOPH_HASH_MODP31) return kP31;
    return kP32;
}

void choose_estimate(LayoutInfo &lay);
void choose_pow2(LayoutInfo &lay);

// Whether the 32-bit narrow view of the permuted range (narrow_value,
// psi_p32_narrow) is exact for this layout: the range ends at or below 2^32 - 1,
// or (2^32 + 15) every region starts below kNarrowTop and the last bin at or
// below kNarrowLow, so every value the view moves lies in the last bin.
bool narrow_view_ok(const LayoutInfo &L) {
    if (L.R <= 0xFFFFFFFFull) return true;
    std::vector<uint64_t> starts;
    host_starts(L, starts);
    // the last bin holds every value psi_p32_narrow views at kNarrowLow or above
    if (starts.size() < 2 || starts[L.k - 1] > kNarrowLow) return false;
    for (uint32_t r = 0; r < L.n_regions; ++r)
        if (L.reg_start[r] >= kNarrowTop) return false;
    return true;
}

hoph_status build_layout(const hoph_sketch_params &p, LayoutInfo &out, std::string &err) {
    if (p.layout != HOPH_LAYOUT_OPH && p.layout != HOPH_LAYOUT_HIER) { err = "unknown layout"; return HOPH_E_INVAL; }
    if (p.k_group == 0 || p.k_group > HOPH_MAX_KGROUP) { err = "k_group must be in [1, 64]"; return HOPH_E_INVAL; }
    if (p.k == 0 || p.k % p.k_group) { err = "k must be a positive multiple of k_group"; return HOPH_E_INVAL; }
    if (p.k / p.k_group > HOPH_MAX_GROUPS) { err = "k / k_group must be <= 64"; return HOPH_E_INVAL; }
    if (p.universe == 0 || p.universe > (1ull << 32)) { err = "universe must be in [1, 2^32]"; return HOPH_E_INVAL; }
    switch (p.hash) {
    case HOPH_HASH_TABLE:
        if (!p.d_perm) { err = "HOPH_HASH_TABLE needs d_perm"; return HOPH_E_INVAL; }
        break;
    case HOPH_HASH_MODP31:
        if (p.universe > kP31) { err = "universe exceeds 2^31 - 1 for HOPH_HASH_MODP31"; return HOPH_E_INVAL; }
        if (p.hash_a == 0 || p.hash_a >= kP31 || p.hash_b >= kP31) { err = "hash coefficients out of range"; return HOPH_E_INVAL; }
        break;
    case HOPH_HASH_MODP32P15:
        if (p.hash_a == 0 || p.hash_a >= kP32 || p.hash_b >= kP32) { err = "hash coefficients out of range"; return HOPH_E_INVAL; }
        break;
    default:
        err = "unknown hash";
        return HOPH_E_INVAL;
    }
    const uint64_t R = range_of(p);
    LayoutInfo L;
    L.R = R;
    L.k = p.k;
    L.kp = p.k_group;
    L.L = p.k / p.k_group;
    L.ra = p.layout == HOPH_LAYOUT_HIER ? p.ratio_a : 1;
    L.rb = p.layout == HOPH_LAYOUT_HIER ? p.ratio_b : 1;
    std::vector<uint64_t> size;
    if (p.layout == HOPH_LAYOUT_OPH) {
        if ((uint64_t)p.k > R) { err = "more bins than permuted values"; return HOPH_E_INVAL; }
        L.n_regions = 1;
        L.nb = p.k;
        L.reg_start = {0, R};
        size = {R};
    } else {
        if (p.ratio_a == 0 || p.ratio_b == 0) { err = "ratio a:b needs a, b >= 1"; return HOPH_E_INVAL; }
        L.n_regions = L.L;
        L.nb = p.k_group;
        uint64_t lo = 0;
        L.reg_start.push_back(0);
        for (uint32_t g = 0; g + 1 < L.L; ++g) {
            uint64_t z = (uint64_t)((u128)(R - lo) * p.ratio_a / ((uint64_t)p.ratio_a + p.ratio_b));
            uint64_t rest = R - lo - z;
            if (z <= p.k_group || rest <= p.k_group) {
                err = "hierarchy deeper than the stop rule allows (a split leaves a part of at most k_group values)";
                return HOPH_E_INVAL;
            }
            size.push_back(z);
            lo += z;
            L.reg_start.push_back(lo);
        }
        if (R - lo < p.k_group) { err = "last group smaller than k_group"; return HOPH_E_INVAL; }
        size.push_back(R - lo);
        L.reg_start.push_back(R);
    }
    for (uint32_t r = 0; r < L.n_regions; ++r) {
        // widest bin of the region: ceil(z / nb)
        if ((size[r] + L.nb - 1) / L.nb > 0xFFFFFFFFull) { err = "a bin is wider than 2^32 - 1 values"; return HOPH_E_INVAL; }
        uint64_t M = (size[r] == L.nb) ? ~0ull : (uint64_t)(((u128)L.nb << 64) / size[r]);
        L.reg_magic.push_back(M);
        const uint64_t M32 = (uint64_t)(((u128)L.nb << 32) / size[r]);
        L.reg_mag32.push_back((uint32_t)std::min<uint64_t>(M32, 0xFFFFFFFFull));
    }
    uint32_t sh = 0;
    while (((R - 1) >> sh) >= kLutMax) ++sh;
    L.lut_shift = sh;
    L.lut_size = (uint32_t)((R - 1) >> sh) + 1;
    choose_estimate(L);
    // log-domain cells: a narrow range with regions, no cell holding two
    // boundaries; over 2^32 + 15 the narrow view (narrow_value) holds when every
    // region and the last bin start below kNarrowTop
    L.log_ok = 0;
    if (L.n_regions > 1 && narrow_view_ok(L)) {
        bool ok = true;
        const uint32_t R1 = narrow_r1(R);
        for (uint32_t r = 1; r + 1 < L.n_regions && ok; ++r)
            ok = log_cell((uint32_t)(L.reg_start[r] - 1), R1) != log_cell((uint32_t)L.reg_start[r + 1], R1);
        L.log_ok = ok ? 1u : 0u;
    }
    choose_pow2(L);
    if (p.hash == HOPH_HASH_MODP32P15 && !narrow_view_ok(L)) {
        // the sketch looks bins up in 32 bits, which needs the last bin to start at or below 2^32 - 15
        err = "a bin at the top of the range is narrower than the 32-bit lookup needs (layout too deep)";
        return HOPH_E_UNSUPPORTED;
    }
    out = std::move(L);
    return HOPH_OK;
}

// The uniform bin estimate: a 32-bit reciprocal of R / k such that, for the
// first and last value of every non-empty bin b, the estimate is b or b - 1
// (the estimate is monotone in v, so every value of the bin then is too).
void choose_estimate(LayoutInfo &lay) {
    lay.est_ok = 0;
    std::vector<uint64_t> starts;
    host_starts(lay, starts);
    const uint32_t sh = lay.R > (1ull << 32) ? 1u : 0u;        // v >> sh fits 32 bits for v < R
    const uint64_t Rs = (lay.R + (1ull << sh) - 1) >> sh;
    if (Rs <= lay.k) return;
    const uint64_t M0 = (uint64_t)(((u128)lay.k << 32) / Rs);
    for (uint64_t t = 0; t < 64 && t <= M0; ++t) {
        const uint32_t M = (uint32_t)(M0 - t);
        bool ok = true;
        for (uint32_t b = 0; b < lay.k && ok; ++b) {
            if (starts[b + 1] <= starts[b]) continue;                // empty bin: no value lands here
            const int64_t lo = bin_estimate(starts[b], M, sh), hi = bin_estimate(starts[b + 1] - 1, M, sh);
            ok = lo >= (int64_t)b - 1 && hi <= (int64_t)b;
        }
        if (ok) {
            lay.est_mul = M;
            lay.est_shift = sh;
            lay.est_ok = 1;
            return;
        }
    }
}

// The power-of-two lookup (see locate_pow2), for a narrow range: each region's
// bin starts must be t 2^s from the region start, and the values of each
// leading-zero class of u = max(R - 1 - v, 1) must lie in one region.
void choose_pow2(LayoutInfo &lay) {
    lay.pow2_ok = 0;
    lay.pow2.assign(4 * kPow2Classes, 0);
    if (lay.R < 2 || lay.R >= 0xFFFFFFFFull) return;
    const uint64_t nb = lay.nb;
    std::vector<uint32_t> shift(lay.n_regions);
    for (uint32_t r = 0; r < lay.n_regions; ++r) {
        const uint64_t s0 = lay.reg_start[r], z = lay.reg_start[r + 1] - s0;
        uint32_t sh = 0;
        while (sh < 31 && (nb << sh) < z) ++sh;                 // smallest s with nb 2^s >= z
        if ((nb << sh) < z) return;
        for (uint64_t t = 0; t < nb; ++t)
            if ((t * z + nb - 1) / nb != (t << sh)) return;     // bin t starts at t 2^s
        shift[r] = sh;
    }
    const uint64_t R1 = lay.R - 1;
    auto region_of = [&](uint64_t v) {
        uint32_t r = 0;
        while (r + 1 < lay.n_regions && v >= lay.reg_start[r + 1]) ++r;
        return r;
    };
    for (uint32_t lz = 0; lz < kPow2Classes; ++lz) {
        const uint64_t ulo = 1ull << (31 - lz), uhi = (1ull << (32 - lz)) - 1;
        if (ulo > R1) continue;                                 // no value has this class
        const uint64_t vlo = R1 - std::min(uhi, R1);
        const uint64_t vhi = ulo == 1 ? R1 : R1 - ulo;          // u = 1 also for v = R - 1
        const uint32_t r = region_of(vlo);
        if (region_of(vhi) != r) return;
        uint32_t *e = &lay.pow2[4 * lz];
        e[0] = (uint32_t)lay.reg_start[r];
        e[1] = shift[r];
        e[2] = (uint32_t)(r * nb);
        e[3] = (uint32_t)((1ull << shift[r]) - 1);
    }
    lay.pow2_ok = 1;
}

void fill_sketch_desc(const hoph_sketch_params &p, const LayoutInfo &lay, SketchDesc &d) {
    std::memset(&d, 0, sizeof(d));
    d.perm = p.d_perm;
    d.universe = p.universe;
    d.ha = p.hash_a;
    d.hb = p.hash_b;
    d.R = lay.R;
    d.hash = p.hash;
    d.k = lay.k;
    d.n_regions = lay.n_regions;
    d.lut_shift = lay.lut_shift;
    d.lut_size = lay.lut_size;
    d.nb = lay.nb;
    d.est_mul = lay.est_mul;
    d.est_shift = lay.est_shift;
    d.est_ok = lay.est_ok;
    d.log_ok = lay.log_ok;
    d.pow2_ok = lay.pow2_ok;
    for (uint32_t c = 0; c < kPow2Classes; ++c)
        for (int j = 0; j < 4; ++j) d.pow2[c][j] = lay.pow2[4 * c + j];
    for (uint32_t r = 0; r <= lay.n_regions; ++r) d.reg_start[r] = lay.reg_start[r];
    for (uint32_t r = 0; r < lay.n_regions; ++r) d.reg_magic[r] = lay.reg_magic[r];
    for (uint32_t r = 0; r < lay.n_regions; ++r) d.reg_mag32[r] = lay.reg_mag32[r];
}

void host_lut(const LayoutInfo &lay, std::vector<uint8_t> &lut) {
    lut.assign(lay.lut_size, 0);
    for (uint32_t g = 0; g < lay.lut_size; ++g) {
        uint64_t v = (uint64_t)g << lay.lut_shift;
        uint32_t r = 0;
        while (r + 1 < lay.n_regions && v >= lay.reg_start[r + 1]) ++r;
        lut[g] = (uint8_t)r;
    }
}

void host_starts(const LayoutInfo &lay, std::vector<uint64_t> &starts) {
    starts.assign((size_t)lay.k + 1, 0);
    for (uint32_t b = 0; b < lay.k; ++b) {
        uint32_t r = b / lay.nb, t = b % lay.nb;
        uint64_t z = lay.reg_start[r + 1] - lay.reg_start[r];
        starts[b] = lay.reg_start[r] + (uint64_t)(((u128)t * z + lay.nb - 1) / lay.nb);
    }
    starts[lay.k] = lay.R;
}

// ---------------------------------------------------------------------------
// Minimal unsigned big integers for exact binomial tails, in fixed storage (no
// heap use, so that table construction allocates nothing).
// ---------------------------------------------------------------------------
struct Big {
    // every value below fits: terms and sums are at most td^n * 2^41 and
    // td^n * ed <= 2^(32 n + 32) for n <= 256 binomial trials
    static constexpr uint32_t kLimbs = 264;
    uint32_t d[kLimbs];        // little-endian limbs; d[n..] are not kept
    uint32_t n = 0;            // limbs in use, no leading zeros
    bool overflow = false;
    static Big of(uint64_t v) {
        Big b;
        while (v) { b.d[b.n++] = (uint32_t)v; v >>= 32; }
        return b;
    }
    bool zero() const { return n == 0; }
    void trim() { while (n && d[n - 1] == 0) --n; }
    void add(const Big &o) {
        overflow |= o.overflow;
        const uint32_t m = n > o.n ? n : o.n;
        uint64_t c = 0;
        for (uint32_t i = 0; i < m; ++i) {
            const uint64_t s = (uint64_t)(i < n ? d[i] : 0) + (i < o.n ? o.d[i] : 0) + c;
            d[i] = (uint32_t)s;
            c = s >> 32;
        }
        n = m;
        if (c) {
            if (n == kLimbs) { overflow = true; return; }
            d[n++] = (uint32_t)c;
        }
    }
    // *this *= v (v < 2^64): two passes of 32-bit factors, every partial
    // product and carry within 64 bits
    void mul_small(uint64_t v) {
        if (v == 0 || n == 0) { n = 0; return; }
        uint32_t tmp[kLimbs + 2] = {};
        for (uint32_t pass = 0; pass < 2; ++pass) {
            const uint32_t f = (uint32_t)(v >> (32 * pass));
            if (!f) continue;
            uint64_t c = 0;
            for (uint32_t i = 0; i < n; ++i) {
                const uint64_t t = (uint64_t)d[i] * f + tmp[i + pass] + c;
                tmp[i + pass] = (uint32_t)t;
                c = t >> 32;
            }
            for (uint32_t k = n + pass; c; ++k) {      // k <= n + 1: the product has at most n + 2 limbs
                const uint64_t t = (uint64_t)tmp[k] + c;
                tmp[k] = (uint32_t)t;
                c = t >> 32;
            }
        }
        uint32_t m = n + 2;
        while (m && tmp[m - 1] == 0) --m;
        if (m > kLimbs) { overflow = true; return; }
        for (uint32_t i = 0; i < m; ++i) d[i] = tmp[i];
        n = m;
    }
    // *this /= v where v (0 < v < 2^64) divides *this exactly; false otherwise
    bool div_exact_small(uint64_t v) {
        unsigned __int128 r = 0;
        for (uint32_t i = n; i-- > 0;) {
            const unsigned __int128 cur = (r << 32) | d[i];
            d[i] = (uint32_t)(cur / v);
            r = cur % v;
        }
        trim();
        return r == 0;
    }
    static int cmp(const Big &a, const Big &b) {
        if (a.n != b.n) return a.n < b.n ? -1 : 1;
        for (uint32_t i = a.n; i-- > 0;)
            if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
        return 0;
    }
};

// With X ~ Bin(n, T), T = tn/td, and q = td - tn:
//   P(X = i) td^n = C(n, i) tn^i q^(n - i) =: term_i,
// term_{i+1} = term_i (n - i) tn / ((i + 1) q) and term_{i-1} = term_i i q / ((n - i + 1) tn),
// both exact divisions, so each tail is accumulated one term at a time.
hoph_status tail_integers(uint32_t n, hoph_ratio T, hoph_ratio eps, int32_t &j_lo, int32_t &j_hi,
                          std::string &err) {
    if (n == 0 || n > 256) { err = "binomial size must be in [1, 256]"; return HOPH_E_INVAL; }
    if (T.den == 0 || T.num == 0 || T.num > T.den) { err = "T must be in (0, 1]"; return HOPH_E_INVAL; }
    if (eps.den == 0 || eps.num >= eps.den) { err = "eps must be in [0, 1)"; return HOPH_E_INVAL; }
    const uint64_t tn = T.num, q = (uint64_t)T.den - T.num;
    // rhs = eps.num td^n; the tail test is eps.den * tail <= rhs
    Big rhs = Big::of(eps.num);
    for (uint32_t i = 0; i < n; ++i) rhs.mul_small(T.den);
    bool exact = true;
    // lower tail: P(X <= j) <= eps, terms from i = 0 upwards
    j_lo = -1;
    {
        Big term = Big::of(1);                         // term_0 = q^n
        for (uint32_t i = 0; i < n; ++i) term.mul_small(q);
        Big cum;
        for (uint32_t j = 0; j <= n; ++j) {
            if (j > 0) {
                if (q == 0) {                          // T = 1: only term_n = tn^n is not zero
                    term = Big();
                    if (j == n) {
                        term = Big::of(1);
                        for (uint32_t i = 0; i < n; ++i) term.mul_small(tn);
                    }
                } else {
                    term.mul_small((uint64_t)(n - j + 1) * tn);
                    exact &= term.div_exact_small((uint64_t)j * q);
                }
            }
            cum.add(term);
            Big lhs = cum;
            lhs.mul_small(eps.den);
            if (Big::cmp(lhs, rhs) <= 0) j_lo = (int32_t)j; else break;
        }
        exact &= !cum.overflow && !term.overflow;
    }
    // upper tail: P(X >= j) <= eps, terms from i = n downwards
    j_hi = (int32_t)n + 1;
    {
        Big term = Big::of(1);                         // term_n = tn^n
        for (uint32_t i = 0; i < n; ++i) term.mul_small(tn);
        Big cu;
        for (int32_t j = (int32_t)n; j >= 0; --j) {
            if (j < (int32_t)n) {
                if (q == 0) {
                    term = Big();
                } else {                                // term_j from term_{j+1}
                    term.mul_small((uint64_t)(j + 1) * q);
                    exact &= term.div_exact_small((uint64_t)(n - (uint32_t)j) * tn);
                }
            }
            cu.add(term);
            Big lhs = cu;
            lhs.mul_small(eps.den);
            if (Big::cmp(lhs, rhs) <= 0) j_hi = j; else break;
        }
        exact &= !cu.overflow && !term.overflow;
    }
    if (!exact || rhs.overflow) { err = "internal error: binomial tail arithmetic"; return HOPH_E_UNSUPPORTED; }
    return HOPH_OK;
}

// ---------------------------------------------------------------------------
// Decision tables
// ---------------------------------------------------------------------------
static i128 floor_div(i128 a, i128 b) {            // b > 0
    i128 q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}
static i128 ceil_div(i128 a, i128 b) {             // b > 0
    i128 q = a / b;
    if ((a % b != 0) && (a > 0)) ++q;
    return q;
}
static uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

hoph_status build_tables(const LayoutInfo &lay, const hoph_query_params &qp, bool goph,
                         hoph_decision_tables &out, std::string &err) {
    if (qp.empty_policy > HOPH_EMPTY_EITHER) { err = "unknown empty policy"; return HOPH_E_INVAL; }
    std::memset(&out, 0, sizeof(out));
    const uint32_t kp = lay.kp, L = lay.L;
    hoph_status st = tail_integers(kp, qp.T, qp.eps, out.j_lo, out.j_hi, err);
    if (st) return st;
    out.L = L;
    out.k_group = kp;
    out.empty_policy = qp.empty_policy;
    out.goph = goph ? 1 : 0;
    const i128 LIM = (i128)INT64_MAX - 2;
    // rate scale: every rate m / (k' - e) is an integer multiple of 1 / lambda
    i128 lam = 1;
    if (qp.empty_policy == HOPH_EMPTY_LITERAL) {
        lam = kp;
    } else {
        for (uint32_t i = 2; i <= kp; ++i) {
            lam = lam / (i128)gcd64((uint64_t)(lam % i), i) * i;
            if (lam > LIM) { err = "lcm(1..k_group) does not fit 64 bits"; return HOPH_E_UNSUPPORTED; }
        }
    }
    // integer group weights W_j over wsum: GOPH 1/L; HOPH a b^(j-1) / (a+b)^j for
    // j < L and (b / (a+b))^(L-1) for the last group
    i128 W[HOPH_MAX_GROUPS], wsum = 0;
    if (goph) {
        for (uint32_t j = 0; j < L; ++j) W[j] = 1;
        wsum = L;
    } else {
        const i128 a = lay.ra, b = lay.rb;
        i128 pb = 1;                       // b^(j-1)
        for (uint32_t j = 0; j + 1 < L; ++j) {
            i128 w = a * pb;
            for (uint32_t t = j + 1; t + 1 < L; ++t) {   // (a+b)^(L-1-j-1)
                w *= (a + b);
                if (w > LIM) { err = "group weights do not fit 64 bits"; return HOPH_E_UNSUPPORTED; }
            }
            W[j] = w;
            pb *= b;
            if (pb > LIM) { err = "group weights do not fit 64 bits"; return HOPH_E_UNSUPPORTED; }
        }
        W[L - 1] = pb;
        for (uint32_t j = 0; j < L; ++j) wsum += W[j];
    }
    if (wsum > LIM / lam) { err = "exact decision state exceeds 64 bits for these parameters"; return HOPH_E_UNSUPPORTED; }
    const i128 Dn = wsum * lam;            // S~ = S * Dn, S~ in [0, Dn]
    const i128 tn = qp.T.num, td = qp.T.den;
    out.lcm = (int64_t)lam;
    out.wsum = (int64_t)wsum;
    for (uint32_t e = 0; e < kp; ++e)
        out.dmul[e] = qp.empty_policy == HOPH_EMPTY_LITERAL ? (e == 0 ? 1 : 0) : (int64_t)(lam / (kp - e));
    out.dmul[kp] = (int64_t)lam;
    auto clampc = [&](i128 v) -> int64_t {
        if (v < -1) return -1;
        if (v > Dn + 1) return (int64_t)(Dn + 1);
        return (int64_t)v;
    };
    i128 Wc = 0;
    for (uint32_t l = 0; l < L; ++l) {
        out.W[l] = (int64_t)W[l];
        Wc += W[l];
        if (l + 1 == L) {
            // after the last group: accept iff S >= T
            i128 acc = ceil_div(tn * Dn, td);
            out.acc[l] = clampc(acc);
            out.rej[l] = clampc(acc - 1);
            break;
        }
        const i128 rem = wsum - Wc;        // (1 - U_l) * wsum > 0
        // P_r < T  <=>  S > T U_l  <=>  S~ > tn Wc lam / td
        const i128 mid = floor_div(tn * Wc * lam, td);
        // accept: P(X < x) <= eps  <=>  x <= j_lo + 1  <=>  S >= T - (j_lo + 1)(1 - U_l) / k'
        const i128 dd = td * kp;
        const i128 a2 = ceil_div(tn * Dn * kp - td * (i128)(out.j_lo + 1) * rem * lam, dd);
        // reject: P(X >= x) <= eps  <=>  x > j_hi - 1  <=>  S < T - (j_hi - 1)(1 - U_l) / k'
        const i128 r2 = ceil_div(tn * Dn * kp - td * (i128)(out.j_hi - 1) * rem * lam, dd) - 1;
        out.acc[l] = clampc(std::max(mid + 1, a2));
        out.rej[l] = clampc(std::min(mid, r2));
    }
    return HOPH_OK;
}

void to_scan_tab(const hoph_decision_tables &t, ScanTab &s) {
    std::memset(&s, 0, sizeof(s));
    for (uint32_t l = 0; l < t.L; ++l) { s.W[l] = t.W[l]; s.acc[l] = t.acc[l]; s.rej[l] = t.rej[l]; }
    for (uint32_t e = 0; e <= t.k_group; ++e) s.dmul[e] = t.dmul[e];
    s.lambda = t.lcm;
    s.L = t.L;
    s.kp = t.k_group;
    s.policy = t.empty_policy;
    // After the first group the state is W_1 * m * unit(e); for e < k' the two
    // cutoffs become thresholds on the matched count m.
    for (uint32_t e = 0; e <= t.k_group; ++e) {
        s.macc0[e] = 65;
        s.mrej0[e] = -1;
        if (e == t.k_group) continue;                 // 0/0 group: decided from the state itself
        const int64_t unit = t.W[0] * (t.empty_policy == HOPH_EMPTY_LITERAL ? 1 : t.dmul[e]);
        if (unit <= 0) continue;
        const i128 a = ceil_div((i128)t.acc[0], unit), r = floor_div((i128)t.rej[0], unit);
        s.macc0[e] = (int32_t)std::max<i128>(0, std::min<i128>(65, a));
        s.mrej0[e] = (int32_t)std::max<i128>(-1, std::min<i128>(64, r));
    }
    // First group on codes: a query with eq empty bins meets sets whose empty
    // count e is <= eq (JOINT; e == kp only when eq == kp) or 0 (LITERAL).  The
    // pair is rejected when m <= thr for the smallest reject threshold over
    // those e; with the code count m = (kp - eq) - dn (dn = query-non-empty bins
    // whose codes differ) that is dn >= (kp - eq) - thr.  thr < 0: never.
    const int32_t kp = (int32_t)t.k_group;
    for (int32_t eq = 0; eq <= kp; ++eq) {
        int32_t thr = -1;
        if (t.empty_policy == HOPH_EMPTY_LITERAL) {
            thr = s.mrej0[0];
        } else if (t.empty_policy == HOPH_EMPTY_JOINT && eq < kp) {
            thr = s.mrej0[0];
            for (int32_t e = 1; e <= eq; ++e) thr = std::min(thr, s.mrej0[e]);
        }
        s.dthr0[eq] = thr < 0 ? kp + 1 : (kp - eq) - thr;
    }
}

uint32_t default_coarse_depth(const ScanTab &tab, uint32_t requested, uint32_t maxd, uint32_t pk) {
    uint32_t d = requested;
    if (d == 0) {
        if (8 * (int64_t)tab.mrej0[0] >= (int64_t)tab.kp && tab.mrej0[0] >= 0) {
            d = 1;
        } else {
            uint32_t g = 0;                  // groups up to and including the first with a reject cutoff
            while (g < tab.L && tab.rej[g] < 0) ++g;
            d = g < tab.L ? g + 2 : maxd;    // one group past it
            if (pk > 1) d = (d + pk - 1) / pk * pk;
        }
    }
    return std::max<uint32_t>(1, std::min(d, maxd));
}

}  // namespace hoph
