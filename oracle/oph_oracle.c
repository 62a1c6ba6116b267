/*
 * Plain C reference for one-permutation hashing (OPH), grouped OPH (GOPH),
 * (a:b) hierarchical OPH (HOPH) and the MinWise comparator, after Zhang et al.,
 * "Hierarchical One Permutation Hashing" (arXiv 1805.11254).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is built into oracle/liboracle.so and
 * is called from tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
 * leg.  The GPU library shares no source, header, table or helper with it.
 *
 * It follows the same conventions as oracle/tiny.py (which states them in
 * full) with slow, plain arithmetic: 128-bit integer division for the hash and
 * the bin bounds, a binary search of the bin-start table for the bin of a
 * value, and exact reduced fractions for every weight, rate and decision.
 * The binomial tail integers (j_lo, j_hi) are passed in; oracle/tiny.py
 * computes them from the exact binomial tails.
 *
 * Return codes: 0 ok, -1 invalid parameters, -2 an id >= universe (the id is
 * skipped), -3 an empty set (its signature is all EMPTY), -5 exact arithmetic
 * would overflow 128 bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;
typedef unsigned __int128 u128;

#define ORC_EMPTY 0xFFFFFFFFu
#define ORC_P31 ((uint64_t)2147483647u)
#define ORC_P32P15 ((uint64_t)4294967311ull)

enum { H_TABLE = 0, H_P31 = 1, H_P32 = 2 };
enum { LAY_OPH = 0, LAY_HIER = 1 };
enum { POL_JOINT = 0, POL_LITERAL = 1, POL_EITHER = 2 };

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Permutation psi (Sec. 3.2)                                              */
/* ---------------------------------------------------------------------- */
static uint64_t range_of(int kind, uint64_t universe) {
    if (kind == H_TABLE) return universe;
    if (kind == H_P31) return ORC_P31;
    return ORC_P32P15;
}

static uint64_t psi(int kind, const uint32_t *perm, uint64_t ha, uint64_t hb, uint64_t x) {
    if (kind == H_TABLE) return perm[x];
    uint64_t p = (kind == H_P31) ? ORC_P31 : ORC_P32P15;
    return (uint64_t)(((u128)ha * x + hb) % p);
}

/* ---------------------------------------------------------------------- */
/* Bin starts: k+1 entries, starts[k] = R (Sec. 3.2 / Sec. 4.1)           */
/* ---------------------------------------------------------------------- */
static int make_starts(int layout, uint64_t R, uint32_t k, uint32_t kp,
                       uint32_t ra, uint32_t rb, uint64_t *starts) {
    if (k == 0 || kp == 0 || k % kp) return -1;
    uint32_t L = k / kp;
    if (layout == LAY_OPH) {
        if ((uint64_t)k > R) return -1;
        for (uint32_t b = 0; b < k; ++b)
            starts[b] = (uint64_t)(((u128)b * R + k - 1) / k);   /* ceil(b R / k) */
    } else if (layout == LAY_HIER) {
        if (ra == 0 || rb == 0) return -1;
        uint64_t lo = 0;
        for (uint32_t g = 0; g < L; ++g) {
            uint64_t size;
            if (g + 1 < L) {
                size = (uint64_t)(((u128)(R - lo) * ra) / ((uint64_t)ra + rb));
                uint64_t rest = R - lo - size;
                if (size <= kp || rest <= kp) return -1;          /* stop rule */
            } else {
                size = R - lo;
                if (size < kp) return -1;
            }
            for (uint32_t t = 0; t < kp; ++t)
                starts[g * kp + t] = lo + (uint64_t)(((u128)t * size + kp - 1) / kp);
            lo += size;
        }
    } else {
        return -1;
    }
    starts[k] = R;
    for (uint32_t b = 0; b < k; ++b)
        if (starts[b + 1] <= starts[b] || starts[b + 1] - starts[b] > 0xFFFFFFFFull) return -1;
    return 0;
}

/* largest b with starts[b] <= v */
static uint32_t find_bin(const uint64_t *starts, uint32_t k, uint64_t v) {
    uint32_t lo = 0, hi = k;            /* invariant: starts[lo] <= v < starts[hi] */
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (starts[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

int orc_layout_starts(int hash_kind, uint64_t universe, int layout, uint32_t k, uint32_t kp,
                      uint32_t ra, uint32_t rb, uint64_t *starts_out) {
    return make_starts(layout, range_of(hash_kind, universe), k, kp, ra, rb, starts_out);
}

/*
 * OPH / HOPH signatures.  which == NULL sketches every set into sigs[n][k];
 * otherwise only sets which[0..n_which) into sigs[n_which][k].
 */
int orc_sketch(int hash_kind, uint64_t universe, uint64_t ha, uint64_t hb, const uint32_t *perm,
               int layout, uint32_t k, uint32_t kp, uint32_t ra, uint32_t rb,
               const uint32_t *ids, const uint64_t *offsets, uint64_t n_sets,
               const uint64_t *which, uint64_t n_which, uint32_t *sigs, int nthreads) {
    uint64_t R = range_of(hash_kind, universe);
    if (hash_kind == H_P31 && universe > ORC_P31) return -1;
    if (hash_kind == H_P32 && universe > ORC_P32P15) return -1;
    uint64_t *starts = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)k + 1));
    if (!starts) return -1;
    if (make_starts(layout, R, k, kp, ra, rb, starts)) { free(starts); return -1; }
    uint64_t n_out = which ? n_which : n_sets;
    int bad_id = 0, empty = 0;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad_id, empty)
    for (int64_t i = 0; i < (int64_t)n_out; ++i) {
        uint64_t s = which ? which[i] : (uint64_t)i;
        uint32_t *sig = sigs + (size_t)i * k;
        for (uint32_t b = 0; b < k; ++b) sig[b] = ORC_EMPTY;
        if (offsets[s + 1] == offsets[s]) empty = 1;
        for (uint64_t j = offsets[s]; j < offsets[s + 1]; ++j) {
            uint64_t x = ids[j];
            if (x >= universe) { bad_id = 1; continue; }
            uint64_t v = psi(hash_kind, perm, ha, hb, x);
            uint32_t b = find_bin(starts, k, v);
            uint64_t off = v - starts[b];
            if (off < sig[b]) sig[b] = (uint32_t)off;
        }
    }
    free(starts);
    if (bad_id) return -2;
    if (empty) return -3;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Exact fractions                                                         */
/* ---------------------------------------------------------------------- */
typedef struct { i128 n, d; } frac;   /* d > 0, reduced */

static i128 gcd_i(i128 a, i128 b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) { i128 t = a % b; a = b; b = t; }
    return a;
}

static int fr_make(i128 n, i128 d, frac *out) {
    if (d == 0) return -5;
    if (d < 0) { n = -n; d = -d; }
    i128 g = gcd_i(n, d);
    if (g > 1) { n /= g; d /= g; }
    out->n = n; out->d = d;
    return 0;
}

static int mul_ok(i128 a, i128 b, i128 *r) { return __builtin_mul_overflow(a, b, r) ? -5 : 0; }
static int add_ok(i128 a, i128 b, i128 *r) { return __builtin_add_overflow(a, b, r) ? -5 : 0; }

static int fr_add(frac a, frac b, frac *out) {
    i128 x, y, n, d;
    if (mul_ok(a.n, b.d, &x) || mul_ok(b.n, a.d, &y) || add_ok(x, y, &n) || mul_ok(a.d, b.d, &d))
        return -5;
    return fr_make(n, d, out);
}

static int fr_sub(frac a, frac b, frac *out) {
    b.n = -b.n;
    return fr_add(a, b, out);
}

static int fr_mul(frac a, frac b, frac *out) {
    i128 g1 = gcd_i(a.n, b.d), g2 = gcd_i(b.n, a.d);
    if (g1 == 0) g1 = 1;
    if (g2 == 0) g2 = 1;
    i128 n, d;
    if (mul_ok(a.n / g1, b.n / g2, &n) || mul_ok(a.d / g2, b.d / g1, &d)) return -5;
    return fr_make(n, d, out);
}

static int fr_div(frac a, frac b, frac *out) {
    frac inv = { b.d, b.n };
    if (inv.d < 0) { inv.n = -inv.n; inv.d = -inv.d; }
    return fr_mul(a, inv, out);
}

/* a < b ? 1 : 0, or -5 */
static int fr_lt(frac a, frac b, int *res) {
    i128 x, y;
    if (mul_ok(a.n, b.d, &x) || mul_ok(b.n, a.d, &y)) return -5;
    *res = x < y;
    return 0;
}

static i128 fr_ceil(frac a) {
    i128 q = a.n / a.d;                 /* truncates toward zero */
    if (a.n % a.d != 0 && a.n > 0) q += 1;
    return q;
}

/* ---------------------------------------------------------------------- */
/* Per-group counts and rate (Eqs. 1-4, Eq. 6)                             */
/* ---------------------------------------------------------------------- */
static void counts(const uint32_t *q, const uint32_t *s, uint32_t n, int policy,
                   uint32_t *m, uint32_t *e, int *all_joint) {
    uint32_t mm = 0, joint = 0, either = 0;
    for (uint32_t i = 0; i < n; ++i) {
        int qe = q[i] == ORC_EMPTY, se = s[i] == ORC_EMPTY;
        if (!qe && !se && q[i] == s[i]) ++mm;
        if (qe && se) ++joint;
        if (qe || se) ++either;
    }
    *m = mm;
    *all_joint = (joint == n);
    *e = (policy == POL_JOINT) ? joint : (policy == POL_EITHER) ? either : 0;
}

static frac rate_of(uint32_t m, uint32_t e, uint32_t n, int all_joint, int policy) {
    frac r;
    if (policy == POL_LITERAL) { fr_make(m, n, &r); return r; }
    if (n == e) { r.n = all_joint ? 1 : 0; r.d = 1; return r; }
    fr_make(m, n - e, &r);
    return r;
}

/* group weights: 1/L for GOPH; a b^(j-1)/(a+b)^j and (b/(a+b))^(L-1) for HOPH */
static int weights(int goph, uint32_t L, uint32_t ra, uint32_t rb, frac *w) {
    if (goph) {
        for (uint32_t j = 0; j < L; ++j) { w[j].n = 1; w[j].d = L; }
        return 0;
    }
    frac r, one_minus_r, pw = { 1, 1 };
    if (fr_make(ra, (i128)ra + rb, &r) || fr_make(rb, (i128)ra + rb, &one_minus_r)) return -5;
    for (uint32_t j = 0; j + 1 < L; ++j) {
        if (fr_mul(r, pw, &w[j])) return -5;
        if (fr_mul(pw, one_minus_r, &pw)) return -5;
    }
    w[L - 1] = pw;
    return 0;
}

/*
 * Alg. 1 / Alg. 2 for one pair.  Returns 1 accept, 0 reject, <0 error;
 * *step is the group after which the decision was taken (1-based).
 */
static int decide_pair(const uint32_t *q, const uint32_t *s, uint32_t L, uint32_t kp,
                       const frac *w, frac T, int32_t j_lo, int32_t j_hi, int policy, int *step) {
    frac S = { 0, 1 }, U = { 0, 1 }, one = { 1, 1 }, kpf = { kp, 1 };
    for (uint32_t l = 1; l <= L; ++l) {
        uint32_t m, e;
        int aj, lt, rc;
        counts(q + (l - 1) * kp, s + (l - 1) * kp, kp, policy, &m, &e, &aj);
        frac r = rate_of(m, e, kp, aj, policy), wr;
        if ((rc = fr_mul(w[l - 1], r, &wr))) return rc;
        if ((rc = fr_add(S, wr, &S))) return rc;
        if ((rc = fr_add(U, w[l - 1], &U))) return rc;
        *step = (int)l;
        if (l == L) {
            if ((rc = fr_lt(S, T, &lt))) return rc;
            return !lt;                       /* accept iff S >= T */
        }
        frac num, den, Pr, x;
        if ((rc = fr_sub(T, S, &num)) || (rc = fr_sub(one, U, &den)) ||
            (rc = fr_div(num, den, &Pr)) || (rc = fr_mul(kpf, Pr, &x)))
            return rc;
        i128 c = fr_ceil(x);
        if ((rc = fr_lt(Pr, T, &lt))) return rc;
        if (lt) {
            if (c - 1 <= j_lo) return 1;      /* P(X < x) <= eps: accept */
        } else {
            if (c >= j_hi) return 0;          /* P(X >= x) <= eps: reject */
        }
    }
    return -1;
}

/*
 * GOPH (goph = 1, bins in contiguous groups of kp, weights 1/L) or (a:b) HOPH
 * (goph = 0) over row-major signatures sigs[n_sets][k] and qsigs[n_q][k].
 * Writes out_offsets[n_q+1] and, up to cap entries, ascending accepted set ids
 * per query (and their stop step when out_steps != NULL).  dense_dec, when not
 * NULL, receives n_q*n_sets bytes: 1 accept / 0 reject; dense_step the step.
 * Returns the number of accepted pairs, or a negative code.
 */
int64_t orc_query(int goph, uint32_t k, uint32_t kp, uint32_t ra, uint32_t rb,
                  const uint32_t *sigs, uint64_t n_sets, const uint32_t *qsigs, uint32_t n_q,
                  uint32_t tn, uint32_t td, int32_t j_lo, int32_t j_hi, int policy,
                  uint64_t *out_offsets, uint32_t *out_ids, uint8_t *out_steps, uint64_t cap,
                  uint8_t *dense_dec, uint8_t *dense_step, int nthreads) {
    if (k == 0 || kp == 0 || k % kp || td == 0 || tn == 0 || tn > td) return -1;
    if (td > (1u << 20)) return -5;
    uint32_t L = k / kp;
    frac *w = (frac *)malloc(sizeof(frac) * L);
    if (!w) return -1;
    if (weights(goph, L, ra, rb, w)) { free(w); return -5; }
    frac T;
    fr_make(tn, td, &T);
    uint8_t *flag = (uint8_t *)malloc(n_sets ? n_sets : 1);
    uint8_t *stp = (uint8_t *)malloc(n_sets ? n_sets : 1);
    if (!flag || !stp) { free(w); free(flag); free(stp); return -1; }
    int err = 0;
    uint64_t total = 0;
    set_threads(nthreads);
    out_offsets[0] = 0;
    for (uint32_t qi = 0; qi < n_q && !err; ++qi) {
        const uint32_t *q = qsigs + (size_t)qi * k;
#pragma omp parallel for schedule(static, 4096) reduction(| : err)
        for (int64_t si = 0; si < (int64_t)n_sets; ++si) {
            int step = 0;
            int d = decide_pair(q, sigs + (size_t)si * k, L, kp, w, T, j_lo, j_hi, policy, &step);
            if (d < 0) { err = 1; d = 0; }
            flag[si] = (uint8_t)d;
            stp[si] = (uint8_t)step;
        }
        for (uint64_t si = 0; si < n_sets; ++si) {
            if (dense_dec) dense_dec[(size_t)qi * n_sets + si] = flag[si];
            if (dense_step) dense_step[(size_t)qi * n_sets + si] = stp[si];
            if (flag[si]) {
                if (total < cap) {
                    out_ids[total] = (uint32_t)si;
                    if (out_steps) out_steps[total] = stp[si];
                }
                ++total;
            }
        }
        out_offsets[qi + 1] = total;
    }
    free(w); free(flag); free(stp);
    return err ? -5 : (int64_t)total;
}

/* Plain OPH comparator: Eq. 6 over all k bins, accept iff >= T. */
int64_t orc_query_oph_full(uint32_t k, const uint32_t *sigs, uint64_t n_sets,
                           const uint32_t *qsigs, uint32_t n_q, uint32_t tn, uint32_t td, int policy,
                           uint64_t *out_offsets, uint32_t *out_ids, uint64_t cap, int nthreads) {
    if (k == 0 || td == 0 || tn == 0 || tn > td) return -1;
    frac T;
    fr_make(tn, td, &T);
    uint8_t *flag = (uint8_t *)malloc(n_sets ? n_sets : 1);
    if (!flag) return -1;
    uint64_t total = 0;
    int err = 0;
    set_threads(nthreads);
    out_offsets[0] = 0;
    for (uint32_t qi = 0; qi < n_q; ++qi) {
        const uint32_t *q = qsigs + (size_t)qi * k;
#pragma omp parallel for schedule(static, 4096) reduction(| : err)
        for (int64_t si = 0; si < (int64_t)n_sets; ++si) {
            uint32_t m, e;
            int aj, lt;
            counts(q, sigs + (size_t)si * k, k, policy, &m, &e, &aj);
            frac r = rate_of(m, e, k, aj, policy);
            if (fr_lt(r, T, &lt)) { err = 1; lt = 1; }
            flag[si] = (uint8_t)!lt;
        }
        for (uint64_t si = 0; si < n_sets; ++si)
            if (flag[si]) {
                if (total < cap) out_ids[total] = (uint32_t)si;
                ++total;
            }
        out_offsets[qi + 1] = total;
    }
    free(flag);
    return err ? -5 : (int64_t)total;
}

/* ---------------------------------------------------------------------- */
/* MinWise comparator: k independent hashes (a_i x + b_i) mod p            */
/* ---------------------------------------------------------------------- */
int orc_minwise_sketch(int hash_kind, uint64_t universe, uint32_t k, const uint64_t *ha, const uint64_t *hb,
                       const uint32_t *ids, const uint64_t *offsets, uint64_t n_sets,
                       const uint64_t *which, uint64_t n_which, uint64_t *sigs, int nthreads) {
    if (hash_kind != H_P31 && hash_kind != H_P32) return -1;
    if (hash_kind == H_P31 && universe > ORC_P31) return -1;
    uint64_t n_out = which ? n_which : n_sets;
    int bad_id = 0, empty = 0;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad_id, empty)
    for (int64_t i = 0; i < (int64_t)n_out; ++i) {
        uint64_t s = which ? which[i] : (uint64_t)i;
        uint64_t *sig = sigs + (size_t)i * k;
        for (uint32_t h = 0; h < k; ++h) sig[h] = UINT64_MAX;
        if (offsets[s + 1] == offsets[s]) empty = 1;
        for (uint64_t j = offsets[s]; j < offsets[s + 1]; ++j) {
            uint64_t x = ids[j];
            if (x >= universe) { bad_id = 1; continue; }
            for (uint32_t h = 0; h < k; ++h) {
                uint64_t v = psi(hash_kind, NULL, ha[h], hb[h], x);
                if (v < sig[h]) sig[h] = v;
            }
        }
    }
    if (bad_id) return -2;
    if (empty) return -3;
    return 0;
}

int64_t orc_minwise_query(uint32_t k, const uint64_t *sigs, uint64_t n_sets, const uint64_t *qsigs,
                          uint32_t n_q, uint32_t tn, uint32_t td,
                          uint64_t *out_offsets, uint32_t *out_ids, uint64_t cap, int nthreads) {
    if (k == 0 || td == 0 || tn == 0 || tn > td) return -1;
    uint8_t *flag = (uint8_t *)malloc(n_sets ? n_sets : 1);
    if (!flag) return -1;
    uint64_t total = 0;
    set_threads(nthreads);
    out_offsets[0] = 0;
    for (uint32_t qi = 0; qi < n_q; ++qi) {
        const uint64_t *q = qsigs + (size_t)qi * k;
#pragma omp parallel for schedule(static, 4096)
        for (int64_t si = 0; si < (int64_t)n_sets; ++si) {
            const uint64_t *s = sigs + (size_t)si * k;
            uint64_t eq = 0;
            for (uint32_t h = 0; h < k; ++h) eq += (q[h] == s[h]);
            /* eq / k >= tn / td */
            flag[si] = (uint8_t)((u128)eq * td >= (u128)tn * k);
        }
        for (uint64_t si = 0; si < n_sets; ++si)
            if (flag[si]) {
                if (total < cap) out_ids[total] = (uint32_t)si;
                ++total;
            }
        out_offsets[qi + 1] = total;
    }
    free(flag);
    return (int64_t)total;
}

/* Per-group (m, e) of one pair, for checking the device counts. */
void orc_pair_counts(const uint32_t *q, const uint32_t *s, uint32_t k, uint32_t kp, int policy,
                     uint32_t *m_out, uint32_t *e_out) {
    for (uint32_t g = 0; g < k / kp; ++g) {
        int aj;
        counts(q + g * kp, s + g * kp, kp, policy, &m_out[g], &e_out[g], &aj);
    }
}
