// Internal declarations shared by the host runtime and the HIP kernels of
// libhoph.  Nothing here is part of the C ABI (include/hoph.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "hoph.h"

namespace hoph {

constexpr uint64_t kP31 = 2147483647ull;        // 2^31 - 1
constexpr uint64_t kP32 = 4294967311ull;        // 2^32 + 15, prime
constexpr uint32_t kLutMax = 4096;              // region lookup entries
constexpr uint32_t kTile = 64;                  // sets per index tile = one wavefront
constexpr uint32_t kMaxDepth = 4;               // coarse groups (code units) kept in registers
// Queries per chunk of the coarse pass, at least (up to the batch size): every
// chunk reads the index's code planes once, and up to about this many queries a
// pass reads more bytes than its integer work hides (32 bytes of planes per set
// against 5-11 lane-operations per pair).
constexpr uint32_t kChunkQueries = 64;
// Narrowed coarse pass: an 8-bit code per bin, stored as 8 bit-planes per
// code unit (bit i of plane p = bit p of the code of bin i of the unit), so
// that one 32-bit word holds one plane of 32 bins.  EMPTY has a code of its own.
constexpr uint32_t kCodeBits = 8;
constexpr uint32_t kCodeEmpty = 0xFFu;           // code of EMPTY; other bins map to [0, 254]
// Small groups share plane words: a code unit is pk consecutive whole groups
// (pk = floor(32 / k') for k' <= 16, at most L; else 1), so a unit spans
// pk k' <= 32 bins (k' <= 32) or one group of two plane words (k' > 32), and
// its planes are written and read as those of one group of pk k' bins.
__host__ __device__ inline uint32_t code_pack(uint32_t kp, uint32_t L) {
    const uint32_t pk = kp <= 16 ? 32u / kp : 1u;
    return pk < L ? pk : (L > 0 ? L : 1u);
}
// Leading groups that carry codes, in whole units: at least the
// register-resident depth in units and enough units to cover a bin budget, at
// most max_code_units (the deep code pass stages that many units of one tile,
// 64 lanes x (planes + set-empty masks), in under 64 KB of LDS: 24 units of one
// plane word, 12 of two), and no unit past the row.  GOPH weighs its groups
// equally and, with small groups or a low threshold, can first reject only
// after one to two hundred bins; HOPH decides most pairs in its heavy first
// group.
constexpr uint32_t kCodeBinsHier = 128;
constexpr uint32_t kCodeBinsFlat = 256;
inline uint32_t max_code_units(uint32_t kp) { return kp > 32 ? 12u : 24u; }
inline uint32_t code_groups(uint32_t kp, uint32_t L, bool hier) {
    const uint32_t pk = code_pack(kp, L), ub = pk * kp;
    const uint32_t bins = hier ? kCodeBinsHier : kCodeBinsFlat, cap = max_code_units(kp);
    uint32_t u = (bins + ub - 1) / ub;
    u = u < kMaxDepth ? kMaxDepth : (u > cap ? cap : u);
    const uint32_t whole = L / pk;            // units inside the row (pk <= L)
    return (u < whole ? u : whole) * pk;
}
// Bins of one code unit, and code units of cg groups.
__host__ __device__ inline uint32_t code_unit_bins(uint32_t kp, uint32_t L) { return code_pack(kp, L) * kp; }
__host__ __device__ inline uint32_t code_units(uint32_t cg, uint32_t kp, uint32_t L) { return cg / code_pack(kp, L); }

// Device error bits (one 32-bit word per device).
constexpr uint32_t kErrRange = 1u;              // an id >= universe, or a table value >= R
constexpr uint32_t kErrEmptySet = 2u;           // a set with no element
constexpr uint32_t kErrBadRange = 4u;           // a set whose end offset is below its start

// ---------------------------------------------------------------------------
// Sketch layout, passed by value to the sketch kernels.  The permuted range
// [0, R) is cut into n_regions regions (OPH: 1 region of k bins; HIER: L
// groups of k' bins).  Inside region r (start s_r, size z_r, n_r bins) bin t
// starts at s_r + ceil(t z_r / n_r).
// ---------------------------------------------------------------------------
struct SketchDesc {
    const uint32_t *perm;
    uint64_t universe, ha, hb, R;
    uint32_t hash, k, n_regions, lut_shift, lut_size, nb;   // nb = bins per region
    // Uniform bin estimate (est_ok): est(v) = mulhi32(v >> est_shift, est_mul) is
    // the bin of v or the bin before it, for every v < R (checked on the host
    // against every bin start), so one read of a pair of bin starts settles it.
    uint32_t est_mul, est_shift, est_ok;
    uint32_t log_ok;     // regions by log-domain cells (see log_cell), narrow ranges only
    uint32_t pow2_ok;    // power-of-two regions and bins (see locate_pow2), narrow ranges only
    uint32_t pow2[32][4];                                    // locate_pow2 table, by leading-zero count
    uint64_t reg_start[HOPH_MAX_GROUPS + 1];                 // reg_start[n_regions] = R
    uint64_t reg_magic[HOPH_MAX_GROUPS];                     // floor(2^64 nb / z_r), see bin_of
    uint32_t reg_mag32[HOPH_MAX_GROUPS];                     // min(2^32 - 1, floor(2^32 nb / z_r))
};

// Host view of a validated layout.
struct LayoutInfo {
    uint64_t R = 0;
    uint32_t k = 0, kp = 0, L = 0, n_regions = 0, nb = 0, ra = 1, rb = 1;
    std::vector<uint64_t> reg_start;   // n_regions + 1
    std::vector<uint64_t> reg_magic;   // n_regions
    std::vector<uint32_t> reg_mag32;   // n_regions
    uint32_t lut_shift = 0, lut_size = 0;
    uint32_t est_mul = 0, est_shift = 0, est_ok = 0;   // see SketchDesc
    uint32_t log_ok = 0;                               // see SketchDesc
    uint32_t pow2_ok = 0;                              // see SketchDesc
    std::vector<uint32_t> pow2;                        // 32 x {region start, shift, first bin, mask}
};

// ---------------------------------------------------------------------------
// Exact integer decision tables, passed by value to the scan kernels.
// ---------------------------------------------------------------------------
struct ScanTab {
    int64_t W[HOPH_MAX_GROUPS];
    int64_t acc[HOPH_MAX_GROUPS];
    int64_t rej[HOPH_MAX_GROUPS];
    int64_t dmul[HOPH_MAX_KGROUP + 1];
    int64_t lambda;                 // rate scale: lcm(1..k') (JOINT, EITHER) or k' (LITERAL)
    int32_t macc0[HOPH_MAX_KGROUP + 1];   // first group, e < k': accept iff m >= macc0[e]
    int32_t mrej0[HOPH_MAX_KGROUP + 1];   // first group, e < k': reject iff m <= mrej0[e]
    // First group on codes, by the query's empty count eq (JOINT, LITERAL):
    // reject when the count of query-non-empty bins whose codes differ is
    // >= dthr0[eq] (a bound that holds for every empty count the set may add).
    int32_t dthr0[HOPH_MAX_KGROUP + 1];
    uint32_t L, kp, policy, pad;
};

// A pair that the coarse pass could not decide: continue at group `depth`.
struct Survivor {
    uint32_t q, s;
    int64_t S;
};

// ---------------------------------------------------------------------------
// Inline arithmetic shared by the kernels and the host self-test hook.
// ---------------------------------------------------------------------------
// 8-bit code of a stored bin value: EMPTY -> kCodeEmpty, any other value to
// [0, 254] by a multiplicative mix (a bijection on 32-bit words) scaled into
// 255 values.  Equal values have equal codes, so a count of equal codes never
// falls below the count of equal values.
__host__ __device__ inline uint32_t bin_code(uint32_t v) {
    if (v == HOPH_EMPTY) return kCodeEmpty;
    return (uint32_t)(((uint64_t)(v * 0x9E3779B1u) * 255u) >> 32);
}

// 32-bit words per plane (k' <= 32: one, else two) and words per (set, group).
__host__ __device__ inline uint32_t code_plane_words(uint32_t kp) { return kp > 32 ? 2u : 1u; }
__host__ __device__ inline uint32_t code_words(uint32_t kp) { return kCodeBits * code_plane_words(kp); }
// A query's record per code group: the planes, then {non-empty mask low word,
// high word, first-group threshold on differing non-empty bins, empty count},
// then the group's words of the linear bound {c, z, y, 0} (LinTab).
__host__ __device__ inline uint32_t code_rec_words(uint32_t kp) { return code_words(kp) + 8u; }

// The multi-group code pass (HOPH or GOPH over 2-4 groups of k' <= 32 bins,
// JOINT or LITERAL) bounds each group's rate from above using the query's
// own empty count e_g only: the codes of the query-non-empty bins that differ
// (dn_g) are real differences, and the set's empty bins there differ too, so
// m_g <= (k' - e_g) - dn_g, and the joint empty count is at most e_g, so
// (JOINT) the state term W_g m_g lambda / (k' - ej) is at most
// C_g ((k' - e_g) - dn_g) with C_g = W_g lambda / (k' - e_g) (LITERAL: C_g = W_g).
// A step's test on the exact state then becomes a test on sum_g C_g dn_g,
// linear in the counts: reject when it reaches Z_s = sum_g C_g (k' - e_g) -
// rej_s, keep ("maybe": an accept cutoff may be reached) when it is at most
// Y_s = sum_g C_g (k' - e_g) - acc_s.  With c_g = floor(C_g / 2^shift),
// z_s = ceil(Z_s / 2^shift) and y_s = floor(Y_s / 2^shift) the tests on
// st_s = sum_{g <= s} c_g dn_g (st_s >= z_s rejects, st_s <= y_s keeps) stay
// on the safe side (fewer rejects, more keeps).  The kernels count agreeing
// bins, st'_s = sum_{g <= s} c_g ((k' - e_g) - dn_g) = S_s - st_s with
// S_s = sum_{g <= s} c_g (k' - e_g) < 2^31, so per query the record of group g
// holds c_g, z'_g = S_g - z_g (-1: never rejects) and y'_g = S_g - y_g
// (INT32_MAX: no accept cutoff reachable): st' <= z' rejects, st' >= y' keeps.
constexpr uint32_t kLinMaxSteps = 4;
struct LinTab {
    int64_t W[kLinMaxSteps], acc[kLinMaxSteps], rej[kLinMaxSteps];
    int64_t dmul[HOPH_MAX_KGROUP + 1];
    int64_t lambda;
    uint32_t steps;                 // groups with linear words (0: none)
    uint32_t shift, policy, kp;
};

// First-group reject thresholds on codes by the query's empty count (ScanTab::dthr0).
struct CodeThr {
    int32_t dthr[HOPH_MAX_KGROUP + 1];
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

// (a x + b) mod (2^31 - 1) for x, a, b < 2^31 - 1: Mersenne folding.  With
// P = 2^31 - 1, w = a x + b <= P (P - 1) < 2^62, and w = (w >> 31) + (w & P)
// (mod P) where both parts are < 2^31, so every step after the one 64-bit
// multiply-add is 32-bit.
__host__ __device__ inline uint32_t shr31_of_64(uint32_t hi, uint32_t lo) {   // ((hi:lo) >> 31) mod 2^32
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(hi, lo, 31);
#else
    return (hi << 1) | (lo >> 31);
#endif
}

// a * b for a, b < 2^24 (full-rate 24-bit multiply on the device).
__host__ __device__ inline uint32_t mul_u24(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return a * b;
#endif
}

// (a x + b) mod (2^31 - 1) for x, a, b < P = 2^31 - 1 (the host checks a, b and the
// universe; ids are clamped below it).  Then w = a x + b <= P (P - 1), so with
// w = h 2^31 + l (2^31 = 1 mod P): h <= 2^31 - 3 and s = l + h <= 2P - 2 < 2P,
// and one conditional subtraction finishes the reduction.
__host__ __device__ inline uint64_t psi_p31(uint64_t x, uint64_t a, uint64_t b) {
    const uint64_t w = (uint64_t)(uint32_t)a * (uint32_t)x + b;   // one 32 x 32 -> 64 multiply-add
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    const uint32_t s = (lo & 0x7FFFFFFFu) + shr31_of_64(hi, lo);   // l + h < 2P
    const uint32_t t = s - 0x7FFFFFFFu;                               // wraps above s when s < P
    return t < s ? t : s;
}

// (a x + b) mod p, p = 2^32 + 15, for x < 2^32 and a, b < p.  With a = a1 2^32 + a0,
// b = b1 2^32 + b0 (a1, b1 in {0, 1}) and 2^32 = -15 (mod p):
//   a x + b = (a0 x + b0) + (a1 x + b1) 2^32, and a0 x + b0 = h 2^32 + l (one
//   32 x 32 -> 64 multiply-add, below 2^64), so a x + b = l - 15 t (mod p) with
//   t = h + a1 x + b1 < 2^33.
// z = l + 32 p - 15 t lies in (0, 2^38) (15 t < 32 p); with z = z1 2^32 + z0
// (z1 < 64), r = z0 + p - 15 z1 = z (mod p) lies in [p - 945, 2^32 + p), and one
// conditional subtraction of p finishes.
__host__ __device__ inline uint64_t psi_p32(uint64_t x, uint64_t a, uint64_t b) {
    const uint64_t w = (uint64_t)(uint32_t)a * (uint32_t)x + (uint32_t)b;
    const uint64_t t = (w >> 32) + ((a >> 32) ? x : 0ull) + (b >> 32);
    const uint64_t z = (w & 0xFFFFFFFFull) + 32ull * kP32 - 15ull * t;
    const uint64_t r = (z & 0xFFFFFFFFull) + kP32 - 15ull * (z >> 32);
    return r >= kP32 ? r - kP32 : r;
}

// The narrow (32-bit) view of a permuted range that may reach past 2^32 - 1
// (R = 2^32 + 15): values at or above kNarrowTop are looked up as kNarrowTop,
// which lies in the last bin as they do (the host checks that the last bin
// starts below it), and every start above it, including the end sentinel R,
// reads as 2^32 - 1, so a value never reaches the end sentinel.  The offset
// from the bin start, below 2^32, is exact in 32-bit arithmetic.
constexpr uint32_t kNarrowTop = 0xFFFFFFFEu;
__host__ __device__ inline uint32_t narrow_value(uint64_t v) { return v > kNarrowTop ? kNarrowTop : (uint32_t)v; }
__host__ __device__ inline uint32_t narrow_start(uint64_t s) { return s > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)s; }
// R - 1 of the narrow view: the value the log-domain cells count down from.
__host__ __device__ inline uint32_t narrow_r1(uint64_t R) { return (uint32_t)(R - 1 > kNarrowTop ? kNarrowTop : R - 1); }
// Smallest 32-bit view psi_p32_narrow may give a value at or above 2^32; the
// narrow view needs the last bin to start at or below it.
constexpr uint32_t kNarrowLow = 0xFFFFFFF1u;

// The narrow view of (a x + b) mod p, p = 2^32 + 15, in 32-bit steps, for
// coefficients a, b < 2^32 (a uniform draw from [0, p) is one but for a 15 / p
// chance).  w = a x + b < 2^64 = h 2^32 + l = l - 15 h (mod p).  With
// X = h (2^32 - 15) + l = h 2^32 + (l - 15 h) (one 32 x 32 -> 64 multiply-add,
// in [0, 2^64)) and X = X1 2^32 + X0: l - 15 h = X0 - c 2^32 with c = h - X1 in
// [0, 15], so w = e (mod p) for e = X0 + 15 c < 2^32 + 240, and at most one p
// comes off.  With e0 = e mod 2^32 and g the carry out of that sum,
// t = e0 - 15 g (mod 2^32):
//   g = 0: the value is e0 = t;
//   g = 1, e0 >= 15: the value is e - p = e0 - 15 = t;
//   g = 1, e0 < 15: the value is 2^32 + e0 (low bits e0), and t wraps to
//   2^32 - 15 + e0, above e0.
// So low = min(t, e0) holds the value's low 32 bits, and view = min(t,
// kNarrowTop) its narrow view, except that the values 2^32 .. p - 1 view as
// some t in [kNarrowLow, kNarrowTop] instead of kNarrowTop: the same (last) bin
// when that bin starts at or below kNarrowLow, which the host checks.
__host__ __device__ inline void psi_p32_narrow(uint32_t x, uint32_t a, uint32_t b, uint32_t &view, uint32_t &low) {
    const uint64_t w = (uint64_t)a * x + b;
    const uint32_t h = (uint32_t)(w >> 32);
    const uint64_t X = (uint64_t)h * 0xFFFFFFF1u + (uint32_t)w;
    const uint32_t c = h - (uint32_t)(X >> 32);
    const uint32_t m = mul_u24(c, 15u);
    const uint32_t e0 = (uint32_t)X + m;
    const uint32_t t = e0 - (e0 < m ? 15u : 0u);
    low = t < e0 ? t : e0;
    view = t < kNarrowTop ? t : kNarrowTop;
}

// One region of the permuted range: its first value and the reciprocal
// M = floor(2^64 nb / z) of its size z (nb bins per region).
struct RegionEntry {
    uint64_t start, magic;
};

// Bin of the permuted value v and the first value of that bin.
//  - region: lut gives the region holding the first value of v's lookup
//    granule; later regions that start inside the granule are stepped over;
//  - bin inside the region: t = floor(y nb / z) for y = v - start; the
//    estimate floor(y M / 2^64) is t or t - 1 (y < 2^34), and one comparison
//    with the next bin start settles it.
// reg has n_regions + 1 entries (the last holds start = R); starts has k + 1.
template <typename S>
__host__ __device__ inline void locate(uint64_t v, const uint8_t *lut, uint32_t lut_shift, const RegionEntry *reg,
                                       uint32_t n_regions, uint32_t nb, const S *starts, uint32_t &bin,
                                       uint64_t &start) {
    uint32_t r = 0;
    if (n_regions > 1) {
        r = lut[v >> lut_shift];
        while (r + 1 < n_regions && v >= reg[r + 1].start) ++r;
    }
    const RegionEntry re = reg[r];
    const uint32_t b = r * nb + (uint32_t)mulhi64(v - re.start, re.magic);
    const uint64_t s0 = starts[b], s1 = starts[b + 1];
    const bool up = v >= s1;
    bin = b + (up ? 1u : 0u);
    start = up ? s1 : s0;
}

// Narrow bin lookup, for a permuted range below 2^32 - 1 (every value and start
// is 32-bit): the region as in locate(), then t' = floor(y M32 / 2^32) with
// M32 = floor(2^32 nb / z) (capped at 2^32 - 1) and y = v - start < 2^31: since
// y nb / z - y M32 / 2^32 < y / 2^32 < 1, t' is the bin t = floor(y nb / z)
// inside the region or t - 1, and the next bin start settles it.
__host__ __device__ inline void locate_narrow(uint32_t v, const uint8_t *lut, uint32_t lut_shift,
                                              const uint32_t *rstart, const uint32_t *rmag, uint32_t n_regions,
                                              uint32_t nb, const uint32_t *starts, uint32_t &bin, uint32_t &start) {
    uint32_t r = 0;
    if (n_regions > 1) {
        r = lut[v >> lut_shift];
        while (r + 1 < n_regions && v >= rstart[r + 1]) ++r;
    }
    const uint32_t y = v - rstart[r];
    const uint32_t b = mul_u24(r, nb) + (uint32_t)(((uint64_t)y * rmag[r]) >> 32);
    const uint32_t s0 = starts[b], s1 = starts[b + 1];
    const bool up = v >= s1;
    bin = b + (up ? 1u : 0u);
    start = up ? s1 : s0;
}

// Log-domain cells of a narrow permuted range, for regions that shrink
// geometrically towards the top (a:b HOPH): with u = max((R - 1 - v) >> 8, 1),
// a cell is the position e of the leading one of u and the four bits after it,
// cell = 16 e + m (at most 384 cells, non-increasing in v; every v within 511
// of the top shares cell 0).  When no cell holds two region boundaries, a
// cell's first region and its one inner boundary give the region of v with
// one comparison.  On the device the cell is read off the bits of u converted
// to f32 (exponent and the four leading mantissa bits; exact, u < 2^24).
constexpr uint32_t kLogCells = 384;

__host__ __device__ inline uint32_t clz32(uint32_t u) {
#if defined(__HIP_DEVICE_COMPILE__)
    return (uint32_t)__clz((int)u);
#else
    return u ? (uint32_t)__builtin_clz(u) : 32u;
#endif
}

__host__ __device__ inline uint32_t log_cell(uint32_t v, uint32_t R1) {
    uint32_t u = (R1 - v) >> 8;
    u = u > 1u ? u : 1u;
#if defined(__HIP_DEVICE_COMPILE__)
    return (__float_as_uint((float)u) >> 19) - 127u * 16u;
#else
    const uint32_t lz = clz32(u);
    return (31u - lz) * 16u + ((u << lz) >> 27 & 15u);
#endif
}

// Cell table entry c: {first region of the cell, start of the next region if
// it lies inside the cell, else 0xFFFFFFFF}.  reg_start has n_regions + 1
// entries (the last is R); the smallest v of a cell is found by bisection
// (the cell index does not increase with v).
template <typename Reg>
__host__ __device__ inline void log_cell_entry(uint32_t c, uint32_t R, const Reg *reg_start, uint32_t n_regions,
                                               uint32_t &first, uint32_t &bound) {
    const uint32_t R1 = R - 1;
    uint32_t lo = 0, hi = R;                 // smallest v with cell(v) <= c, or R
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (log_cell(mid, R1) <= c) hi = mid; else lo = mid + 1;
    }
    uint32_t r = 0;
    if (lo < R)
        while (r + 1 < n_regions && lo >= (uint32_t)reg_start[r + 1]) ++r;
    first = r;
    bound = 0xFFFFFFFFu;
    if (lo < R && r + 1 < n_regions && log_cell((uint32_t)reg_start[r + 1], R1) == c) bound = (uint32_t)reg_start[r + 1];
}

// Narrow bin lookup with the cell table (cells: {first, bound}) and the region
// table (regs: {start, 32-bit reciprocal}); see locate_narrow for the bin step.
// Power-of-two regions: where every region's bins are 2^s values wide (bin t
// of region r starts at s_r + t 2^s; the last one may be shorter) and every
// class of u = max(R - 1 - v, 1) with one leading-zero count lies inside one
// region (the 1:1 hierarchy over R = 2^31 - 1 splits exactly there), the
// leading-zero count of u names the region: tab[clz(u)] = {region start, s,
// first bin of the region, 2^s - 1}, and the bin and the offset are a shift
// and a mask of v minus the region start.  The host checks both conditions.
constexpr uint32_t kPow2Classes = 32;
__host__ __device__ inline void locate_pow2(uint32_t v, uint32_t R1, const uint32_t (*tab)[4], uint32_t &bin,
                                            uint32_t &off) {
    uint32_t u = R1 - v;
    u = u > 1u ? u : 1u;
    const uint32_t *e = tab[clz32(u)];
    const uint32_t d = v - e[0];
    bin = e[2] + (d >> e[1]);
    off = d & e[3];
}

__host__ __device__ inline void locate_log(uint32_t v, uint32_t R1, const uint32_t (*cells)[2],
                                           const uint32_t (*regs)[2], uint32_t nb, const uint32_t *starts,
                                           uint32_t &bin, uint32_t &start) {
    const uint32_t c = log_cell(v, R1);
    const uint32_t r = cells[c][0] + (v >= cells[c][1] ? 1u : 0u);
    const uint32_t y = v - regs[r][0];
    const uint32_t b = mul_u24(r, nb) + (uint32_t)(((uint64_t)y * regs[r][1]) >> 32);   // r < 64, nb <= 4096
    const uint32_t s0 = starts[b], s1 = starts[b + 1];
    const bool up = v >= s1;
    bin = b + (up ? 1u : 0u);
    start = up ? s1 : s0;
}

// Bin of v by the uniform estimate: est(v) is the bin of v or the one before.
__host__ __device__ inline uint32_t bin_estimate(uint64_t v, uint32_t mul, uint32_t shift) {
    return (uint32_t)(((uint64_t)(uint32_t)(v >> shift) * mul) >> 32);
}
template <typename S>
__host__ __device__ inline void locate_est(uint64_t v, uint32_t mul, uint32_t shift, const S *starts, uint32_t &bin,
                                           uint64_t &start) {
    const uint32_t b = bin_estimate(v, mul, shift);
    const uint64_t s0 = starts[b], s1 = starts[b + 1];
    const bool up = v >= s1;
    bin = b + (up ? 1u : 0u);
    start = up ? s1 : s0;
}

// ---------------------------------------------------------------------------
// Host runtime (host_tables.cpp)
// ---------------------------------------------------------------------------
hoph_status build_layout(const hoph_sketch_params &p, LayoutInfo &out, std::string &err);
bool narrow_view_ok(const LayoutInfo &L);
void fill_sketch_desc(const hoph_sketch_params &p, const LayoutInfo &lay, SketchDesc &d);
void host_lut(const LayoutInfo &lay, std::vector<uint8_t> &lut);
void host_starts(const LayoutInfo &lay, std::vector<uint64_t> &starts);
hoph_status tail_integers(uint32_t n, hoph_ratio T, hoph_ratio eps, int32_t &j_lo, int32_t &j_hi,
                          std::string &err);
hoph_status build_tables(const LayoutInfo &lay, const hoph_query_params &qp, bool goph,
                         hoph_decision_tables &out, std::string &err);
void to_scan_tab(const hoph_decision_tables &t, ScanTab &s);
// Coarse depth when the caller leaves it to the library: the first group alone
// when it rejects at least one eighth of its bins' match counts (the
// one-group pass, whose survivors are then sparse); else one group past the
// first step that has a reject cutoff, rounded up to a whole code unit of pk
// groups (a pass that stops before any step can reject keeps every pair; one
// more step settles most of the rest, and the per-survivor pass the few left);
// at most maxd.  `requested` > 0 wins, clamped to [1, maxd].  A query whose
// pass at the library's depth overflows the survivor buffer is re-run at maxd
// before it is split into sub-batches.
uint32_t default_coarse_depth(const ScanTab &tab, uint32_t requested, uint32_t maxd, uint32_t pk);

// ---------------------------------------------------------------------------
// Kernel launchers (k_*.hip).  All return hipError_t of the launch.
// ---------------------------------------------------------------------------
int device_cu_count();   // compute units of the current device (cached)
// desc[0] = a, desc[1] = b, written by a one-thread kernel in stream order (the
// values travel as kernel arguments, so no host buffer has to outlive the call).
hipError_t launch_set_desc(uint64_t *desc, uint64_t a, uint64_t b, hipStream_t st);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t value, hipStream_t st);
// Reads bytes (a multiple of 16) at p, 4096 x 256 threads; a thread may write
// its own word of sink (kSweepSinkBytes) only in a case the data never meets.
constexpr uint64_t kSweepSinkBytes = 4096ull * 256 * 4;
hipError_t launch_read_sweep(const void *p, uint64_t bytes, uint32_t *sink, hipStream_t st);
// Where the sketch of an index append also writes the new rows' code planes
// (the index's tiled layout, see k_index.hip): set i of the launch is index row
// first + i.  codes == nullptr: signatures only.
struct CodeSink {
    uint32_t *codes;
    uint64_t first, ctiles;          // ctiles = index capacity / 64
    uint32_t cu, ub;                 // code units, bins per unit
};
hipError_t launch_sketch(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets,
                         uint64_t n_sets, uint32_t *sigs, uint32_t *err_flag, hipStream_t st,
                         const CodeSink &sink = CodeSink{});
// Sketch of a batch whose size is desc[0] (at most max_sets), split into chunks of
// `chunk` ids so that uneven sets balance; prefix needs max_sets + 1 entries.
// Set ranges are clamped to the first max_ids staged ids (a malformed range is empty).
hipError_t launch_sketch_chunked(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets,
                                 const uint64_t *desc, uint64_t *prefix, uint32_t chunk, uint32_t max_sets,
                                 uint64_t max_ids, uint32_t *sigs, uint32_t *err_flag, uint32_t waves_per_cu,
                                 hipStream_t st);
// Whether the code planes of new rows have a row kernel reading each code unit
// (ub bins) as 16- or 8-byte loads (ub and k even); otherwise a plain
// per-(set, unit) kernel writes them, and the sketch of an append writes them
// from its LDS signature.
bool codes_have_row_kernel(uint32_t k, uint32_t ub);
// Code planes of index rows [first, first + n_new) from the rows themselves:
// cu code units of ub bins each.
hipError_t launch_codes_from_slab(const uint32_t *slab, uint64_t capacity, uint32_t k, uint32_t ub, uint64_t first,
                                  uint64_t n_new, uint32_t *codes, uint32_t cu, hipStream_t st);
// Copies signature rows into index rows [first, first + n_new) and, when codes
// is not null, writes the code planes of the first cu code units of ub bins
// each (layout in k_index.hip).
hipError_t launch_index_store(const uint32_t *sigs, uint64_t n_new, uint64_t first, uint32_t k, uint64_t capacity,
                              uint32_t *slab, uint32_t *codes, uint32_t ub, uint32_t cu, hipStream_t st);
hipError_t launch_pair_counts(const uint32_t *slab, uint64_t capacity, uint64_t n_sets, uint32_t kpad,
                              uint32_t kp, uint32_t L, uint32_t k, const uint32_t *qsigs, uint32_t n_q,
                              const uint32_t *pairs, uint64_t n_pairs, uint32_t policy, uint32_t *m,
                              uint32_t *e, hipStream_t st);

struct ScanLaunch {
    const uint32_t *slab;       // index rows, k words per set (see k_index.hip)
    uint64_t capacity;          // sets the slab can hold (multiple of 64)
    uint64_t n_sets;
    uint32_t kpad, kp, L, k;
    const uint32_t *qsigs;      // row-major n_q x k
    const uint64_t *qmasks;     // n_q x L empty-bin masks of the queries
    const uint32_t *codes;      // index code planes, or null: coarse pass on the 32-bit words
    const uint32_t *qcodes;     // n_q x cg x code_rec_words(kp) query code records
    uint32_t cg;                // groups with codes (index and queries)
    bool tri;                   // self-join (queries are the index rows): only set id > query row
    uint32_t q0, q1;            // query rows [q0, q1)
    uint32_t depth;             // coarse groups
    uint32_t q_per_wave;
    Survivor *surv;
    uint64_t surv_cap;
    uint64_t *keys;
    uint64_t keys_cap;
    uint64_t *counters;         // [0] survivors, [1] accepted
    const uint64_t *desc;       // nullable: desc[0] = n_q, desc[1] = n_sets, read on the device
    uint32_t waves_per_cu;      // persistent grid size with desc (0 = default)
    const double *keep_rate;    // nullable: sample_keep_rates of these records, for the first-group plan
};
// Empty-bin masks of every (query, group) and, when qcodes is not null, the code
// records (code_rec_words each) of each query's first cg groups; thr is then required.
// lin (nullable): the linear-bound words of the first lin->steps groups.
// zero (nullable): n_zero <= 256 words set to 0 by the same launch (the pass
// counters, so that no fill launch precedes the pass).
hipError_t launch_query_masks(const uint32_t *qsigs, uint32_t n_q, const uint64_t *desc, uint32_t k, uint32_t kp,
                              uint32_t L, uint64_t *out, uint32_t *qcodes, uint32_t cg, const CodeThr *thr,
                              hipStream_t st, const LinTab *lin = nullptr, uint64_t *zero = nullptr,
                              uint32_t n_zero = 0);
// Whether query records for this index and these parameters carry the words of
// the linear bound (the multi-group code pass may run at some depth); if so
// and lin is not null, its LinTab for launch_query_masks.  a needs codes, tri,
// kp, L and cg set.
bool lin_records(const ScanLaunch &a, const ScanTab &tab, LinTab *lin);
hipError_t launch_scan_coarse(const ScanLaunch &a, const ScanTab &tab, hipStream_t st);
// The first-group code pass's shape for these tables (first_group_plan):
// out[0] first-phase planes, out[1] 1 for scan_codes_fast1_kernel, out[2]
// tiles per wavefront (hoph_first_group_plan).
void first_group_shape(const ScanTab &tab, uint32_t kp, bool tri, bool small_batch, const double *keep_rate,
                       uint32_t out[3]);
// Phase-1 lane keep rates of the first-group code pass (one plane word) on the
// data, rate[p] for p = 2 .. 6, from sampled pairs of the first n_sets index
// rows' code planes and the reject thresholds dthr0 (ScanTab::dthr0);
// synchronises st.
hipError_t sample_keep_rates(const uint32_t *codes, uint64_t n_sets, uint32_t kp, const int32_t *dthr0,
                             double rate[8], hipStream_t st);
// Tiles of 64 sets one wavefront of the coarse pass holds for this launch.
uint32_t coarse_tiles_per_wave(const ScanLaunch &a, const ScanTab &tab);
// The coarse pass launch_scan_coarse runs for a: depth, HOPH_PLAN_* kernel,
// first-phase planes, tiles per wavefront (hoph_coarse_plan).
void describe_coarse(const ScanLaunch &a, const ScanTab &tab, uint32_t out[4]);
hipError_t launch_scan_fine(const ScanLaunch &a, const ScanTab &tab, hipStream_t st);
hipError_t launch_oph_full(const ScanLaunch &a, hoph_ratio T, uint32_t policy, hipStream_t st);
hipError_t launch_pair_estimates(const uint32_t *slab, uint64_t n_sets, uint32_t k, uint32_t kp, uint32_t L,
                                 const uint32_t *qsigs, uint32_t n_q, const uint32_t *pairs, uint64_t n_pairs,
                                 uint32_t policy, const double *unions, int64_t *est, uint32_t *mb, uint32_t *eb,
                                 double *var, const ScanTab &tab, hipStream_t st);
hipError_t launch_sort_keys(uint64_t *keys, uint64_t n, uint64_t n_pow2, hipStream_t st);
// counters: [1] accepted keys (read), [2] total written, [3] flags (bit 0: a query
// has more than seg_max ids, bit 1: total > out_cap).  desc (nullable): desc[0] =
// n_q.  seg_max: ids per query sorted in LDS, a power of two in [2, 16384].
constexpr uint32_t kSegMaxPlan = 4096;
hipError_t launch_segmented_output(const uint64_t *keys, const uint64_t *counters_ro, uint64_t keys_cap,
                                   uint32_t *qcount, const uint64_t *desc, uint32_t n_q, uint64_t *offsets,
                                   uint64_t *cursor, uint32_t *ids, uint64_t out_cap, uint64_t *counters,
                                   uint32_t max_queries, uint64_t max_keys, uint32_t seg_max, hipStream_t st);
// The output stage in one workgroup for a batch of up to kSmallOutKeys
// accepted keys (counters[1], read on the device): the same CSR, counters[2]
// and counters[3] bit 1 as launch_segmented_output; with more keys it writes
// nothing but counters[3] = 4 (run launch_segmented_output then).  desc
// (nullable): desc[0] = n_q, read on the device.
constexpr uint32_t kSmallOutKeys = 2048;
constexpr uint32_t kSmallOutQueries = 4096;
hipError_t launch_small_output(const uint64_t *keys, uint64_t *counters, uint64_t keys_cap, const uint64_t *desc,
                               uint32_t n_q, uint64_t *offsets, uint32_t *ids, uint64_t out_cap, hipStream_t st);
hipError_t launch_results(const uint64_t *keys, uint64_t n, uint32_t n_q, uint64_t *offsets,
                          uint32_t *set_ids, hipStream_t st);
hipError_t launch_minwise_sketch(uint32_t k, uint32_t hash, uint64_t universe, const uint64_t *ha,
                                 const uint64_t *hb, const uint32_t *ids, const uint64_t *offsets,
                                 uint64_t n_sets, uint64_t *sigs, uint32_t *err_flag,
                                 hipStream_t st);
hipError_t launch_minwise_scan(uint32_t k, const uint64_t *sigs, uint64_t n_sets,
                               const uint64_t *qsigs, uint32_t q0, uint32_t q1, hoph_ratio T,
                               uint64_t *keys, uint64_t keys_cap, uint64_t *counters,
                               hipStream_t st);

}  // namespace hoph
