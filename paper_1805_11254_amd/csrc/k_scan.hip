// The grouped comparison of Alg. 1 (GOPH) and Alg. 2 ((a:b) HOPH): matched
// and empty bins are counted group by group (Eqs. 1-4), the per-group rate
// (Eq. 6) is added to an exact weighted state, and the pair stops as soon as
// the small-probability event of Def. 1 decides it.  The per-step tests are
// precomputed on the host as integer cutoffs on the state, so the device only
// counts, multiplies, adds and compares integers.
//
// Coarse pass: one wavefront per (tile(s) of 64 indexed sets, chunk of
// queries), one set per lane, every query word a scalar load.  By default it
// compares 8-bit bin codes held as bit-planes and only rejects
// (scan_codes_fast_kernel for the first group, in two phases of planes;
// scan_codes_kernel for up to 4 code units in VGPRs, a unit being one group or
// several small ones sharing plane words; scan_codes_deep_kernel past that,
// later units staged in LDS); on request it compares the 32-bit words and
// accepts too (scan_coarse_kernel: with G = 1 the decision after the first
// group is a pair of thresholds on the matched count, with G > 1 the exact
// 64-bit state is carried).  Pairs not rejected are appended to a survivor
// list: the code passes gather a wavefront's survivors in LDS and append them
// in batches (one atomic per batch), the word pass with one atomic per
// wavefront and step (ballot + rank).
//
// Fine pass: one wavefront per survivor; floor(64 / k') groups side by side
// across the lanes of a load (one lane per bin) and two to four loads per
// step; counts come from ballots and popcounts, the decision is wave-uniform,
// and the wavefront leaves at the first deciding group.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hoph_internal.h"

namespace hoph {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kFineAhead = 4;          // most loads per step in the fine pass (k' > 32; else 2)
// Tiles of 64 sets per wavefront in the first-group code pass: eight for the
// two-plane first phase over one plane word (its registers hold 8 planes of 8
// tiles), else four (two with two plane words).
constexpr int fast_tiles(int W, int P1) { return W == 1 ? (P1 == 2 ? 8 : 4) : 2; }
// Tiles per wavefront of the first-group pass that keeps only its first-phase
// planes in VGPRs (one plane word): 16 for up to three planes, else 8.
constexpr int fast1_tiles(int P1) { return P1 <= 3 ? 16 : 8; }
// The first-group pass's shape: planes of phase 1 (0: one phase), whether it
// runs in scan_codes_fast1_kernel, and its tiles per wavefront.
struct FirstGroupPlan {
    int planes;
    bool fast1;
    int tiles;
};

// Planes compared first in the first-group code pass, and its kernel.  A
// background pair (independent, uniform codes) agrees on a query-non-empty
// bin's first p planes with probability 2^-p, so phase 1 keeps one of its
// lanes when at least kp - thr + 1 of the kp bins agree there (a binomial
// tail), and a wavefront goes on to phase 2 when any of its 64 TPW lanes is
// kept.  Expected lane-ops per pair, with constants fitted to the measured
// rates of both kernels: scan_codes_fast_kernel (every plane in VGPRs)
// W p + 2 (W p + 2.4 with 8 tiles), plus W (8 - p) + 2 in phase 2, one phase
// over all 8 planes 8 W + 3; scan_codes_fast1_kernel (one plane word; only
// the first p planes in VGPRs, so twice the tiles) p + 1.6, plus about p + 10
// in phase 2 (phase 1 again for the tiles, then the kept tiles' planes read
// again).  The least of these is taken.  A batch of fewer than
// kFast1MinQueries queries (known on the host) keeps the kernel with more
// wavefronts: there the pass is bound by reading the planes, and twice the
// tiles per wavefront halve the wavefronts that read them.
//
// keep_rate (nullable): the lane keep rate of each p measured on sampled pairs
// of the data (sample_keep_rates), taken where it exceeds the binomial tail:
// sets that share common elements agree on more bins than independent codes.
// In a self-join each tile of scan_codes_fast1_kernel kept beyond the
// binomial rate (which the fitted constants cover) also costs the wait for
// its planes read again, about kRereadCost lane-ops per pair of that tile
// (fitted to a self-join of 10^6 rows where 1.6% of the tiles kept a lane at
// p = 2: 2.5 times the time at p = 3; a wavefront there works through
// thousands of queries per item, and its tiles' planes have left the caches
// when they are read again; with a query batch the same kept-tile rate cost
// less than the phase-2 term above).  A self-join (tri) with one
// plane word runs scan_codes_fast1_kernel unless even its best plane count
// costs more than one phase over all planes: the rows' records stream from
// memory through the scalar unit, and that kernel shares each record over
// twice the tiles (measured 1.5 to 1.7 times faster than
// scan_codes_fast_kernel at 2, 3 and 4 planes on that self-join).
constexpr uint32_t kFast1MinQueries = 32;
constexpr double kRereadCost = 520.0;
FirstGroupPlan first_group_plan(const ScanTab &tab, uint32_t kp, bool tri, bool small_batch,
                                const double *keep_rate) {
    const int32_t k = (int32_t)kp, need = k - tab.dthr0[0] + 1;   // agreeing bins that keep a lane
    const int W = (int)code_plane_words(kp);
    const bool light = W == 1 && !small_batch;                     // scan_codes_fast1_kernel may run
    const bool light_only = light && tri;
    FirstGroupPlan best{0, false, fast_tiles(W, 0)};
    double best_cost = 8.0 * W + 3.0;
    FirstGroupPlan best1{0, false, 0};
    double best1_cost = HUGE_VAL;
    for (int p = 2; p <= 6; ++p) {
        const double f = std::ldexp(1.0, -p);
        double tail = need <= 0 ? 1.0 : 0.0, term = std::pow(1.0 - f, k);   // P(j = 0)
        for (int j = 0; j <= k && need > 0; ++j) {
            if (j >= need) tail += term;
            term *= (double)(k - j) / (double)(j + 1) * f / (1.0 - f);
        }
        const double keep0 = 1.0 - std::min(tail, 1.0);
        const double lane = keep_rate ? std::max(tail, keep_rate[p]) : tail;
        const double keep = 1.0 - std::min(lane, 1.0);
        if (!light_only) {
            const double open = 1.0 - std::pow(keep, 64.0 * fast_tiles(W, p));
            const double cost = W * p + (fast_tiles(W, p) == 8 ? 2.4 : 2.0) + open * (W * (8 - p) + 2.0);
            if (cost < best_cost) {
                best_cost = cost;
                best = FirstGroupPlan{p, false, fast_tiles(W, p)};
            }
        }
        if (light) {
            const double open1 = 1.0 - std::pow(keep, 64.0 * fast1_tiles(p));
            double cost1 = p + 1.6 + open1 * (p + 10.0);
            if (tri) cost1 += (std::pow(keep0, 64.0) - std::pow(keep, 64.0)) * kRereadCost;
            if (cost1 < best1_cost) {
                best1_cost = cost1;
                best1 = FirstGroupPlan{p, true, fast1_tiles(p)};
            }
        }
    }
    // (with light_only, best is still the one-phase pass and best_cost its cost)
    if (best1.fast1 && best1_cost < best_cost) return best1;
    return best;
}


struct CoarseArgs {
    uint64_t capacity, n_sets, surv_cap, keys_cap;
    uint32_t k, kp, kpad, L, q0, q1, q_per_wave, policy, depth, cg;
    uint32_t tri;        // self-join: only pairs with set id > query row
    uint32_t pk;         // groups per code unit
    uint32_t cdepth;     // groups the code pass walks
};

__device__ __forceinline__ uint32_t wave_id_in_block() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ uint64_t lane_rank(uint64_t mask, uint32_t lane) {
    return __popcll(mask & ((1ull << lane) - 1ull));
}

// Queries per (tile, query chunk) work item.  A plan's kernels read the batch
// size from the descriptor, so the tuned chunk is raised here to the whole
// batch up to kChunkQueries (a batch split into chunks reads the planes once per
// chunk).  Never 0 (a.q_per_wave >= 1).
__device__ __forceinline__ uint32_t chunk_queries(const CoarseArgs &a, const uint64_t *desc, uint32_t nq) {
    return desc ? max(a.q_per_wave, min(nq, kChunkQueries)) : a.q_per_wave;
}

// Append the lanes with `flag` set: one atomic per wavefront.  Returns the slot
// of this lane (valid only where flag is set).  Call with the whole wave active.
__device__ __forceinline__ uint64_t wave_append(bool flag, unsigned long long *counter, uint32_t lane) {
    const uint64_t bal = __ballot(flag);
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd(counter, (unsigned long long)__popcll(bal));
    base = __shfl(base, 0);
    return base + lane_rank(bal, lane);
}

// Orders one wavefront's LDS accesses across its lanes.
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// A wavefront's survivors gathered in its own LDS buffer and appended to the
// list in batches of up to N: one atomic on the counter per batch.  One atomic
// per (query, tile) that has a survivor serialises on the counter when
// survivors are spread thinly over many (query, tile) items (about 12 ns each:
// 2.5 ms for the 2*10^5 survivors of 3*10^8 pairs).  The order of the list is
// not specified (the output is sorted per query).  Every call with the whole
// wave active; `n` is wave-uniform.
template <uint32_t N>
struct SurvBatch {
    Survivor *buf;                   // this wavefront's N entries in LDS
    uint32_t n;

    __device__ __forceinline__ void flush(Survivor *__restrict__ surv, uint64_t cap, unsigned long long *counter,
                                          uint32_t lane) {
        if (n == 0) return;
        wave_lds_fence();
        uint64_t base = 0;
        if (lane == 0) base = atomicAdd(counter, (unsigned long long)n);
        base = __shfl(base, 0);
        for (uint32_t j = lane; j < n; j += 64)
            if (base + j < cap) surv[base + j] = buf[j];
        wave_lds_fence();
        n = 0;
    }
    // bal: the surviving lanes (wave-uniform); this lane's pair is (q, s).
    __device__ __forceinline__ void push(uint64_t bal, uint32_t q, uint32_t s, Survivor *__restrict__ surv,
                                         uint64_t cap, unsigned long long *counter, uint32_t lane) {
        const uint32_t c = (uint32_t)__popcll(bal);
        if (c == 0) return;
        if (n + c > N) flush(surv, cap, counter, lane);
        if ((bal >> lane) & 1ull) buf[n + (uint32_t)lane_rank(bal, lane)] = Survivor{q, s, 0};
        n += c;
    }
};
constexpr uint32_t kSurvBatch = 128;       // per wavefront: 2 KB of LDS
constexpr uint32_t kSurvBatchDeep = 64;    // the deep pass's LDS is mostly its staging

// One group of one set row (row-major words) into registers; pad words
// (k' not a multiple of 4) read as EMPTY.  16-byte loads when k' and k are
// multiples of 4 (EXACT and vec).
template <int KPAD, bool EXACT>
__device__ __forceinline__ void load_group_row(const uint32_t *__restrict__ row, uint32_t kp, bool vec,
                                               uint32_t (&w)[KPAD]) {
    if (EXACT && vec) {
        const uint4 *r4 = reinterpret_cast<const uint4 *>(row);
#pragma unroll
        for (int qd = 0; qd < KPAD / 4; ++qd) {
            const uint4 v = r4[qd];
            w[4 * qd + 0] = v.x;
            w[4 * qd + 1] = v.y;
            w[4 * qd + 2] = v.z;
            w[4 * qd + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < KPAD; ++i) w[i] = (EXACT || i < (int)kp) ? row[i] : HOPH_EMPTY;
    }
}

// lambda * rate of one group (Eq. 6 per group) from the counts.
__device__ __forceinline__ int64_t group_rho(uint32_t eq, uint32_t ej, uint32_t ee, uint32_t kp, uint32_t policy,
                                             const int64_t *dmul, int64_t lambda) {
    const uint32_t m = eq - ej;                 // equal and non-empty
    if (policy == HOPH_EMPTY_LITERAL) return (int64_t)m;
    const uint32_t e = policy == HOPH_EMPTY_JOINT ? ej : ee;
    if (e == kp) return ej == kp ? lambda : 0;  // 0/0: 1 iff the group is empty in both
    return (int64_t)m * dmul[e];
}

// Bits of the EMPTY words among w[0 .. n), n <= 64; with vec (n a multiple of
// 4, w 16-byte aligned) read as 16-byte words, four loads issued together.
__device__ __forceinline__ uint64_t empty_bits(const uint32_t *__restrict__ w, uint32_t n, bool vec) {
    uint64_t m = 0;
    if (vec) {
        const uint4 *w4 = reinterpret_cast<const uint4 *>(w);
#pragma unroll 4
        for (uint32_t j = 0; j < n / 4; ++j) {
            const uint4 v = w4[j];
            const uint32_t b = (uint32_t)(v.x == HOPH_EMPTY) | (uint32_t)(v.y == HOPH_EMPTY) << 1 |
                               (uint32_t)(v.z == HOPH_EMPTY) << 2 | (uint32_t)(v.w == HOPH_EMPTY) << 3;
            m |= (uint64_t)b << (4 * j);
        }
    } else {
        for (uint32_t i = 0; i < n; ++i) m |= (uint64_t)(w[i] == HOPH_EMPTY) << i;
    }
    return m;
}

// Code planes of the ub <= 64 bins at w: bit b & 31 of lo[p] (b < 32) or hi[p]
// (b >= 32) is bit p of bin b's code; 16-byte reads with vec as above.
__device__ __forceinline__ void code_planes_of(const uint32_t *__restrict__ w, uint32_t ub, bool vec,
                                               uint32_t (&lo)[kCodeBits], uint32_t (&hi)[kCodeBits]) {
#pragma unroll
    for (int p = 0; p < (int)kCodeBits; ++p) lo[p] = hi[p] = 0;
    auto put = [&](uint32_t v, uint32_t b) {
        const uint32_t c = bin_code(v), bit = b & 31;
        if (b < 32) {
#pragma unroll
            for (int p = 0; p < (int)kCodeBits; ++p) lo[p] |= ((c >> p) & 1u) << bit;
        } else {
#pragma unroll
            for (int p = 0; p < (int)kCodeBits; ++p) hi[p] |= ((c >> p) & 1u) << bit;
        }
    };
    if (vec) {
        const uint4 *w4 = reinterpret_cast<const uint4 *>(w);
#pragma unroll 4
        for (uint32_t j = 0; j < ub / 4; ++j) {
            const uint4 v = w4[j];
            put(v.x, 4 * j);
            put(v.y, 4 * j + 1);
            put(v.z, 4 * j + 2);
            put(v.w, 4 * j + 3);
        }
    } else {
        for (uint32_t b = 0; b < ub; ++b) put(w[b], b);
    }
}

// Empty-bin mask of every (query, group): bit i set when bin i of the group is
// EMPTY; for the first cg groups also the query's code record: the planes of
// the group's code unit (same word order as the index's: plane p of the unit's
// bins [32 w, 32 w + 32) at p * W + w; every group of a unit holds the same
// planes), the group's non-empty mask (bits from 0), the first group's keep
// threshold on codes (a pair is kept when more than this many of the query's
// non-empty bins have equal codes: (k' - e) - ScanTab::dthr0[e], negative when
// the first group rejects nothing) and the group's empty count e.  A group
// with a record takes its empty mask from the planes (code 255, every plane
// set, is EMPTY and nothing else); rows are read as 16-byte words when k and
// k' are multiples of 4, and each record is written as 16-byte words.
__global__ __launch_bounds__(kThreads) void query_masks_kernel(const uint32_t *__restrict__ qsigs, uint32_t n_q_arg,
                                                              const uint64_t *__restrict__ desc, uint32_t k,
                                                              uint32_t kp, uint32_t L, uint64_t *__restrict__ out,
                                                              uint32_t *__restrict__ qcodes, uint32_t cg,
                                                              const CodeThr thr, const LinTab lin,
                                                              uint64_t *__restrict__ zero, uint32_t n_zero) {
    if (zero && blockIdx.x == 0 && threadIdx.x < n_zero) zero[threadIdx.x] = 0;   // the pass counters
    const uint32_t n_q = desc ? (uint32_t)desc[0] : n_q_arg;
    const uint64_t n = (uint64_t)n_q * L;
    const uint32_t W = code_plane_words(kp), PW = code_words(kp), RW = code_rec_words(kp);
    const uint32_t pk = code_pack(kp, L), ub = pk * kp;
    const uint64_t kpmask = kp >= 64 ? ~0ull : ((1ull << kp) - 1ull);
    const bool vec = (k % 4 == 0) && (kp % 4 == 0) && ((reinterpret_cast<uintptr_t>(qsigs) & 15) == 0);
    for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < n; t += (uint64_t)gridDim.x * kThreads) {
        const uint64_t q = t / L, g = t % L;
        const uint32_t *row = qsigs + q * k;
        if (!(qcodes && g < cg)) {
            out[t] = empty_bits(row + g * kp, kp, vec);
            continue;
        }
        uint32_t lo[kCodeBits], hi[kCodeBits];
        code_planes_of(row + (g / pk) * ub, ub, vec, lo, hi);  // the group's code unit (cg <= L / pk * pk)
        uint32_t elo = lo[0], ehi = hi[0];
#pragma unroll
        for (int p = 1; p < (int)kCodeBits; ++p) {
            elo &= lo[p];
            ehi &= hi[p];
        }
        const uint64_t m = ((((uint64_t)ehi << 32) | elo) >> ((g % pk) * kp)) & kpmask;
        out[t] = m;
        uint32_t rec[2 * kCodeBits + 8];         // code_rec_words for two plane words
#pragma unroll
        for (int p = 0; p < (int)kCodeBits; ++p) {
            rec[p * W] = lo[p];
            if (W == 2) rec[p * W + 1] = hi[p];
        }
        const uint64_t nqm = ~m & kpmask;
        const uint32_t e = (uint32_t)__popcll(m);
        rec[PW + 0] = (uint32_t)nqm;
        rec[PW + 1] = (uint32_t)(nqm >> 32);
        rec[PW + 2] = (uint32_t)((int32_t)(kp - e) - thr.dthr[e]);   // keep iff more agreeing bins
        rec[PW + 3] = e;
        uint32_t lc = 0, lz = 0xFFFFFFFFu, ly = 0x7FFFFFFFu;
        if (g < lin.steps) {
            // linear bound of step g (see LinTab): sums over this query's groups 0..g
            int64_t sum_ck = 0, sum_cn = 0;
            for (uint32_t h = 0; h <= g; ++h) {
                const uint32_t eh = h == g ? e : (uint32_t)__popcll(empty_bits(row + h * kp, kp, vec));
                int64_t c, ck;
                if (lin.policy == HOPH_EMPTY_LITERAL) {
                    c = eh < kp ? lin.W[h] : 0;
                    ck = lin.W[h] * (int64_t)(kp - eh);
                } else {                      // JOINT: C (k' - e) = W lambda
                    c = eh < kp ? lin.W[h] * lin.dmul[eh] : 0;
                    ck = lin.W[h] * lin.lambda;
                }
                sum_ck += ck;
                const int64_t ch = c >> lin.shift;
                sum_cn += ch * (int64_t)(kp - eh);
                if (h == g) lc = (uint32_t)ch;
            }
            // the tests on st = sum c_h dn_h, restated on the agreeing counts
            // st' = sum c_h (k' - e_h - dn_h) = sum_cn - st (below 2^31)
            const int64_t one = (int64_t)1 << lin.shift;
            if (lin.rej[g] >= 0) {
                const int64_t Z = sum_ck - lin.rej[g];
                const int64_t zc = Z <= 0 ? 0 : (Z + one - 1) >> lin.shift;   // reject: st >= zc
                lz = zc <= sum_cn ? (uint32_t)(sum_cn - zc) : 0xFFFFFFFFu;
            }
            const int64_t Y = sum_ck - lin.acc[g];
            if (Y >= 0) ly = (uint32_t)(int32_t)(sum_cn - min<int64_t>(Y >> lin.shift, sum_cn + 0x7FFFFFFFll));
        }
        rec[PW + 4] = lc;
        rec[PW + 5] = lz;
        rec[PW + 6] = ly;
        rec[PW + 7] = 0;
        uint4 *dst = reinterpret_cast<uint4 *>(qcodes + (q * cg + g) * RW);   // RW is a multiple of 4
        if (W == 1) {
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[j] = make_uint4(rec[4 * j], rec[4 * j + 1], rec[4 * j + 2], rec[4 * j + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < 6; ++j) dst[j] = make_uint4(rec[4 * j], rec[4 * j + 1], rec[4 * j + 2], rec[4 * j + 3]);
        }
    }
}

// Bins of one group whose codes differ, as a bit mask per 32 bins: the XOR of
// plane 0, then (acc | (set plane ^ query plane)) for the other planes in one
// three-input bit operation each (truth table 0xF6 = F0 | (CC ^ AA)).
template <int W>
__device__ __forceinline__ uint32_t code_diff(const uint32_t *P, const uint32_t *__restrict__ Q, int w) {
    uint32_t d = P[w] ^ Q[w];
#pragma unroll
    for (int p = 1; p < (int)kCodeBits; ++p) d = __builtin_amdgcn_bitop3_b32(d, P[p * W + w], Q[p * W + w], 0xF6);
    return d;
}

// The agreeing-bin mask of the query's non-empty bins over planes [P0, P1),
// continuing the chain from a; at P0 = 0 the chain starts from the query's
// non-empty mask m instead.  A bin's bit stays set while each plane so far
// agrees, so the popcount over all planes counts the query-non-empty bins
// with equal codes.  One three-input bit operation per plane: 0x82 =
// m & ~(P ^ Q) for plane 0, 0x90 = a & ~(P ^ Q) after it.
template <int W, int P0, int P1>
__device__ __forceinline__ uint32_t code_agree_part(uint32_t a, uint32_t m, const uint32_t *P,
                                                    const uint32_t *__restrict__ Q, int w) {
#pragma unroll
    for (int p = P0; p < P1; ++p)
        a = p == 0 ? __builtin_amdgcn_bitop3_b32(P[w], Q[w], m, 0x82)
                   : __builtin_amdgcn_bitop3_b32(a, P[p * W + w], Q[p * W + w], 0x90);
    return a;
}

// The differing-bin mask over planes [P0, P1) only, continuing the chain from d
// (d is ignored when P0 = 0).  A mask over the first planes is a subset of the
// mask over all of them.
template <int W, int P0, int P1>
__device__ __forceinline__ uint32_t code_diff_part(uint32_t d, const uint32_t *P, const uint32_t *__restrict__ Q,
                                                   int w) {
#pragma unroll
    for (int p = P0; p < P1; ++p)
        d = p == 0 ? (P[w] ^ Q[w]) : __builtin_amdgcn_bitop3_b32(d, P[p * W + w], Q[p * W + w], 0xF6);
    return d;
}

// One group of the coarse pass on codes: bits [o, o + k') of its code unit's
// differing-code mask d and set-empty mask em (o = 0 unless small groups share
// a unit) against the query's empty mask qm of the group, added to the
// weighted state S, and the step's cutoffs applied to a lane still undecided
// (maybe: an accept cutoff was reached, so the pair must go on to the fine
// pass).  UNITW: every weight is 1 (GOPH), no multiply.
template <int W, bool UNITW>
__device__ __forceinline__ void code_group_step(const uint32_t (&d)[W], const uint32_t *em, uint32_t o, uint64_t qm,
                                                uint64_t kpmask, uint32_t kp, uint32_t policy, const int64_t *s_dmul,
                                                int64_t lambda, int64_t Wg, int64_t accg, int64_t rejg, int64_t &S,
                                                bool &undecided, bool &maybe) {
    const uint64_t nqm = ~qm & kpmask;
    uint32_t dn = 0, de = 0, ee = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t qmw = (uint32_t)(qm >> (32 * w)) << o, nqmw = (uint32_t)(nqm >> (32 * w)) << o;
        const uint32_t gmw = (uint32_t)(kpmask >> (32 * w)) << o;
        dn += __popc(d[w] & nqmw);
        de += __popc(d[w] & qmw);
        ee += __popc((em[w] & gmw) | qmw);
    }
    const uint32_t eq_q = (uint32_t)__popcll(qm);
    const uint32_t m = kp - eq_q - dn;        // >= the matched non-empty bins
    const uint32_t ej = eq_q - de;            // jointly empty bins, exact
    const int64_t rho = group_rho(m + ej, ej, ee, kp, policy, s_dmul, lambda);
    if constexpr (UNITW) S += rho;
    else S += Wg * rho;
    if (undecided) {
        if (S >= accg) {
            maybe = true;
            undecided = false;
        } else if (S <= rejg) {
            undecided = false;
        }
    }
}

// The groups of code unit u (planes P, set-empty masks em) for one query, up
// to group cd: the unit's differing-code mask is formed once and each of its
// groups (pk of them; one without PACK) takes its own bits.
template <int W, bool PACK, bool UNITW>
__device__ __forceinline__ void code_unit_steps(uint32_t u, const uint32_t *P, const uint32_t *em,
                                                const uint32_t *__restrict__ qc, const uint64_t *__restrict__ qmk,
                                                uint32_t pk, uint32_t cd, uint64_t kpmask, uint32_t kp,
                                                uint32_t policy, const int64_t *s_dmul, const ScanTab &tab,
                                                int64_t &S, bool &undecided, bool &maybe) {
    constexpr int RW = (int)kCodeBits * W + 8;           // record stride (code_rec_words)
    const uint32_t g0 = PACK ? u * pk : u;
    uint32_t d[W];
#pragma unroll
    for (int w = 0; w < W; ++w) d[w] = code_diff<W>(P, qc + (uint64_t)g0 * RW, w);
    if constexpr (PACK) {
        for (uint32_t j = 0, g = g0; j < pk && g < cd; ++j, ++g) {
            if (j > 0 && !__any(undecided)) break;
            code_group_step<W, UNITW>(d, em, j * kp, qmk[g], kpmask, kp, policy, s_dmul, tab.lambda, tab.W[g], tab.acc[g],
                               tab.rej[g], S, undecided, maybe);
        }
    } else {
        code_group_step<W, UNITW>(d, em, 0u, qmk[g0], kpmask, kp, policy, s_dmul, tab.lambda, tab.W[g0], tab.acc[g0],
                           tab.rej[g0], S, undecided, maybe);
    }
}

// Coarse pass on codes (reject-only).  Same (tile, query chunk) items as the
// word kernel below; the tile's code planes of the first G code units stay in
// VGPRs.  Codes never under-count matched bins (equal values have equal codes)
// and count empty bins exactly (EMPTY has a code of its own), and the per-step
// cutoffs are monotone in the matched count, so a pair is dropped here only
// where the exact algorithm rejects it too: at a step whose code state is at or
// below the reject cutoff, with no earlier step at or above an accept cutoff.
// Every other pair goes to the fine pass, which restarts from the first group
// on the 32-bit words.  PACK: units of several small groups, walked up to group
// a.cdepth; UNITW: every weight up to that depth is 1.  (Depth 1 under JOINT or
// LITERAL runs in scan_codes_fast_kernel instead.)
template <int W, int G, bool PACK, bool UNITW>
__global__ __launch_bounds__(kThreads) void scan_codes_kernel(const uint32_t *__restrict__ codes,
                                                             const uint32_t *__restrict__ qcodes,
                                                             const uint64_t *__restrict__ qmasks,
                                                             Survivor *__restrict__ surv,
                                                             unsigned long long *__restrict__ counters,
                                                             const uint64_t *__restrict__ desc,
                                                             const CoarseArgs a, const ScanTab tab) {
    constexpr int PW = (int)kCodeBits * W, RW = PW + 8;     // RW: record stride (code_rec_words)
    __shared__ int64_t s_dmul[HOPH_MAX_KGROUP + 1];
    for (uint32_t i = threadIdx.x; i <= tab.kp; i += kThreads) s_dmul[i] = tab.dmul[i];
    __syncthreads();

    __shared__ Survivor s_surv[kWaves][kSurvBatch];
    const uint32_t lane = threadIdx.x & 63;
    SurvBatch<kSurvBatch> sb{s_surv[wave_id_in_block()], 0};
    const uint64_t n_sets = desc ? desc[1] : a.n_sets;
    const uint32_t q_lo = desc ? 0u : a.q0, q_hi = desc ? (uint32_t)desc[0] : a.q1;
    const uint32_t qpw = chunk_queries(a, desc, q_hi - q_lo);
    const uint64_t ntiles = (n_sets + 63) / 64;
    const uint32_t nchunks = (q_hi - q_lo + qpw - 1) / qpw;
    const uint64_t n_items = ntiles * nchunks;
    const uint64_t wstride = (uint64_t)gridDim.x * kWaves;
    const uint32_t kp = a.kp, pk = a.pk, cd = a.cdepth;
    const uint64_t kpmask = kp >= 64 ? ~0ull : ((1ull << kp) - 1ull);
    const uint64_t ctiles = a.capacity / 64;
    const uint32_t policy = a.policy;
    for (uint64_t item = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); item < n_items; item += wstride) {
    const uint64_t tile = item % ntiles;
    const uint32_t chunk = (uint32_t)(item / ntiles);
    // self-join: skip (before any load) a tile with no set id above the chunk's first query row
    if (a.tri && tile * 64 + 63 <= (uint64_t)q_lo + (uint64_t)chunk * qpw) continue;
    const uint64_t s = tile * 64 + lane;
    const bool valid = s < n_sets;

    uint32_t P[G][PW];
    uint32_t em[G][W];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const uint4 *src = reinterpret_cast<const uint4 *>(codes + (((uint64_t)u * ctiles + tile) * 64 + lane) * PW);
#pragma unroll
        for (int j = 0; j < PW / 4; ++j) {
            const uint4 v = src[j];
            P[u][4 * j + 0] = v.x;
            P[u][4 * j + 1] = v.y;
            P[u][4 * j + 2] = v.z;
            P[u][4 * j + 3] = v.w;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            // set-empty bins: code 0xFF, every plane set
            uint32_t e = P[u][w];
#pragma unroll
            for (int p = 1; p < (int)kCodeBits; ++p) e &= P[u][p * W + w];
            em[u][w] = e;
        }
    }

    const uint32_t qa = q_lo + chunk * qpw;
    const uint32_t qb = min(q_hi, qa + qpw);
    for (uint32_t q = qa; q < qb; ++q) {
        const uint32_t *qc = qcodes + (uint64_t)q * a.cg * RW;
        const uint64_t *qmk = qmasks + (uint64_t)q * a.L;
        bool survive;
        {
            int64_t S = 0;
            bool undecided = valid && (!a.tri || s > q), maybe = false;
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (!__any(undecided)) break;
                code_unit_steps<W, PACK, UNITW>((uint32_t)u, P[u], em[u], qc, qmk, pk, cd, kpmask, kp, policy, s_dmul,
                                                tab, S, undecided, maybe);
            }
            survive = maybe || undecided;
        }
        sb.push(__ballot(survive), q, (uint32_t)s, surv, a.surv_cap, counters + 0, lane);
    }
    }
    sb.flush(surv, a.surv_cap, counters + 0, lane);
}

// Coarse pass on codes deeper than the register-resident units (GOPH with
// small groups or a low threshold, whose first useful rejecting step comes
// many groups in).  One wavefront per block, one (tile, query chunk) item at a
// time.  The first R code units of the tile (R <= cu) stay in VGPRs as in
// scan_codes_kernel; the later ones (up to unit cu) are staged in LDS unit by
// unit, the first time a query of the chunk reaches that unit (each lane only
// reads back its own words, so the wavefront's program order is the only
// ordering needed).  Each query walks the groups, up to group a.cdepth, until
// every lane is decided.
template <int W, bool PACK, int R, bool UNITW>
__global__ __launch_bounds__(64) void scan_codes_deep_kernel(const uint32_t *__restrict__ codes,
                                                           const uint32_t *__restrict__ qcodes,
                                                           const uint64_t *__restrict__ qmasks,
                                                           Survivor *__restrict__ surv,
                                                           unsigned long long *__restrict__ counters,
                                                           const uint64_t *__restrict__ desc, const CoarseArgs a,
                                                           const ScanTab tab, uint32_t cu) {
    constexpr int PW = (int)kCodeBits * W, RW = PW + 8, PV = PW / 4;     // RW: record stride
    extern __shared__ uint4 s_pl[];      // units >= R: [unit - R][PV][lane] planes, then [unit - R][W][lane] masks
    __shared__ int64_t s_dmul[HOPH_MAX_KGROUP + 1];
    __shared__ Survivor s_surv[kSurvBatchDeep];
    SurvBatch<kSurvBatchDeep> sb{s_surv, 0};
    uint32_t *s_em = reinterpret_cast<uint32_t *>(s_pl + (size_t)(cu - R) * PV * 64);
    for (uint32_t i = threadIdx.x; i <= tab.kp; i += 64) s_dmul[i] = tab.dmul[i];
    __syncthreads();

    const uint32_t lane = threadIdx.x;
    const uint64_t n_sets = desc ? desc[1] : a.n_sets;
    const uint32_t q_lo = desc ? 0u : a.q0, q_hi = desc ? (uint32_t)desc[0] : a.q1;
    const uint32_t qpw = chunk_queries(a, desc, q_hi - q_lo);
    const uint64_t ntiles = (n_sets + 63) / 64;
    const uint32_t nchunks = (q_hi - q_lo + qpw - 1) / qpw;
    const uint64_t n_items = ntiles * nchunks;
    const uint32_t kp = a.kp, pk = a.pk, cd = a.cdepth;
    const uint64_t kpmask = kp >= 64 ? ~0ull : ((1ull << kp) - 1ull);
    const uint64_t ctiles = a.capacity / 64;
    const uint32_t policy = a.policy;
    for (uint64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const uint64_t tile = item % ntiles;
        const uint32_t chunk = (uint32_t)(item / ntiles);
        const uint32_t qa = q_lo + chunk * qpw;
        // self-join: skip a tile with no set id above the chunk's first query row
        if (a.tri && tile * 64 + 63 <= (uint64_t)qa) continue;
        const uint32_t qb = min(q_hi, qa + qpw);
        const uint64_t s = tile * 64 + lane;
        const bool valid = s < n_sets;

        uint32_t P[R][PW], em[R][W];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const uint4 *src = reinterpret_cast<const uint4 *>(codes + (((uint64_t)u * ctiles + tile) * 64 + lane) * PW);
#pragma unroll
            for (int j = 0; j < PV; ++j) {
                const uint4 v = src[j];
                P[u][4 * j + 0] = v.x;
                P[u][4 * j + 1] = v.y;
                P[u][4 * j + 2] = v.z;
                P[u][4 * j + 3] = v.w;
            }
#pragma unroll
            for (int w = 0; w < W; ++w) {
                // set-empty bins: code 0xFF, every plane set
                uint32_t e = P[u][w];
#pragma unroll
                for (int p = 1; p < (int)kCodeBits; ++p) e &= P[u][p * W + w];
                em[u][w] = e;
            }
        }

        uint32_t staged = R;
        for (uint32_t q = qa; q < qb; ++q) {
            const uint32_t *qc = qcodes + (uint64_t)q * a.cg * RW;
            const uint64_t *qmk = qmasks + (uint64_t)q * a.L;
            int64_t S = 0;
            bool undecided = valid && (!a.tri || s > q), maybe = false;
#pragma unroll
            for (int u = 0; u < R; ++u) {
                if (!__any(undecided)) break;
                code_unit_steps<W, PACK, UNITW>((uint32_t)u, P[u], em[u], qc, qmk, pk, cd, kpmask, kp, policy, s_dmul,
                                                tab, S, undecided, maybe);
            }
            for (uint32_t u = R; u < cu; ++u) {
                if (!__any(undecided)) break;
                uint32_t Pu[PW], emu[W];
                const size_t r = u - R;
                if (u == staged) {           // wave-uniform: first query of the item to reach unit u
                    const uint4 *src =
                        reinterpret_cast<const uint4 *>(codes + (((uint64_t)u * ctiles + tile) * 64 + lane) * PW);
#pragma unroll
                    for (int j = 0; j < PV; ++j) {
                        const uint4 v = src[j];
                        s_pl[(r * PV + j) * 64 + lane] = v;
                        Pu[4 * j + 0] = v.x;
                        Pu[4 * j + 1] = v.y;
                        Pu[4 * j + 2] = v.z;
                        Pu[4 * j + 3] = v.w;
                    }
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        uint32_t e = Pu[w];
#pragma unroll
                        for (int p = 1; p < (int)kCodeBits; ++p) e &= Pu[p * W + w];
                        emu[w] = e;
                        s_em[(r * W + w) * 64 + lane] = e;
                    }
                    ++staged;
                } else {
#pragma unroll
                    for (int j = 0; j < PV; ++j) {
                        const uint4 v = s_pl[(r * PV + j) * 64 + lane];
                        Pu[4 * j + 0] = v.x;
                        Pu[4 * j + 1] = v.y;
                        Pu[4 * j + 2] = v.z;
                        Pu[4 * j + 3] = v.w;
                    }
#pragma unroll
                    for (int w = 0; w < W; ++w) emu[w] = s_em[(r * W + w) * 64 + lane];
                }
                code_unit_steps<W, PACK, UNITW>(u, Pu, emu, qc, qmk, pk, cd, kpmask, kp, policy, s_dmul, tab, S,
                                                undecided, maybe);
            }
            const bool survive = maybe || undecided;
            sb.push(__ballot(survive), q, (uint32_t)s, surv, a.surv_cap, counters + 0, lane);
        }
    }
    sb.flush(surv, a.surv_cap, counters + 0, lane);
}

// The self-join's (tile group, query chunk) items that hold a set id above the
// chunk's first query row: the tile groups of chunk c start at first(c), and
// the items are numbered chunk by chunk, so that consecutive wavefronts take
// consecutive items of the upper triangle (wavefronts past the item count exit
// at once) instead of half of them landing on items below the diagonal.
struct TriItems {
    uint64_t ngroups, span;         // tile groups, sets per tile group
    uint32_t q_lo, qpw, nchunks;
    __device__ __forceinline__ uint64_t first(uint32_t c) const {
        const uint64_t qa = q_lo + (uint64_t)c * qpw;
        return min(ngroups, (qa + 1) / span);
    }
    __device__ __forceinline__ uint64_t total() const {
        uint64_t t = 0;
        for (uint32_t c = 0; c < nchunks; ++c) t += ngroups - first(c);
        return t;
    }
};

// First-group code pass (depth 1, JOINT or LITERAL), TPW tiles of 64 indexed
// sets per wavefront: each query's record (read with scalar loads, one query
// ahead) is compared with TPW tiles, so the scalar work of a query is shared
// by 64 TPW sets.  A pair is kept when more of the query's non-empty bins
// have equal codes than the query's keep threshold (the record's; the same
// test as a count of differing bins below ScanTab::dthr0), counted as the
// popcount of a chain of agreeing-bin masks that starts from the query's
// non-empty mask.  With P1 > 0 the first P1 planes are compared first, for all
// TPW tiles: bins that differ there differ in the full code too, so when no
// lane's largest partial count over the tiles exceeds the threshold the query
// is done with these tiles (the usual case for pairs far from the threshold),
// and otherwise the remaining planes continue each tile's chain and the pairs
// are tested one by one (lanes past the last set or, in the self-join, below
// the diagonal only cost a second phase that keeps none of them).  TRI: the self-join's upper-triangle filter.  Lane sets are
// combined as 64-bit wave masks (one ballot per tile and test).
template <int W, int TPW, int P1, bool TRI>
__global__ __launch_bounds__(kThreads) void scan_codes_fast_kernel(const uint32_t *__restrict__ codes,
                                                                  const uint32_t *__restrict__ qcodes,
                                                                  Survivor *__restrict__ surv,
                                                                  unsigned long long *__restrict__ counters,
                                                                  const uint64_t *__restrict__ desc,
                                                                  const CoarseArgs a) {
    constexpr int PW = (int)kCodeBits * W, RW = PW + 4, RS = PW + 8;   // words read per record, record stride
    __shared__ Survivor s_surv[kWaves][kSurvBatch];
    const uint32_t lane = threadIdx.x & 63;
    SurvBatch<kSurvBatch> sb{s_surv[wave_id_in_block()], 0};
    const uint64_t n_sets = desc ? desc[1] : a.n_sets;
    const uint32_t q_lo = desc ? 0u : a.q0, q_hi = desc ? (uint32_t)desc[0] : a.q1;
    const uint32_t qpw = chunk_queries(a, desc, q_hi - q_lo);
    const uint64_t ntiles = (n_sets + 63) / 64;
    const uint64_t ngroups = (ntiles + TPW - 1) / TPW;
    const uint32_t nchunks = (q_hi - q_lo + qpw - 1) / qpw;
    const TriItems tri{ngroups, (uint64_t)TPW * 64, q_lo, qpw, nchunks};
    const uint64_t n_items = TRI ? tri.total() : ngroups * nchunks;
    const uint64_t wstride = (uint64_t)gridDim.x * kWaves;
    const uint64_t ctiles = a.capacity / 64;
    const uint64_t rstride = (uint64_t)a.cg * RS;
    uint32_t tri_c = 0;                  // self-join: chunk of the cursor, and its first item
    uint64_t tri_base = 0;
    for (uint64_t item = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); item < n_items; item += wstride) {
        uint64_t tg;
        uint32_t chunk;
        if constexpr (TRI) {
            // items come in increasing order, so the cursor only moves forward
            while (item >= tri_base + (ngroups - tri.first(tri_c))) {
                tri_base += ngroups - tri.first(tri_c);
                ++tri_c;
            }
            chunk = tri_c;
            tg = tri.first(tri_c) + (item - tri_base);
        } else {
            tg = item % ngroups;
            chunk = (uint32_t)(item / ngroups);
        }
        const uint32_t qa = q_lo + chunk * qpw;
        const uint32_t qb = min(q_hi, qa + qpw);
        uint32_t P[TPW][PW];
        uint64_t vmask[TPW];                 // lanes holding an indexed set, per tile
        uint32_t sid[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const uint64_t tile = tg * TPW + t;
            const uint64_t s = tile * 64 + lane;
            vmask[t] = __builtin_amdgcn_ballot_w64(s < n_sets);
            sid[t] = (uint32_t)s;
            if (tile < ntiles) {             // wave-uniform; tiles below ntiles exist (ntiles <= ctiles)
                const uint4 *src = reinterpret_cast<const uint4 *>(codes + (tile * 64 + lane) * PW);
#pragma unroll
                for (int j = 0; j < PW / 4; ++j) {
                    const uint4 v = src[j];
                    P[t][4 * j + 0] = v.x;
                    P[t][4 * j + 1] = v.y;
                    P[t][4 * j + 2] = v.z;
                    P[t][4 * j + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int j = 0; j < PW; ++j) P[t][j] = 0;
            }
        }
        (void)ctiles;
        uint32_t ra[RW], rb[RW];
#pragma unroll
        for (int j = 0; j < RW; ++j) ra[j] = qcodes[qa * rstride + j];
// one query against the TPW tiles, with the survivor append per tile (written
// out twice below, on the kernel's own restrict pointers, so that the record
// loads stay scalar)
#define HOPH_CODE_QUERY_T(r, qq)                                                                   \
        {                                                                                          \
            uint32_t aa[TPW][W];                                                                   \
            bool open = true;                                                                      \
            if constexpr (P1 > 0) {                                                                \
                int32_t best = 0;                                                                  \
                _Pragma("unroll") for (int t = 0; t < TPW; ++t) {                                  \
                    uint32_t ag = 0;                                                               \
                    _Pragma("unroll") for (int w = 0; w < W; ++w) {                                \
                        aa[t][w] = code_agree_part<W, 0, P1>(0u, r[PW + w], P[t], r, w);           \
                        ag += __popc(aa[t][w]);                                                    \
                    }                                                                              \
                    best = max(best, (int32_t)ag);                                                 \
                }                                                                                  \
                open = __builtin_amdgcn_ballot_w64(best > (int32_t)r[PW + 2]) != 0;                \
            }                                                                                      \
            if (open) {                                                                            \
                uint64_t lanes[TPW];                                                               \
                _Pragma("unroll") for (int t = 0; t < TPW; ++t)                                    \
                    lanes[t] = TRI ? vmask[t] & __builtin_amdgcn_ballot_w64(sid[t] > (qq)) : vmask[t]; \
                _Pragma("unroll") for (int t = 0; t < TPW; ++t) {                                  \
                    uint32_t ag = 0;                                                               \
                    _Pragma("unroll") for (int w = 0; w < W; ++w) {                                \
                        const uint32_t x = P1 > 0                                                  \
                            ? code_agree_part<W, P1, (int)kCodeBits>(aa[t][w], 0u, P[t], r, w)     \
                            : code_agree_part<W, 0, (int)kCodeBits>(0u, r[PW + w], P[t], r, w);    \
                        ag += __popc(x);                                                           \
                    }                                                                              \
                    const uint64_t bal =                                                           \
                        __builtin_amdgcn_ballot_w64((int32_t)ag > (int32_t)r[PW + 2]) & lanes[t];   \
                    sb.push(bal, (qq), sid[t], surv, a.surv_cap, counters + 0, lane);              \
                }                                                                                  \
            }                                                                                      \
        }
        for (uint32_t q = qa; q < qb; q += 2) {
#pragma unroll
            for (int j = 0; j < RW; ++j) rb[j] = qcodes[(q + 1) * rstride + j];
            HOPH_CODE_QUERY_T(ra, q)
            if (q + 1 >= qb) break;
#pragma unroll
            for (int j = 0; j < RW; ++j) ra[j] = qcodes[(q + 2) * rstride + j];
            HOPH_CODE_QUERY_T(rb, q + 1)
        }
#undef HOPH_CODE_QUERY_T
    }
    sb.flush(surv, a.surv_cap, counters + 0, lane);
}

// The first-group pass with only the first P1 planes of its tiles in VGPRs
// (one plane word; TRI: the self-join's filter), so that TPW tiles share each query's
// scalar work: phase 1 as in scan_codes_fast_kernel (the largest partial
// agreeing count over the tiles, one test per query); when some lane is kept
// the tiles that hold one are worked out from the registers, and each of them
// reads its 8 planes again (from L2 or HBM) and tests its pairs on the full
// codes.  A lane that phase 1 does not keep has too few agreeing bins on the
// full codes too, so testing every lane of such a tile gives the same pairs.
template <int TPW, int P1, bool TRI>
__global__ __launch_bounds__(kThreads) void scan_codes_fast1_kernel(const uint32_t *__restrict__ codes,
                                                                   const uint32_t *__restrict__ qcodes,
                                                                   Survivor *__restrict__ surv,
                                                                   unsigned long long *__restrict__ counters,
                                                                   const uint64_t *__restrict__ desc,
                                                                   const CoarseArgs a) {
    constexpr int PW = (int)kCodeBits, RW = PW + 4, RS = PW + 8;   // words read per record, record stride
    static_assert(P1 >= 2 && P1 <= 6, "phase-1 planes");
    __shared__ Survivor s_surv[kWaves][kSurvBatch];
    const uint32_t lane = threadIdx.x & 63;
    SurvBatch<kSurvBatch> sb{s_surv[wave_id_in_block()], 0};
    const uint64_t n_sets = desc ? desc[1] : a.n_sets;
    const uint32_t q_lo = desc ? 0u : a.q0, q_hi = desc ? (uint32_t)desc[0] : a.q1;
    const uint32_t qpw = chunk_queries(a, desc, q_hi - q_lo);
    const uint64_t ntiles = (n_sets + 63) / 64;
    const uint64_t ngroups = (ntiles + TPW - 1) / TPW;
    const uint32_t nchunks = (q_hi - q_lo + qpw - 1) / qpw;
    const TriItems tri{ngroups, (uint64_t)TPW * 64, q_lo, qpw, nchunks};
    const uint64_t n_items = TRI ? tri.total() : ngroups * nchunks;
    const uint64_t wstride = (uint64_t)gridDim.x * kWaves;
    const uint64_t rstride = (uint64_t)a.cg * RS;
    uint32_t tri_c = 0;                  // self-join: chunk of the cursor, and its first item
    uint64_t tri_base = 0;
    for (uint64_t item = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); item < n_items; item += wstride) {
        uint64_t tg;
        uint32_t chunk;
        if constexpr (TRI) {
            while (item >= tri_base + (ngroups - tri.first(tri_c))) {
                tri_base += ngroups - tri.first(tri_c);
                ++tri_c;
            }
            chunk = tri_c;
            tg = tri.first(tri_c) + (item - tri_base);
        } else {
            tg = item % ngroups;
            chunk = (uint32_t)(item / ngroups);
        }
        const uint32_t qa = q_lo + chunk * qpw;
        const uint32_t qb = min(q_hi, qa + qpw);
        uint32_t P[TPW][P1];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const uint64_t tile = tg * TPW + t;
            if (tile < ntiles) {             // wave-uniform; tiles below ntiles exist (ntiles <= ctiles)
                const uint4 *src = reinterpret_cast<const uint4 *>(codes + (tile * 64 + lane) * PW);
                const uint4 v0 = src[0];
                uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, 0u, 0u, 0u, 0u};
                if constexpr (P1 > 4) {
                    const uint4 v1 = src[1];
                    w[4] = v1.x;
                    w[5] = v1.y;
                }
#pragma unroll
                for (int j = 0; j < P1; ++j) P[t][j] = w[j];
            } else {
#pragma unroll
                for (int j = 0; j < P1; ++j) P[t][j] = 0;
            }
        }
        uint32_t ra[RW], rb[RW];
#pragma unroll
        for (int j = 0; j < RW; ++j) ra[j] = qcodes[qa * rstride + j];
// one query against the TPW tiles (written out twice below, on the kernel's
// own restrict pointers, so that the record loads stay scalar)
#define HOPH_CODE_QUERY_1(r, qq)                                                                   \
        {                                                                                          \
            int32_t best = 0;                                                                      \
            _Pragma("unroll") for (int t = 0; t < TPW; ++t) {                                      \
                const uint32_t x = code_agree_part<1, 0, P1>(0u, r[PW], P[t], r, 0);               \
                best = max(best, (int32_t)__popc(x));                                              \
            }                                                                                      \
            if (__builtin_amdgcn_ballot_w64(best > (int32_t)r[PW + 2])) {                          \
                uint32_t tiles_kept = 0;                                                           \
                _Pragma("unroll") for (int t = 0; t < TPW; ++t) {                                  \
                    const uint32_t x = code_agree_part<1, 0, P1>(0u, r[PW], P[t], r, 0);           \
                    const uint64_t sv = (tg * TPW + t) * 64 + lane;                                \
                    const bool in = sv < n_sets && (!TRI || sv > (qq));   /* pairs the pass may emit */ \
                    tiles_kept |= __builtin_amdgcn_ballot_w64(in && (int32_t)__popc(x) > (int32_t)r[PW + 2]) \
                                      ? (1u << t) : 0u;                                            \
                }                                                                                  \
                _Pragma("unroll 1") for (int t = 0; t < TPW; ++t) {                                \
                    if (!((tiles_kept >> t) & 1u)) continue;                                       \
                    const uint64_t tile = tg * TPW + t;                                            \
                    const uint64_t sv = tile * 64 + lane;                                          \
                    const uint4 *src = reinterpret_cast<const uint4 *>(codes + sv * PW);           \
                    const uint4 v0 = src[0], v1 = src[1];                                          \
                    const uint32_t Pf[PW] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};      \
                    const uint32_t x = code_agree_part<1, 0, (int)kCodeBits>(0u, r[PW], Pf, r, 0); \
                    const uint64_t bal = __builtin_amdgcn_ballot_w64((int32_t)__popc(x) > (int32_t)r[PW + 2]) & \
                                         __builtin_amdgcn_ballot_w64(sv < n_sets && (!TRI || sv > (qq))); \
                    sb.push(bal, (qq), (uint32_t)sv, surv, a.surv_cap, counters + 0, lane);        \
                }                                                                                  \
            }                                                                                      \
        }
        for (uint32_t q = qa; q < qb; q += 2) {
#pragma unroll
            for (int j = 0; j < RW; ++j) rb[j] = qcodes[(q + 1) * rstride + j];
            HOPH_CODE_QUERY_1(ra, q)
            if (q + 1 >= qb) break;
#pragma unroll
            for (int j = 0; j < RW; ++j) ra[j] = qcodes[(q + 2) * rstride + j];
            HOPH_CODE_QUERY_1(rb, q + 1)
        }
#undef HOPH_CODE_QUERY_1
    }
    sb.flush(surv, a.surv_cap, counters + 0, lane);
}

// Multi-group code pass with the linear bound of LinTab: D groups (one per
// code unit, k' <= 32 bins, one plane word), TPW tiles of 64 indexed sets per
// wavefront sharing each query's scalar work (its record: planes, non-empty
// mask and the words c, z', y' of every group), one set per lane.  The state
// of a pair after step s is st_s = sum_{g <= s} c_g dn_g, dn_g the
// query-non-empty bins of group g whose codes differ; st_s <= y_s keeps the
// pair ("maybe": an accept cutoff may be reached), else st_s >= z_s rejects
// it.  The kernel counts agreeing bins instead (ag_g = (k' - e_g) - dn_g, the
// popcount of an agreeing-bin chain started from the query's non-empty mask,
// see code_agree_part) and tests st'_s = sum_{g <= s} c_g ag_g against the
// record's z'_s and y'_s: st' <= z' rejects (z' < 0: never), st' >= y' keeps
// (y' = INT32_MAX: never), the same tests as on st.
// Phase 1 (P1 > 0) compares the first P1 planes of groups 0..R, R the first
// step with a reject cutoff: a bin that differs there differs in the full
// code, so the partial state never exceeds the full one (the partial agreeing
// counts never fall below the full ones).  A lane whose partial
// state is rejected at step R and kept at no step up to R is rejected by the
// full test too (the steps before R cannot reject), so when no lane of the
// wavefront is kept the query is done with these tiles.  Phase 2 continues the
// plane chains and takes the steps in order; pairs still undecided after D
// groups are kept.  Kept pairs go on to the fine pass from the first group.
template <int D, int TPW, int P1>
__global__ __launch_bounds__(kThreads) void scan_codes_lin_kernel(const uint32_t *__restrict__ codes,
                                                                 const uint32_t *__restrict__ qcodes,
                                                                 Survivor *__restrict__ surv,
                                                                 unsigned long long *__restrict__ counters,
                                                                 const uint64_t *__restrict__ desc,
                                                                 const CoarseArgs a, const uint32_t R) {
    constexpr int PW = (int)kCodeBits, RS = PW + 8;       // planes per unit, record stride
    __shared__ Survivor s_surv[kWaves][kSurvBatch];
    const uint32_t lane = threadIdx.x & 63;
    SurvBatch<kSurvBatch> sb{s_surv[wave_id_in_block()], 0};
    const uint64_t n_sets = desc ? desc[1] : a.n_sets;
    const uint32_t q_lo = desc ? 0u : a.q0, q_hi = desc ? (uint32_t)desc[0] : a.q1;
    const uint32_t qpw = chunk_queries(a, desc, q_hi - q_lo);
    const uint64_t ntiles = (n_sets + 63) / 64;
    const uint64_t ngroups = (ntiles + TPW - 1) / TPW;
    const uint32_t nchunks = (q_hi - q_lo + qpw - 1) / qpw;
    const uint64_t n_items = ngroups * nchunks;
    const uint64_t wstride = (uint64_t)gridDim.x * kWaves;
    const uint64_t ctiles = a.capacity / 64;
    const uint64_t rstride = (uint64_t)a.cg * RS;
    for (uint64_t item = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); item < n_items; item += wstride) {
        const uint64_t tg = item % ngroups;
        const uint32_t chunk = (uint32_t)(item / ngroups);
        const uint32_t qa = q_lo + chunk * qpw;
        const uint32_t qb = min(q_hi, qa + qpw);
        uint32_t P[TPW][D][PW];
        uint64_t vmask[TPW];
        uint32_t sid[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const uint64_t tile = tg * TPW + t;
            const uint64_t s = tile * 64 + lane;
            vmask[t] = __builtin_amdgcn_ballot_w64(s < n_sets);
            sid[t] = (uint32_t)s;
            if (tile < ntiles) {             // wave-uniform; tiles below ntiles exist (ntiles <= ctiles)
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    const uint4 *src = reinterpret_cast<const uint4 *>(codes + (((uint64_t)u * ctiles + tile) * 64 + lane) * PW);
#pragma unroll
                    for (int j = 0; j < PW / 4; ++j) {
                        const uint4 v = src[j];
                        P[t][u][4 * j + 0] = v.x;
                        P[t][u][4 * j + 1] = v.y;
                        P[t][u][4 * j + 2] = v.z;
                        P[t][u][4 * j + 3] = v.w;
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < D; ++u)
#pragma unroll
                    for (int j = 0; j < PW; ++j) P[t][u][j] = 0;
            }
        }
        for (uint32_t q = qa; q < qb; ++q) {
            const uint32_t *rec = qcodes + (uint64_t)q * rstride;
            uint32_t nq[D], c[D];
            int32_t z[D], y[D];
#pragma unroll
            for (int g = 0; g < D; ++g) {
                nq[g] = rec[g * RS + PW];
                c[g] = rec[g * RS + PW + 4];
                z[g] = (int32_t)rec[g * RS + PW + 5];
                y[g] = (int32_t)rec[g * RS + PW + 6];
            }
            const int32_t zR = (int32_t)rec[R * RS + PW + 5];   // the reject cutoff of step R
            uint32_t aa[TPW][D];
            bool open = true;
            if constexpr (P1 > 0) {
                uint64_t keep = 0;
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    uint32_t st = 0;
                    bool mb = false;
#pragma unroll
                    for (int g = 0; g < D; ++g) {
                        if ((uint32_t)g <= R) {
                            aa[t][g] = code_agree_part<1, 0, P1>(0u, nq[g], P[t][g], rec + g * RS, 0);
                            st = __umul24(c[g], (uint32_t)__popc(aa[t][g])) + st;
                            mb = mb || (int32_t)st >= y[g];
                        }
                    }
                    keep |= __builtin_amdgcn_ballot_w64(mb || (int32_t)st > zR) & vmask[t];
                }
                open = keep != 0;
            }
            if (open) {
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    uint32_t st = 0;
                    bool und = true, mb = false;
#pragma unroll
                    for (int g = 0; g < D; ++g) {
                        if ((uint32_t)g > R && !__any(und)) break;
                        const uint32_t x =
                            (P1 > 0 && (uint32_t)g <= R)
                                ? code_agree_part<1, P1, (int)kCodeBits>(aa[t][g], 0u, P[t][g], rec + g * RS, 0)
                                : code_agree_part<1, 0, (int)kCodeBits>(0u, nq[g], P[t][g], rec + g * RS, 0);
                        st = __umul24(c[g], (uint32_t)__popc(x)) + st;
                        if (und) {
                            if ((int32_t)st >= y[g]) {
                                mb = true;
                                und = false;
                            } else if ((int32_t)st <= z[g]) {
                                und = false;
                            }
                        }
                    }
                    const uint64_t bal = __builtin_amdgcn_ballot_w64(mb || und) & vmask[t];
                    sb.push(bal, q, sid[t], surv, a.surv_cap, counters + 0, lane);
                }
            }
        }
    }
    sb.flush(surv, a.surv_cap, counters + 0, lane);
}

// The linear-bound pass when a first phase of P1 planes decides the
// background pairs (see scan_codes_lin_kernel): only the first P1 planes of
// groups 0..G1-1 (G1 = R + 1) stay in VGPRs, so TPW tiles of 64 sets share each
// query's scalar work; a tile with a lane that phase 1 keeps reads its full
// planes of all D groups again (from L2 or HBM) and takes the steps in order.
// A lane that phase 1 does not keep is rejected by the full test (see
// scan_codes_lin_kernel), so running the full test on every lane of such a tile
// gives the same pairs.
template <int G1, int D, int TPW, int P1>
__global__ __launch_bounds__(kThreads) void scan_codes_lin1_kernel(const uint32_t *__restrict__ codes,
                                                                  const uint32_t *__restrict__ qcodes,
                                                                  Survivor *__restrict__ surv,
                                                                  unsigned long long *__restrict__ counters,
                                                                  const uint64_t *__restrict__ desc,
                                                                  const CoarseArgs a) {
    constexpr int PW = (int)kCodeBits, RS = PW + 8, R = G1 - 1;
    static_assert(P1 >= 1 && P1 <= 4 && G1 >= 1 && G1 <= D, "phase-1 shape");
    __shared__ Survivor s_surv[kWaves][kSurvBatch];
    const uint32_t lane = threadIdx.x & 63;
    SurvBatch<kSurvBatch> sb{s_surv[wave_id_in_block()], 0};
    const uint64_t n_sets = desc ? desc[1] : a.n_sets;
    const uint32_t q_lo = desc ? 0u : a.q0, q_hi = desc ? (uint32_t)desc[0] : a.q1;
    const uint32_t qpw = chunk_queries(a, desc, q_hi - q_lo);
    const uint64_t ntiles = (n_sets + 63) / 64;
    const uint64_t ngroups = (ntiles + TPW - 1) / TPW;
    const uint32_t nchunks = (q_hi - q_lo + qpw - 1) / qpw;
    const uint64_t n_items = ngroups * nchunks;
    const uint64_t wstride = (uint64_t)gridDim.x * kWaves;
    const uint64_t ctiles = a.capacity / 64;
    const uint64_t rstride = (uint64_t)a.cg * RS;
    for (uint64_t item = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); item < n_items; item += wstride) {
        const uint64_t tg = item % ngroups;
        const uint32_t chunk = (uint32_t)(item / ngroups);
        const uint32_t qa = q_lo + chunk * qpw;
        const uint32_t qb = min(q_hi, qa + qpw);
        uint32_t P[TPW][G1][P1];
        uint64_t vmask[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const uint64_t tile = tg * TPW + t;
            vmask[t] = __builtin_amdgcn_ballot_w64(tile * 64 + lane < n_sets);
            if (tile < ntiles) {             // wave-uniform; tiles below ntiles exist (ntiles <= ctiles)
#pragma unroll
                for (int u = 0; u < G1; ++u) {
                    const uint4 v =
                        *reinterpret_cast<const uint4 *>(codes + (((uint64_t)u * ctiles + tile) * 64 + lane) * PW);
                    const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int j = 0; j < P1; ++j) P[t][u][j] = w4[j];
                }
            } else {
#pragma unroll
                for (int u = 0; u < G1; ++u)
#pragma unroll
                    for (int j = 0; j < P1; ++j) P[t][u][j] = 0;
            }
        }
        for (uint32_t q = qa; q < qb; ++q) {
            const uint32_t *rec = qcodes + (uint64_t)q * rstride;
            uint32_t nq[G1], c[G1];
            int32_t y[G1];
#pragma unroll
            for (int g = 0; g < G1; ++g) {
                nq[g] = rec[g * RS + PW];
                c[g] = rec[g * RS + PW + 4];
                y[g] = (int32_t)rec[g * RS + PW + 6];
            }
            // keep at step R when st' > zk: above the reject cutoff, or at or above
            // the maybe cutoff (y'_R - 1 < z'_R only when rounding meets them)
            const int32_t zR = (int32_t)rec[R * RS + PW + 5];
            const int32_t zk = y[R] - 1 < zR ? y[R] - 1 : zR;
            // phase 1: the largest partial state of each step over the tiles (the
            // keep tests are thresholds on them), then one test per query
            int32_t top[G1];
#pragma unroll
            for (int g = 0; g < G1; ++g) top[g] = 0;
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                uint32_t st = 0;
#pragma unroll
                for (int g = 0; g < G1; ++g) {
                    const uint32_t x = code_agree_part<1, 0, P1>(0u, nq[g], P[t][g], rec + g * RS, 0);
                    st = __umul24(c[g], (uint32_t)__popc(x)) + st;
                    top[g] = max(top[g], (int32_t)st);
                }
            }
            bool any = top[R] > zk;
#pragma unroll
            for (int g = 0; g < R; ++g) any = any || top[g] >= y[g];
            if (!__builtin_amdgcn_ballot_w64(any)) continue;
            // some lane is kept (rare): which tiles
            uint32_t tiles_kept = 0;         // bit t: a lane of tile t is kept
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                uint32_t st = 0;
                bool mb = false;
#pragma unroll
                for (int g = 0; g < G1; ++g) {
                    const uint32_t x = code_agree_part<1, 0, P1>(0u, nq[g], P[t][g], rec + g * RS, 0);
                    st = __umul24(c[g], (uint32_t)__popc(x)) + st;
                    if (g < R) mb = mb || (int32_t)st >= y[g];
                }
                tiles_kept |= (__builtin_amdgcn_ballot_w64(mb || (int32_t)st > zk) & vmask[t]) ? (1u << t) : 0u;
            }
            if (tiles_kept == 0) continue;
            // phase 2 (rare): full planes of every group, steps in order
            uint32_t nqf[D], cf[D];
            int32_t zf[D], yf[D];
#pragma unroll
            for (int g = 0; g < D; ++g) {
                nqf[g] = rec[g * RS + PW];
                cf[g] = rec[g * RS + PW + 4];
                zf[g] = (int32_t)rec[g * RS + PW + 5];
                yf[g] = (int32_t)rec[g * RS + PW + 6];
            }
            // one tile at a time (not unrolled: the full planes of one tile are live at once)
#pragma unroll 1
            for (int t = 0; t < TPW; ++t) {
                if (!((tiles_kept >> t) & 1u)) continue;
                const uint64_t tile = tg * TPW + t;
                const uint64_t vm = __builtin_amdgcn_ballot_w64(tile * 64 + lane < n_sets);
                uint32_t st = 0;
                bool und = true, mb = false;
#pragma unroll
                for (int g = 0; g < D; ++g) {
                    if (g > R && !__any(und)) break;
                    const uint4 *src =
                        reinterpret_cast<const uint4 *>(codes + (((uint64_t)g * ctiles + tile) * 64 + lane) * PW);
                    const uint4 v0 = src[0], v1 = src[1];
                    const uint32_t Pf[PW] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
                    const uint32_t x = code_agree_part<1, 0, (int)kCodeBits>(0u, nqf[g], Pf, rec + g * RS, 0);
                    st = __umul24(cf[g], (uint32_t)__popc(x)) + st;
                    if (und) {
                        if ((int32_t)st >= yf[g]) {
                            mb = true;
                            und = false;
                        } else if ((int32_t)st <= zf[g]) {
                            und = false;
                        }
                    }
                }
                const uint64_t bal = __builtin_amdgcn_ballot_w64(mb || und) & vm;
                sb.push(bal, q, (uint32_t)(tile * 64 + lane), surv, a.surv_cap, counters + 0, lane);
            }
        }
    }
    sb.flush(surv, a.surv_cap, counters + 0, lane);
}

template <int KPAD, int G, bool EXACT>
__global__ __launch_bounds__(kThreads) void scan_coarse_kernel(const uint32_t *__restrict__ slab,
                                                              const uint32_t *__restrict__ qsigs,
                                                              const uint64_t *__restrict__ qmasks,
                                                              Survivor *__restrict__ surv,
                                                              uint64_t *__restrict__ keys,
                                                              unsigned long long *__restrict__ counters,
                                                              const uint64_t *__restrict__ desc,
                                                              const CoarseArgs a, const ScanTab tab) {
    __shared__ int64_t s_dmul[HOPH_MAX_KGROUP + 1];
    __shared__ int32_t s_macc[HOPH_MAX_KGROUP + 1], s_mrej[HOPH_MAX_KGROUP + 1];
    for (uint32_t i = threadIdx.x; i <= tab.kp; i += kThreads) {
        s_dmul[i] = tab.dmul[i];
        s_macc[i] = tab.macc0[i];
        s_mrej[i] = tab.mrej0[i];
    }
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63;
    const uint64_t n_sets = desc ? desc[1] : a.n_sets;
    const uint32_t q_lo = desc ? 0u : a.q0, q_hi = desc ? (uint32_t)desc[0] : a.q1;
    const uint32_t qpw = chunk_queries(a, desc, q_hi - q_lo);
    const uint64_t ntiles = (n_sets + 63) / 64;
    const uint32_t nchunks = (q_hi - q_lo + qpw - 1) / qpw;
    const uint64_t n_items = ntiles * nchunks;
    const uint64_t wstride = (uint64_t)gridDim.x * kWaves;
    const uint32_t kp = EXACT ? KPAD : a.kp;
    const uint64_t kpmask = kp >= 64 ? ~0ull : ((1ull << kp) - 1ull);
    const bool vec = (a.k & 3u) == 0;
    const uint32_t policy = a.policy;
    for (uint64_t item = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); item < n_items; item += wstride) {
    const uint64_t tile = item % ntiles;
    const uint32_t chunk = (uint32_t)(item / ntiles);
    // self-join: skip (before any load) a tile with no set id above the chunk's first query row
    if (a.tri && tile * 64 + 63 <= (uint64_t)q_lo + (uint64_t)chunk * qpw) continue;
    const uint64_t s = tile * 64 + lane;
    const bool valid = s < n_sets;

    uint32_t w[G][KPAD];
    uint64_t emask[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // this lane's set row (rows up to the capacity exist, so rows past the
        // last set are read and then ignored)
        load_group_row<KPAD, EXACT>(slab + s * a.k + (uint64_t)g * kp, kp, vec, w[g]);
        uint64_t em = 0;
#pragma unroll
        for (int i = 0; i < KPAD; ++i) em |= (uint64_t)(w[g][i] == HOPH_EMPTY) << i;
        emask[g] = em & kpmask;
    }

    const uint32_t qa = q_lo + chunk * qpw;
    const uint32_t qb = min(q_hi, qa + qpw);
    for (uint32_t q = qa; q < qb; ++q) {
        const uint32_t *qw = qsigs + (uint64_t)q * a.k;
        const uint64_t *qmk = qmasks + (uint64_t)q * a.L;
        int64_t S = 0;
        bool undecided = valid && (!a.tri || s > q), accept = false;
        if constexpr (G == 1) {
            uint32_t eq = 0;
            const uint64_t qm = qmk[0];
#pragma unroll
            for (int i = 0; i < KPAD; ++i) {
                if (EXACT || i < (int)kp) eq += (w[0][i] == qw[i]) ? 1u : 0u;
            }
            uint32_t ej = 0, e = 0;
            if (qm != 0) ej = __popcll(emask[0] & qm);
            if (policy == HOPH_EMPTY_JOINT) e = ej;
            else if (policy == HOPH_EMPTY_EITHER) e = __popcll(emask[0] | qm);
            const uint32_t m = eq - ej;
            bool acc, rej;
            if (e < kp) {
                acc = (int32_t)m >= s_macc[e];
                rej = (int32_t)m <= s_mrej[e];
            } else {
                const int64_t S0 = tab.W[0] * (ej == kp ? tab.lambda : 0);
                acc = S0 >= tab.acc[0];
                rej = S0 <= tab.rej[0];
            }
            const bool pair_ok = valid && (!a.tri || s > q);
            accept = pair_ok && acc;
            undecided = pair_ok && !acc && !rej;
            if (__any(undecided)) {
                // the state after the first group, for the pairs that continue
                const int64_t rho = policy == HOPH_EMPTY_LITERAL ? (int64_t)m
                                    : (e < kp ? (int64_t)m * s_dmul[e] : (ej == kp ? tab.lambda : 0));
                S = tab.W[0] * rho;
            }
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (!__any(undecided)) break;
                const uint32_t *qg = qw + g * kp;
                uint32_t eq = 0;
                const uint64_t qm = qmk[g];
#pragma unroll
                for (int i = 0; i < KPAD; ++i) {
                    if (EXACT || i < (int)kp) eq += (w[g][i] == qg[i]) ? 1u : 0u;
                }
                const uint32_t ej = qm ? (uint32_t)__popcll(emask[g] & qm) : 0u;
                const uint32_t ee = __popcll(emask[g] | qm);
                S += tab.W[g] * group_rho(eq, ej, ee, kp, policy, s_dmul, tab.lambda);
                if (undecided) {
                    if (S >= tab.acc[g]) {
                        accept = true;
                        undecided = false;
                    } else if (S <= tab.rej[g]) {
                        undecided = false;
                    }
                }
            }
        }
        if (__any(accept)) {
            const uint64_t slot = wave_append(accept, counters + 1, lane);
            if (accept && slot < a.keys_cap) keys[slot] = ((uint64_t)q << 32) | s;
        }
        if (__any(undecided)) {
            const uint64_t slot = wave_append(undecided, counters + 0, lane);
            if (undecided && slot < a.surv_cap) surv[slot] = Survivor{q, (uint32_t)s, S};
        }
    }
    }
}

// Per-survivor pass (Alg. 1 / Alg. 2 from the group the coarse pass stopped
// at): one wavefront per surviving pair, P = 64 / k' groups side by side across
// the lanes of one load and R loads in flight, the exact weighted state
// updated group by group until an accept or reject cutoff (or the last group).
// Accepted keys wait in the wavefront's LDS buffer and are written in batches:
// a slot reservation per pair on the one accepted-pairs counter would queue
// every wavefront at that counter.
__global__ __launch_bounds__(kThreads) void scan_fine_kernel(const uint32_t *__restrict__ slab,
                                                            const uint32_t *__restrict__ qsigs,
                                                            const Survivor *__restrict__ surv,
                                                            uint64_t *__restrict__ keys,
                                                            unsigned long long *__restrict__ counters,
                                                            const CoarseArgs a, const ScanTab tab) {
    __shared__ int64_t s_dmul[HOPH_MAX_KGROUP + 1];
    __shared__ uint64_t s_keys[kWaves][64];      // accepted keys of each wavefront, not yet written
    __shared__ uint32_t s_nk[kWaves];
    __shared__ unsigned long long s_base;
    for (uint32_t i = threadIdx.x; i <= tab.kp; i += kThreads) s_dmul[i] = tab.dmul[i];
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wib = wave_id_in_block();
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    const uint64_t n = min((uint64_t)counters[0], a.surv_cap);
    const uint32_t kp = a.kp;
    uint32_t nk = 0;                              // keys in s_keys[wib] (wave-uniform)
    // P groups side by side across the lanes of one load (lane = c k' + bin),
    // R loads per step: P R groups are read at once (independent loads in
    // flight), then decided in order; reads past the deciding group are discarded
    const uint32_t P = 64u / kp, R = kp > 32 ? (uint32_t)kFineAhead : 2u, span = P * R;
    const uint32_t lc = lane / kp, lb = lane - lc * kp;
    const bool in = lc < P;
    const uint64_t kpmask = kp >= 64 ? ~0ull : ((1ull << kp) - 1ull);
    for (uint64_t idx = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); idx < n; idx += nw) {
        const Survivor sv = surv[idx];
        int64_t S = sv.S;
        bool accept = false;
        const uint64_t s = sv.s;
        const uint32_t *qw = qsigs + (uint64_t)sv.q * a.k + lb;
        const uint32_t *sb = slab + s * a.k + lb;
        bool done = false;
        for (uint32_t g0 = a.depth; g0 < a.L && !done; g0 += span) {
            uint32_t sw[kFineAhead], qv[kFineAhead];
#pragma unroll
            for (int r = 0; r < kFineAhead; ++r) {
                const uint32_t g = g0 + (uint32_t)r * P + lc;
                sw[r] = qv[r] = 0;
                if ((uint32_t)r < R && in && g < a.L) {
                    sw[r] = sb[g * kp];
                    qv[r] = qw[g * kp];
                }
            }
#pragma unroll
            for (int r = 0; r < kFineAhead; ++r) {
                if ((uint32_t)r >= R || done) break;
                const uint32_t gr = g0 + (uint32_t)r * P;
                if (gr >= a.L) break;
                const bool live = in && gr + lc < a.L;
                const uint64_t eqb = __ballot(live && sw[r] == qv[r]);
                const uint64_t qe = __ballot(live && qv[r] == HOPH_EMPTY);
                const uint64_t se = __ballot(live && sw[r] == HOPH_EMPTY);
                for (uint32_t c = 0; c < P; ++c) {
                    const uint32_t g = gr + c;
                    if (g >= a.L) break;
                    const uint32_t sh = c * kp;
                    const uint64_t qec = (qe >> sh) & kpmask, sec = (se >> sh) & kpmask;
                    const uint32_t ej = __popcll(qec & sec), ee = __popcll(qec | sec);
                    const uint32_t eq = __popcll((eqb >> sh) & kpmask);
                    S += tab.W[g] * group_rho(eq, ej, ee, kp, a.policy, s_dmul, tab.lambda);
                    if (S >= tab.acc[g]) { accept = true; done = true; break; }
                    if (S <= tab.rej[g]) { done = true; break; }
                }
            }
        }
        if (accept) {                             // wave-uniform
            if (nk == 64) {                       // a full buffer: one reservation for 64 keys
                wave_lds_fence();
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(counters + 1, 64ull);
                base = __shfl(base, 0);
                if (base + lane < a.keys_cap) keys[base + lane] = s_keys[wib][lane];
                wave_lds_fence();
                nk = 0;
            }
            if (lane == 0) s_keys[wib][nk] = ((uint64_t)sv.q << 32) | s;
            ++nk;
        }
    }
    // the rest: one reservation per workgroup (a counter that every accepted
    // pair of the pass bumps by one serialises at its memory channel)
    wave_lds_fence();
    if (lane == 0) s_nk[wib] = nk;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long total = 0;
        for (uint32_t v = 0; v < kWaves; ++v) total += s_nk[v];
        s_base = total ? atomicAdd(counters + 1, total) : 0ull;
    }
    __syncthreads();
    unsigned long long off = s_base;
    for (uint32_t v = 0; v < wib; ++v) off += s_nk[v];
    for (uint32_t j = lane; j < nk; j += 64)
        if (off + j < a.keys_cap) keys[off + j] = s_keys[wib][j];
}

// Full-signature estimate of pairs (query row q, set id s), one wavefront per
// pair and one lane per bin: the exact weighted state over every group
// (Lemma 3 for HOPH, the mean of the group rates for GOPH, scaled by the
// tables' weight sum times lambda), the matched and empty counts over all k
// bins (Eq. 6), and the variance of Eq. 8 with the observed 1 / (k - N_eb) in
// place of its expectation and g = |D1 u D2| from `unions` (the large-g limit
// R (1 - R) / (k - N_eb) when it is null).
__global__ __launch_bounds__(kThreads) void pair_estimates_kernel(const uint32_t *__restrict__ slab, uint64_t n_sets,
                                                                 uint32_t k, uint32_t kp, uint32_t L,
                                                                 const uint32_t *__restrict__ qsigs, uint32_t n_q,
                                                                 const uint32_t *__restrict__ pairs, uint64_t n_pairs,
                                                                 uint32_t policy, const double *__restrict__ unions,
                                                                 int64_t *__restrict__ est, uint32_t *__restrict__ mb,
                                                                 uint32_t *__restrict__ eb, double *__restrict__ var,
                                                                 const ScanTab tab) {
    __shared__ int64_t s_dmul[HOPH_MAX_KGROUP + 1];
    for (uint32_t i = threadIdx.x; i <= tab.kp; i += kThreads) s_dmul[i] = tab.dmul[i];
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63;
    const bool in = lane < kp;
    const uint64_t nw = (uint64_t)gridDim.x * kWaves;
    for (uint64_t p = (uint64_t)blockIdx.x * kWaves + wave_id_in_block(); p < n_pairs; p += nw) {
        const uint64_t q = pairs[2 * p], s = pairs[2 * p + 1];
        if (q >= n_q || s >= n_sets) {
            if (lane == 0) {
                est[p] = -1;
                mb[p] = eb[p] = 0xFFFFFFFFu;
                var[p] = __builtin_nan("");
            }
            continue;
        }
        int64_t S = 0;
        uint32_t M = 0, EJ = 0, EE = 0;
        const uint32_t *sr = slab + s * k + lane, *qr = qsigs + q * k + lane;
        for (uint32_t g = 0; g < L; ++g) {
            uint32_t sw = 0, qv = 0;
            if (in) {
                sw = sr[g * kp];
                qv = qr[g * kp];
            }
            const uint64_t eqb = __ballot(in && sw == qv);
            const uint64_t qe = __ballot(in && qv == HOPH_EMPTY);
            const uint64_t se = __ballot(in && sw == HOPH_EMPTY);
            const uint32_t ej = __popcll(qe & se), ee = __popcll(qe | se), eq = __popcll(eqb);
            S += tab.W[g] * group_rho(eq, ej, ee, kp, policy, s_dmul, tab.lambda);
            M += eq - ej;
            EJ += ej;
            EE += ee;
        }
        if (lane == 0) {
            const uint32_t e = policy == HOPH_EMPTY_JOINT ? EJ : policy == HOPH_EMPTY_EITHER ? EE : 0u;
            double R, inv;
            if (policy == HOPH_EMPTY_LITERAL) {
                R = (double)M / k;
                inv = 1.0 / k;
            } else if (e < k) {
                R = (double)M / (k - e);
                inv = 1.0 / (k - e);
            } else {
                R = EJ == k ? 1.0 : 0.0;          // the 0/0 rule of the per-group rate
                inv = 0.0;
            }
            double v = R * (1.0 - R) * inv;       // g -> infinity
            if (unions) {
                const double gg = unions[p];
                v = gg > 1.0 ? R * (1.0 - R) * (inv * (1.0 + 1.0 / (gg - 1.0)) - 1.0 / (gg - 1.0)) : 0.0;
            }
            est[p] = S;
            mb[p] = M;
            eb[p] = e;
            var[p] = v;
        }
    }
}

// Plain OPH comparator (Eq. 6 over all k bins, no early stop).
template <int KPAD, bool EXACT>
__global__ __launch_bounds__(kThreads) void oph_full_kernel(const uint32_t *__restrict__ slab,
                                                           const uint32_t *__restrict__ qsigs,
                                                           uint64_t *__restrict__ keys,
                                                           unsigned long long *__restrict__ counters,
                                                           const CoarseArgs a, uint32_t tn, uint32_t td) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t)blockIdx.x * kWaves + wave_id_in_block();
    const uint64_t ntiles = (a.n_sets + 63) / 64;
    const uint32_t nq = a.q1 - a.q0;
    const uint32_t nchunks = (nq + a.q_per_wave - 1) / a.q_per_wave;
    if (wave >= ntiles * nchunks) return;
    const uint64_t tile = wave % ntiles;
    const uint32_t chunk = (uint32_t)(wave / ntiles);
    const uint64_t s = tile * 64 + lane;
    const bool valid = s < a.n_sets;
    const uint32_t kp = EXACT ? KPAD : a.kp, k = a.k;
    const bool vec = (k & 3u) == 0;
    const uint32_t qa = a.q0 + chunk * a.q_per_wave;
    const uint32_t qb = min(a.q1, qa + a.q_per_wave);
    for (uint32_t q = qa; q < qb; ++q) {
        const uint32_t *qw = qsigs + (uint64_t)q * k;
        uint32_t eq = 0, ej = 0, ee = 0;
        for (uint32_t g = 0; g < a.L; ++g) {
            uint32_t row[KPAD];
            load_group_row<KPAD, EXACT>(slab + s * k + (uint64_t)g * kp, kp, vec, row);
            const uint32_t *qg = qw + g * kp;
#pragma unroll
            for (int qd = 0; qd < KPAD / 4; ++qd) {
                const uint32_t vv[4] = {row[4 * qd], row[4 * qd + 1], row[4 * qd + 2], row[4 * qd + 3]};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int i = 4 * qd + t;
                    if (EXACT || i < (int)kp) {
                        const uint32_t qv = qg[i];
                        const bool se = vv[t] == HOPH_EMPTY;
                        eq += (vv[t] == qv) ? 1u : 0u;
                        if (qv == HOPH_EMPTY) {
                            ej += se ? 1u : 0u;
                            ee += 1u;
                        } else {
                            ee += se ? 1u : 0u;
                        }
                    }
                }
            }
        }
        const uint32_t m = eq - ej;
        bool accept;
        if (a.policy == HOPH_EMPTY_LITERAL) {
            accept = (uint64_t)m * td >= (uint64_t)tn * k;
        } else {
            const uint32_t e = a.policy == HOPH_EMPTY_JOINT ? ej : ee;
            if (e == k) accept = ej == k;
            else accept = (uint64_t)m * td >= (uint64_t)tn * (k - e);
        }
        accept = accept && valid;
        if (__any(accept)) {
            const uint64_t slot = wave_append(accept, counters + 1, lane);
            if (accept && slot < a.keys_cap) keys[slot] = ((uint64_t)q << 32) | s;
        }
    }
}

uint32_t waves_to_blocks(uint64_t waves) { return (uint32_t)((waves + kWaves - 1) / kWaves); }

CoarseArgs coarse_args(const ScanLaunch &l, uint32_t policy) {
    CoarseArgs a{};
    a.capacity = l.capacity;
    a.n_sets = l.n_sets;
    a.surv_cap = l.surv_cap;
    a.keys_cap = l.keys_cap;
    a.k = l.k;
    a.kp = l.kp;
    a.kpad = l.kpad;
    a.L = l.L;
    a.q0 = l.q0;
    a.q1 = l.q1;
    a.q_per_wave = l.q_per_wave;
    a.policy = policy;
    a.depth = l.codes ? 0u : l.depth;      // where the fine pass starts
    a.cg = l.cg;
    a.tri = l.tri ? 1u : 0u;
    a.pk = code_pack(l.kp, l.L);
    a.cdepth = l.depth;
    return a;
}

// The code pass over du code units held in VGPRs (du <= kMaxDepth): depth 1
// (JOINT or LITERAL) in scan_codes_fast_kernel, else scan_codes_kernel.
template <int W, bool PACK, bool UNITW>
void codes_launch(const ScanLaunch &l, const CoarseArgs &a, const ScanTab &tab, hipStream_t st, uint32_t blocks,
                  uint32_t du) {
    auto *cnt = reinterpret_cast<unsigned long long *>(l.counters);
#define HOPH_CODES(G)                                                                                         \
    hipLaunchKernelGGL((scan_codes_kernel<W, G, PACK, UNITW>), dim3(blocks), dim3(kThreads), 0, st, l.codes, \
                       l.qcodes, l.qmasks, l.surv, cnt, l.desc, a, tab)
    if (l.depth == 1 && tab.policy != HOPH_EMPTY_EITHER) {
        const FirstGroupPlan fg = first_group_plan(tab, l.kp, l.tri, !l.desc && l.q1 - l.q0 < kFast1MinQueries, l.keep_rate);
        const int split = fg.planes;
#define HOPH_FAST(P1, TRI)                                                                                     \
    hipLaunchKernelGGL((scan_codes_fast_kernel<W, fast_tiles(W, P1), P1, TRI>), dim3(blocks), dim3(kThreads), 0, st, \
                       l.codes, l.qcodes, l.surv, cnt, l.desc, a)
        if (l.tri && W == 1 && fg.fast1) {
#define HOPH_FAST1T(P1)                                                                                          \
    hipLaunchKernelGGL((scan_codes_fast1_kernel<fast1_tiles(P1), P1, true>), dim3(blocks), dim3(kThreads), 0, st, \
                       l.codes, l.qcodes, l.surv, cnt, l.desc, a)
            switch (split) {
            case 2: HOPH_FAST1T(2); break;
            case 3: HOPH_FAST1T(3); break;
            case 4: HOPH_FAST1T(4); break;
            case 5: HOPH_FAST1T(5); break;
            default: HOPH_FAST1T(6); break;
            }
#undef HOPH_FAST1T
        } else if (l.tri) {
            switch (split) {
            case 2: HOPH_FAST(2, true); break;
            case 3: HOPH_FAST(3, true); break;
            case 4: HOPH_FAST(4, true); break;
            case 5: HOPH_FAST(5, true); break;
            case 6: HOPH_FAST(6, true); break;
            default: HOPH_FAST(0, true); break;
            }
        } else if (W == 1 && fg.fast1) {
#define HOPH_FAST1(P1)                                                                                          \
    hipLaunchKernelGGL((scan_codes_fast1_kernel<fast1_tiles(P1), P1, false>), dim3(blocks), dim3(kThreads), 0, st, l.codes, \
                       l.qcodes, l.surv, cnt, l.desc, a)
            switch (split) {
            case 2: HOPH_FAST1(2); break;
            case 3: HOPH_FAST1(3); break;
            case 4: HOPH_FAST1(4); break;
            case 5: HOPH_FAST1(5); break;
            default: HOPH_FAST1(6); break;
            }
#undef HOPH_FAST1
        } else {
            switch (split) {
            case 2: HOPH_FAST(2, false); break;
            case 3: HOPH_FAST(3, false); break;
            case 4: HOPH_FAST(4, false); break;
            case 5: HOPH_FAST(5, false); break;
            case 6: HOPH_FAST(6, false); break;
            default: HOPH_FAST(0, false); break;
            }
        }
#undef HOPH_FAST
        return;
    }
    switch (du) {
    case 1: HOPH_CODES(1); break;
    case 2: HOPH_CODES(2); break;
    case 3: HOPH_CODES(3); break;
    default: HOPH_CODES(4); break;     // 4 units (deeper runs in scan_codes_deep_kernel)
    }
#undef HOPH_CODES
}

template <int KPAD, bool EXACT>
void coarse_launch(const ScanLaunch &l, const CoarseArgs &a, const ScanTab &tab, hipStream_t st, uint32_t blocks) {
    auto *cnt = reinterpret_cast<unsigned long long *>(l.counters);
#define HOPH_COARSE(G)                                                                                        \
    hipLaunchKernelGGL((scan_coarse_kernel<KPAD, G, EXACT>), dim3(blocks), dim3(kThreads), 0, st, l.slab,    \
                       l.qsigs, l.qmasks, l.surv, l.keys, cnt, l.desc, a, tab)
    switch (l.depth) {
    case 1: HOPH_COARSE(1); break;
    case 2: if constexpr (KPAD * 2 <= 128) HOPH_COARSE(2); break;
    case 3: if constexpr (KPAD * 3 <= 128) HOPH_COARSE(3); break;
    default: if constexpr (KPAD * 4 <= 128) HOPH_COARSE(4); break;
    }
#undef HOPH_COARSE
}

template <int KPAD>
void coarse_kp(const ScanLaunch &l, const CoarseArgs &a, const ScanTab &tab, hipStream_t st, uint32_t blocks) {
    if (l.kp == (uint32_t)KPAD) coarse_launch<KPAD, true>(l, a, tab, st, blocks);
    else coarse_launch<KPAD, false>(l, a, tab, st, blocks);
}

template <int KPAD>
void oph_kp(const ScanLaunch &l, const CoarseArgs &a, hoph_ratio T, hipStream_t st, uint32_t blocks) {
    auto *cnt = reinterpret_cast<unsigned long long *>(l.counters);
    if (l.kp == (uint32_t)KPAD)
        hipLaunchKernelGGL((oph_full_kernel<KPAD, true>), dim3(blocks), dim3(kThreads), 0, st, l.slab, l.qsigs, l.keys,
                           cnt, a, T.num, T.den);
    else
        hipLaunchKernelGGL((oph_full_kernel<KPAD, false>), dim3(blocks), dim3(kThreads), 0, st, l.slab, l.qsigs, l.keys,
                           cnt, a, T.num, T.den);
}

#define HOPH_KPAD_SWITCH(F, ...)                                       \
    switch (l.kpad) {                                                  \
    case 4: F<4>(__VA_ARGS__); break;                                  \
    case 8: F<8>(__VA_ARGS__); break;                                  \
    case 12: F<12>(__VA_ARGS__); break;                                \
    case 16: F<16>(__VA_ARGS__); break;                                \
    case 20: F<20>(__VA_ARGS__); break;                                \
    case 24: F<24>(__VA_ARGS__); break;                                \
    case 28: F<28>(__VA_ARGS__); break;                                \
    case 32: F<32>(__VA_ARGS__); break;                                \
    case 36: F<36>(__VA_ARGS__); break;                                \
    case 40: F<40>(__VA_ARGS__); break;                                \
    case 44: F<44>(__VA_ARGS__); break;                                \
    case 48: F<48>(__VA_ARGS__); break;                                \
    case 52: F<52>(__VA_ARGS__); break;                                \
    case 56: F<56>(__VA_ARGS__); break;                                \
    case 60: F<60>(__VA_ARGS__); break;                                \
    default: F<64>(__VA_ARGS__); break;                                \
    }

}  // namespace

void first_group_shape(const ScanTab &tab, uint32_t kp, bool tri, bool small_batch, const double *keep_rate,
                       uint32_t out[3]) {
    const FirstGroupPlan f = first_group_plan(tab, kp, tri, small_batch, keep_rate);
    out[0] = (uint32_t)f.planes;
    out[1] = f.fast1 ? 1u : 0u;
    out[2] = (uint32_t)f.tiles;
}

// Phase-1 lane keep rates of the first-group pass measured on the data: up to
// kKeepSample index rows spaced evenly over [0, n_sets), each as the query
// (its non-empty bins and keep threshold worked out from its planes as the
// query records hold them: a bin is empty where its code is 255, every plane
// set) against every other sampled row as the set; rate[p] (p = 2 .. 6) is
// the fraction of those ordered pairs with more agreeing bins on the first p
// planes than the query's threshold, as the kernels test it.  One strided copy
// of the first code unit's planes (one plane word) and a count on the host,
// on st (synchronised).  rate[] is all 0 when fewer than two rows.
constexpr uint32_t kKeepSample = 512;
hipError_t sample_keep_rates(const uint32_t *codes, uint64_t n_sets, uint32_t kp, const int32_t *dthr0,
                             double rate[8], hipStream_t st) {
    for (int p = 0; p < 8; ++p) rate[p] = 0.0;
    if (code_plane_words(kp) != 1 || n_sets < 2) return hipSuccess;
    constexpr uint32_t PW = kCodeBits;
    const uint32_t S = (uint32_t)std::min<uint64_t>(n_sets, kKeepSample);
    const uint64_t step = n_sets / S;
    uint32_t h[kKeepSample * PW];                        // row i's planes at h[i * PW]
    hipError_t e = hipMemcpy2DAsync(h, PW * sizeof(uint32_t), codes, step * PW * sizeof(uint32_t),
                                    PW * sizeof(uint32_t), S, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    const uint32_t kpmask = kp >= 32 ? 0xFFFFFFFFu : ((1u << kp) - 1u);
    uint32_t mask[kKeepSample];
    int32_t thr[kKeepSample];
    for (uint32_t i = 0; i < S; ++i) {
        uint32_t em = kpmask;
        for (uint32_t p = 0; p < PW; ++p) em &= h[i * PW + p];
        const uint32_t ne = (uint32_t)__builtin_popcount(em);
        mask[i] = ~em & kpmask;
        thr[i] = (int32_t)(kp - ne) - dthr0[ne];
    }
    uint64_t kept[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t i = 0; i < S; ++i) {
        const uint32_t *q = &h[i * PW];
        for (uint32_t j = 0; j < S; ++j) {
            if (j == i) continue;
            const uint32_t *c = &h[j * PW];
            uint32_t a = mask[i];
            for (int p = 0; p < 6; ++p) {
                a &= ~(q[p] ^ c[p]);
                if ((int32_t)__builtin_popcount(a) <= thr[i]) break;   // the chain only loses bins
                if (p >= 1) ++kept[p + 1];
            }
        }
    }
    const double pairs = (double)S * (double)(S - 1);
    for (int p = 2; p <= 6; ++p) rate[p] = (double)kept[p] / pairs;
    return hipSuccess;
}

// Whether the index and query parameters allow linear-bound records (see
// LinTab): code planes, one plane word (k' <= 32), one group per code unit,
// JOINT or LITERAL, not the self-join; then lin (if not null) gets the table
// for the first min(cg, kLinMaxSteps) groups.
bool lin_records(const ScanLaunch &l, const ScanTab &tab, LinTab *lin) {
    if (!l.codes || l.tri || l.kp > 32 || code_pack(l.kp, l.L) != 1) return false;
    if (tab.policy != HOPH_EMPTY_JOINT && tab.policy != HOPH_EMPTY_LITERAL) return false;
    if (lin) {
        std::memset(lin, 0, sizeof(*lin));
        lin->steps = std::min<uint32_t>(l.cg, kLinMaxSteps);
        lin->policy = tab.policy;
        lin->kp = l.kp;
        lin->lambda = tab.lambda;
        for (uint32_t e = 0; e <= l.kp; ++e) lin->dmul[e] = tab.dmul[e];
        // the largest C_g over every empty count: W_g lambda (JOINT, k' - e = 1) or W_g
        uint64_t cmax = 1;
        for (uint32_t g = 0; g < lin->steps; ++g) {
            lin->W[g] = tab.W[g];
            lin->acc[g] = tab.acc[g];
            lin->rej[g] = tab.rej[g];
            const uint64_t cg = (uint64_t)tab.W[g] * (tab.policy == HOPH_EMPTY_LITERAL ? 1u : (uint64_t)tab.lambda);
            cmax = std::max(cmax, cg);
        }
        // c_g below 2^24: one 24-bit multiply per group and a sum below 2^31 (4 groups x 32 bins)
        uint32_t bits = 0;
        while (bits < 64 && (cmax >> bits) != 0) ++bits;
        lin->shift = bits > 24 ? bits - 24 : 0;
    }
    return true;
}

// The first step (0-based) with a reject cutoff, or L.
static uint32_t first_reject_step(const ScanTab &tab) {
    uint32_t r = 0;
    while (r < tab.L && tab.rej[r] < 0) ++r;
    return r;
}

static bool lin_code_pass(const ScanLaunch &l, const ScanTab &tab, LinTab *lin) {
    if (!lin_records(l, tab, lin)) return false;
    const uint32_t du = l.depth;                     // one group per unit
    return du >= 2 && du <= kLinMaxSteps && du <= l.cg && first_reject_step(tab) < du;
}

// Tiles per wavefront of the linear-bound pass: 4 for two groups, else 2
// (the planes of D groups of TPW tiles stay in VGPRs); with a first phase
// (only its P1 <= 4 planes of G1 groups in VGPRs): 8 for one or two groups,
// else 4.
static constexpr int lin_tiles(int D) { return D == 2 ? 4 : 2; }
static constexpr int lin1_tiles(int G1) { return G1 <= 2 ? 8 : 4; }

// Planes of phase 1 of the linear-bound pass: a background pair matches a
// bin's first p planes with probability 2^-p, so phase 1 settles it when that
// fraction of matches, summed over the weighted groups 0..R, stays well below
// the reject cutoff of step R (a third of the largest reject fraction tau);
// 0: one phase over all 8 planes.
static int lin_plane_split(const ScanTab &tab, uint32_t kp, uint32_t R) {
    if (R >= tab.L || tab.rej[R] < 0) return 0;
    const double unit = tab.policy == HOPH_EMPTY_LITERAL ? 1.0 : (double)tab.dmul[0];
    double full = 0;
    for (uint32_t g = 0; g <= R; ++g) full += (double)tab.W[g] * unit * kp;
    const double tau = (double)tab.rej[R] / full;
    for (int p = 2; p <= 4; ++p)
        if (std::ldexp(1.0, -p) * 3.0 <= tau) return p;
    return 0;
}

uint32_t coarse_tiles_per_wave(const ScanLaunch &l, const ScanTab &tab) {
    const uint32_t policy = tab.policy;
    if (lin_code_pass(l, tab, nullptr)) {
        const uint32_t R = first_reject_step(tab);
        return (uint32_t)(lin_plane_split(tab, l.kp, R) > 0 ? lin1_tiles((int)R + 1) : lin_tiles((int)l.depth));
    }
    if (!(l.codes && l.depth == 1 && policy != HOPH_EMPTY_EITHER)) return 1u;
    return (uint32_t)first_group_plan(tab, l.kp, l.tri, !l.desc && l.q1 - l.q0 < kFast1MinQueries, l.keep_rate).tiles;
}

void describe_coarse(const ScanLaunch &l, const ScanTab &tab, uint32_t out[4]) {
    out[0] = l.depth;
    out[1] = l.codes ? HOPH_PLAN_CODES : HOPH_PLAN_WORDS;
    out[2] = 0;
    out[3] = coarse_tiles_per_wave(l, tab);
    if (!l.codes) return;
    if (lin_code_pass(l, tab, nullptr)) {
        const int p1 = lin_plane_split(tab, l.kp, first_reject_step(tab));
        out[1] = p1 > 0 ? HOPH_PLAN_LINEAR_LIGHT : HOPH_PLAN_LINEAR;
        out[2] = (uint32_t)p1;
    } else if (l.depth == 1 && tab.policy != HOPH_EMPTY_EITHER) {
        const FirstGroupPlan fg =
            first_group_plan(tab, l.kp, l.tri, !l.desc && l.q1 - l.q0 < kFast1MinQueries, l.keep_rate);
        out[1] = fg.fast1 ? HOPH_PLAN_FIRST_GROUP_LIGHT : HOPH_PLAN_FIRST_GROUP;
        out[2] = (uint32_t)fg.planes;
    }
}

uint32_t max_depth_for_kpad(uint32_t kpad) {
    uint32_t d = 128 / kpad;
    return d < kMaxDepth ? d : kMaxDepth;
}

hipError_t launch_query_masks(const uint32_t *qsigs, uint32_t n_q, const uint64_t *desc, uint32_t k, uint32_t kp,
                              uint32_t L, uint64_t *out, uint32_t *qcodes, uint32_t cg, const CodeThr *thr,
                              hipStream_t st, const LinTab *lin, uint64_t *zero, uint32_t n_zero) {
    if (qcodes && !thr) return hipErrorInvalidValue;
    if (n_zero > kThreads) return hipErrorInvalidValue;
    CodeThr t{};
    if (thr) t = *thr;
    LinTab lt;
    std::memset(&lt, 0, sizeof(lt));
    if (lin && qcodes) lt = *lin;
    const uint64_t n = (uint64_t)n_q * L;         // n_q: the batch size, or its upper bound with desc
    if (n == 0) return zero && n_zero ? launch_fill_u64(zero, n_zero, 0, st) : hipSuccess;
    uint64_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(query_masks_kernel, dim3((uint32_t)blocks), dim3(kThreads), 0, st, qsigs, n_q, desc, k, kp, L,
                       out, qcodes, cg, t, lt, zero, n_zero);
    return hipGetLastError();
}

hipError_t launch_scan_coarse(const ScanLaunch &l, const ScanTab &tab, hipStream_t st) {
    uint32_t blocks;
    if (l.desc) {
        // persistent: a fixed grid walks the (tile, query chunk) items of whatever batch desc describes
        blocks = waves_to_blocks((uint64_t)device_cu_count() * (l.waves_per_cu ? l.waves_per_cu : 16));
    } else {
        const uint64_t ntiles = (l.n_sets + 63) / 64;
        const uint32_t nq = l.q1 - l.q0;
        if (ntiles == 0 || nq == 0) return hipSuccess;
        const uint64_t nchunks = (nq + l.q_per_wave - 1) / l.q_per_wave;
        const uint32_t tpw = coarse_tiles_per_wave(l, tab);
        blocks = waves_to_blocks((ntiles + tpw - 1) / tpw * nchunks);
    }
    const CoarseArgs a = coarse_args(l, tab.policy);
    if (l.codes && lin_code_pass(l, tab, nullptr)) {
        // two to four groups with the linear bound (the query records carry its words)
        const uint32_t R = first_reject_step(tab);
        const int p1 = lin_plane_split(tab, l.kp, R);
        auto *cnt = reinterpret_cast<unsigned long long *>(l.counters);
        if (p1 > 0) {
            // phase-1 planes of groups 0..R in VGPRs, the rest read again where a lane is kept
#define HOPH_LIN1(G1, DD, P1)                                                                                    \
    hipLaunchKernelGGL((scan_codes_lin1_kernel<G1, DD, lin1_tiles(G1), P1>), dim3(blocks), dim3(kThreads), 0, st, \
                       l.codes, l.qcodes, l.surv, cnt, l.desc, a)
#define HOPH_LIN1_P(G1, DD)                  \
    do {                                     \
        if (p1 == 4) HOPH_LIN1(G1, DD, 4);   \
        else if (p1 == 3) HOPH_LIN1(G1, DD, 3); \
        else HOPH_LIN1(G1, DD, 2);           \
    } while (0)
            switch (l.depth * 4 + R) {
            case 2 * 4 + 0: HOPH_LIN1_P(1, 2); break;
            case 2 * 4 + 1: HOPH_LIN1_P(2, 2); break;
            case 3 * 4 + 0: HOPH_LIN1_P(1, 3); break;
            case 3 * 4 + 1: HOPH_LIN1_P(2, 3); break;
            case 3 * 4 + 2: HOPH_LIN1_P(3, 3); break;
            case 4 * 4 + 0: HOPH_LIN1_P(1, 4); break;
            case 4 * 4 + 1: HOPH_LIN1_P(2, 4); break;
            case 4 * 4 + 2: HOPH_LIN1_P(3, 4); break;
            default: HOPH_LIN1_P(4, 4); break;
            }
#undef HOPH_LIN1_P
#undef HOPH_LIN1
            return hipGetLastError();
        }
#define HOPH_LIN(DD, P1)                                                                                      \
    hipLaunchKernelGGL((scan_codes_lin_kernel<DD, lin_tiles(DD), P1>), dim3(blocks), dim3(kThreads), 0, st,   \
                       l.codes, l.qcodes, l.surv, cnt, l.desc, a, R)
#define HOPH_LIN_P(DD)                                 \
    do {                                               \
        if (p1 == 4) HOPH_LIN(DD, 4);                  \
        else if (p1 == 3) HOPH_LIN(DD, 3);             \
        else if (p1 == 2) HOPH_LIN(DD, 2);             \
        else HOPH_LIN(DD, 0);                          \
    } while (0)
        switch (l.depth) {
        case 2: HOPH_LIN_P(2); break;
        case 3: HOPH_LIN_P(3); break;
        default: HOPH_LIN_P(4); break;
        }
#undef HOPH_LIN_P
#undef HOPH_LIN
        return hipGetLastError();
    }
    if (l.codes) {
        if (l.depth == 0 || l.depth > l.cg) return hipErrorInvalidValue;
        const uint32_t W = code_plane_words(l.kp), pk = a.pk, du = (l.depth + pk - 1) / pk;   // code units walked
        const bool pack = pk > 1;            // only with one plane word (k' <= 16)
        bool unitw = true;                   // every weight the pass can reach is 1 (GOPH)
        for (uint32_t g = 0; g < std::min<uint32_t>(du * pk, tab.L); ++g) unitw = unitw && tab.W[g] == 1;
        if (du > kMaxDepth) {
            // past the register-resident units: one wavefront per block, planes staged in LDS
            if (du > max_code_units(l.kp)) return hipErrorInvalidValue;
            uint64_t waves;
            if (l.desc) {
                waves = (uint64_t)device_cu_count() * (l.waves_per_cu ? l.waves_per_cu : 16);
            } else {
                const uint64_t ntiles = (l.n_sets + 63) / 64;
                waves = ntiles * ((l.q1 - l.q0 + l.q_per_wave - 1) / l.q_per_wave);
            }
            const uint32_t deep_blocks = (uint32_t)std::min<uint64_t>(waves, 1u << 30);
            // Units held in VGPRs: 8 (no or little LDS staging, 4 wavefronts per SIMD
            // by registers) when a unit packs several groups or the first step that
            // can reject lies past the fourth unit, so that most pairs walk that far;
            // else 4, the rest staged only when a query reaches it (plain groups that
            // reject within 4 units: loading 8 up front cost 16% at k' = 32).
            uint32_t g1 = 0;                 // first step with a reject cutoff (0-based)
            while (g1 < l.depth && tab.rej[g1] < 0) ++g1;
            const bool r8 = W == 1 && du >= 8 && (pk > 1 || g1 / pk + 1 > kMaxDepth);
            const uint32_t R = r8 ? 8u : kMaxDepth;
            const size_t lds = (size_t)(du - R) * 64 * (code_words(l.kp) * 4 + 4 * W);
            auto *cnt = reinterpret_cast<unsigned long long *>(l.counters);
#define HOPH_DEEP(WW, PACK, RR)                                                                                \
    do {                                                                                                       \
        if (unitw)                                                                                             \
            hipLaunchKernelGGL((scan_codes_deep_kernel<WW, PACK, RR, true>), dim3(deep_blocks), dim3(64), lds,  \
                               st, l.codes, l.qcodes, l.qmasks, l.surv, cnt, l.desc, a, tab, du);               \
        else                                                                                                   \
            hipLaunchKernelGGL((scan_codes_deep_kernel<WW, PACK, RR, false>), dim3(deep_blocks), dim3(64), lds, \
                               st, l.codes, l.qcodes, l.qmasks, l.surv, cnt, l.desc, a, tab, du);               \
    } while (0)
            if (W == 1) {
                if (r8) {
                    if (pack) HOPH_DEEP(1, true, 8);
                    else HOPH_DEEP(1, false, 8);
                } else {
                    if (pack) HOPH_DEEP(1, true, 4);
                    else HOPH_DEEP(1, false, 4);
                }
            } else {
                HOPH_DEEP(2, false, 4);
            }
#undef HOPH_DEEP
            return hipGetLastError();
        }
        if (W == 1) {
            if (pack) {
                if (unitw) codes_launch<1, true, true>(l, a, tab, st, blocks, du);
                else codes_launch<1, true, false>(l, a, tab, st, blocks, du);
            } else {
                if (unitw) codes_launch<1, false, true>(l, a, tab, st, blocks, du);
                else codes_launch<1, false, false>(l, a, tab, st, blocks, du);
            }
        } else {
            if (unitw) codes_launch<2, false, true>(l, a, tab, st, blocks, du);
            else codes_launch<2, false, false>(l, a, tab, st, blocks, du);
        }
        return hipGetLastError();
    }
    HOPH_KPAD_SWITCH(coarse_kp, l, a, tab, st, blocks)
    return hipGetLastError();
}

hipError_t launch_scan_fine(const ScanLaunch &l, const ScanTab &tab, hipStream_t st) {
    if (!l.codes && l.depth >= l.L) return hipSuccess;
    const uint32_t blocks = (uint32_t)device_cu_count() * 8;
    const CoarseArgs a = coarse_args(l, tab.policy);
    hipLaunchKernelGGL(scan_fine_kernel, dim3(blocks), dim3(kThreads), 0, st, l.slab, l.qsigs, l.surv, l.keys,
                       reinterpret_cast<unsigned long long *>(l.counters), a, tab);
    return hipGetLastError();
}

hipError_t launch_pair_estimates(const uint32_t *slab, uint64_t n_sets, uint32_t k, uint32_t kp, uint32_t L,
                                 const uint32_t *qsigs, uint32_t n_q, const uint32_t *pairs, uint64_t n_pairs,
                                 uint32_t policy, const double *unions, int64_t *est, uint32_t *mb, uint32_t *eb,
                                 double *var, const ScanTab &tab, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    uint64_t blocks = (n_pairs + kWaves - 1) / kWaves;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(pair_estimates_kernel, dim3((uint32_t)blocks), dim3(kThreads), 0, st, slab, n_sets, k, kp, L,
                       qsigs, n_q, pairs, n_pairs, policy, unions, est, mb, eb, var, tab);
    return hipGetLastError();
}

hipError_t launch_oph_full(const ScanLaunch &l, hoph_ratio T, uint32_t policy, hipStream_t st) {
    const uint64_t ntiles = (l.n_sets + 63) / 64;
    const uint32_t nq = l.q1 - l.q0;
    if (ntiles == 0 || nq == 0) return hipSuccess;
    const uint64_t nchunks = (nq + l.q_per_wave - 1) / l.q_per_wave;
    const uint32_t blocks = waves_to_blocks(ntiles * nchunks);
    const CoarseArgs a = coarse_args(l, policy);
    HOPH_KPAD_SWITCH(oph_kp, l, a, T, st, blocks)
    return hipGetLastError();
}

}  // namespace hoph
