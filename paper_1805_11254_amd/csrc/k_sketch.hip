// OPH / HOPH sketching (Sec. 3.2, Sec. 4.1): every element goes through the
// one shared permutation, lands in one of k contiguous bins of the permuted
// range, and each bin keeps its smallest offset from the bin start.
//
// One wavefront per set, persistent over sets (no workgroup barrier inside the
// set loop).  The bin-start table (32-bit where the permuted range fits) and,
// for layouts that need it, the region table and the region lookup table are
// built once per workgroup in LDS; each wavefront owns a k-word LDS signature
// updated with ds_min (the minimum is order-free, so the order of lanes does
// not matter) and written back with 16-byte stores.  Element ids are read with
// unconditional (clamped) coalesced loads from one load site, four per lane;
// the next four are in flight while the current ones are hashed and binned,
// and a set's first ids are read during the previous set's last batch.  The
// element path is straight-line code (out-of-range lanes are masked, only the
// LDS minimum is predicated) so the loads of the four elements interleave.
// An index append with no vector-load code-plane row kernel (odd k' or k) also
// writes the new rows' code planes from the LDS signature.
//
// Hash: the shared permutation is computed in 32-bit steps where it can be:
// (a x + b) mod (2^31 - 1) folds the high part once; (a x + b) mod (2^32 + 15)
// with a, b < 2^32 takes two 32 x 32 -> 64 multiply-adds and a carry
// (psi_p32_narrow), and only coefficients at or above 2^32 take the 64-bit
// reduction.  Every lookup reads the value's 32-bit view; the offset is the
// value's low 32 bits minus the bin start.
//
// Bin lookup: where regions and bins fall on powers of two (the 1:1 hierarchy
// and power-of-two k over R = 2^31 - 1) one read of a 32-entry table indexed
// by a leading-zero count gives the region, and a shift and a mask give the
// bin and the offset (LOC_POW2); where the bins are near-uniform (plain OPH,
// a:b = 1:1 HOPH) a 32-bit reciprocal estimate gives the bin or the one before
// it and one read of a pair of bin starts settles it (LOC_EST); narrow ranges
// with geometric regions find the region from log-domain cells (LOC_LOG);
// otherwise from the lookup table and the region's own reciprocal
// (LOC_REGION).
#include <algorithm>
#include <type_traits>

#include "hoph_internal.h"

namespace hoph {

namespace {

constexpr int kUnroll = 4;

constexpr int LOC_EST = 0, LOC_REGION = 1, LOC_LOG = 2, LOC_POW2 = 3;

// The (a x + b) mod (2^31 - 1) and (a x + b) mod (2^32 + 15) hashes look bins
// up in 32 bits (NARROW: values clamped to kNarrowTop, starts to 2^32 - 1, see
// narrow_value); the table hash keeps 64-bit values and starts.
template <uint32_t HASH>
constexpr bool kNarrow = HASH != HOPH_HASH_TABLE;

// The (a x + b) mod (2^32 + 15) hash with a, b < 2^32, in 32-bit steps
// (psi_p32_narrow): a template value of its own, which the host picks.
constexpr uint32_t kHashP32Small = 0x100u | HOPH_HASH_MODP32P15;

// The permuted value of id x as the narrow lookups read it: its 32-bit view
// and its low 32 bits.  (a x + b) mod (2^31 - 1) is reduced for x < P only, so
// its ids are clamped to the universe; the 2^32 + 15 forms take any 32-bit x.
template <uint32_t HASH>
__device__ __forceinline__ void permute_narrow(uint32_t x, uint32_t umax, const SketchDesc &d, uint32_t &view,
                                               uint32_t &low) {
    if constexpr (HASH == HOPH_HASH_MODP31) {
        view = low = (uint32_t)psi_p31(min(x, umax), d.ha, d.hb);     // below 2^31 - 1
    } else if constexpr (HASH == kHashP32Small) {
        psi_p32_narrow(x, (uint32_t)d.ha, (uint32_t)d.hb, view, low);
    } else {
        const uint64_t v = psi_p32(x, d.ha, d.hb);
        view = narrow_value(v);
        low = (uint32_t)v;
    }
}
template <uint32_t HASH>
using StartT = typename std::conditional<kNarrow<HASH>, uint32_t, uint64_t>::type;

// LDS layout of one workgroup (byte offsets, all 16-byte aligned).
struct SketchLds {
    uint32_t starts, reg, lut, sigs, sig_stride, total;
};

__host__ __device__ inline SketchLds sketch_lds(uint32_t k, uint32_t nr, uint32_t lut_size, uint32_t waves,
                                                bool narrow, int loc) {
    SketchLds l;
    l.starts = 0;
    l.reg = ((narrow ? 4u : 8u) * (k + 1) + 15u) & ~15u;
    uint32_t reg_bytes = 0, lut_bytes = 0;
    if (loc == LOC_REGION) {
        reg_bytes = narrow ? (8u * nr + 4u + 15u) & ~15u : 16u * (nr + 1);
        lut_bytes = nr > 1 ? lut_size : 0u;
    } else if (loc == LOC_LOG) {
        reg_bytes = 8u * nr;                       // {start, 32-bit reciprocal}
        lut_bytes = 8u * kLogCells;                // {first region, inner boundary}
    } else if (loc == LOC_POW2) {
        lut_bytes = 16u * kPow2Classes;            // {region start, shift, first bin, mask}
    }
    l.lut = (l.reg + reg_bytes + 15u) & ~15u;
    l.sigs = (l.lut + lut_bytes + 15u) & ~15u;
    l.sig_stride = (4u * k + 15u) & ~15u;
    l.total = l.sigs + l.sig_stride * waves;
    return l;
}

template <uint32_t HASH>
struct Tables {
    const StartT<HASH> *start;
    const RegionEntry *reg;                  // wide: {start, 64-bit reciprocal}, n_regions + 1
    const uint32_t *rstart, *rmag;           // narrow: region starts (n_regions + 1), 32-bit reciprocals
    const uint8_t *lut;
    const uint32_t (*cells)[2];              // log cells: {first region, inner boundary}
    const unsigned char *cells_f;            // the same table, 8 (127 * 16) bytes early (see cell_entry)
    const uint32_t (*regs)[2];               // log cells: {region start, 32-bit reciprocal}
    const uint4 *pow2;                       // power-of-two regions, by leading-zero count
};

// Builds the workgroup's LDS tables (call with the whole workgroup, then barrier).
template <uint32_t HASH, int LOC>
__device__ Tables<HASH> build_tables(const SketchDesc &d, unsigned char *smem, const SketchLds &L) {
    using S = StartT<HASH>;
    const uint32_t k = d.k, nr = d.n_regions, nb = d.nb, tid = threadIdx.x;
    Tables<HASH> t{};
    if constexpr (LOC == LOC_POW2) {
        // only the 32-entry table: no bin starts are read
        uint4 *pt = reinterpret_cast<uint4 *>(smem + L.lut);
        for (uint32_t c = tid; c < kPow2Classes; c += blockDim.x)
            pt[c] = make_uint4(d.pow2[c][0], d.pow2[c][1], d.pow2[c][2], d.pow2[c][3]);
        t.pow2 = pt;
        return t;
    }
    S *s_start = reinterpret_cast<S *>(smem + L.starts);
    for (uint32_t b = tid; b < k; b += blockDim.x) {
        const uint32_t r = b / nb, i = b - r * nb;
        const uint64_t z = d.reg_start[r + 1] - d.reg_start[r];
        const uint64_t s = d.reg_start[r] + ((uint64_t)i * z + nb - 1) / nb;
        if constexpr (kNarrow<HASH>) s_start[b] = narrow_start(s);
        else s_start[b] = (S)s;
    }
    if (tid == 0) {
        if constexpr (kNarrow<HASH>) s_start[k] = narrow_start(d.R);
        else s_start[k] = (S)d.R;
    }
    t.start = s_start;
    if constexpr (LOC == LOC_LOG) {
        uint32_t(*rg)[2] = reinterpret_cast<uint32_t(*)[2]>(smem + L.reg);
        uint32_t(*cl)[2] = reinterpret_cast<uint32_t(*)[2]>(smem + L.lut);
        for (uint32_t r = tid; r < nr; r += blockDim.x) {
            rg[r][0] = (uint32_t)d.reg_start[r];
            rg[r][1] = d.reg_mag32[r];
        }
        for (uint32_t c = tid; c < kLogCells; c += blockDim.x)
            log_cell_entry(c, narrow_r1(d.R) + 1u, d.reg_start, nr, cl[c][0], cl[c][1]);
        t.regs = rg;
        t.cells = cl;
        t.cells_f = reinterpret_cast<const unsigned char *>(cl) - 8u * 127u * 16u;
    }
    if constexpr (LOC == LOC_REGION) {
        if constexpr (kNarrow<HASH>) {
            uint32_t *rs = reinterpret_cast<uint32_t *>(smem + L.reg), *rm = rs + nr + 1;
            for (uint32_t r = tid; r <= nr; r += blockDim.x) rs[r] = narrow_start(d.reg_start[r]);
            for (uint32_t r = tid; r < nr; r += blockDim.x) rm[r] = d.reg_mag32[r];
            t.rstart = rs;
            t.rmag = rm;
        } else {
            RegionEntry *re = reinterpret_cast<RegionEntry *>(smem + L.reg);
            for (uint32_t r = tid; r <= nr; r += blockDim.x)
                re[r] = RegionEntry{d.reg_start[r], r < nr ? d.reg_magic[r] : 0ull};
            t.reg = re;
        }
        uint8_t *s_lut = smem + L.lut;
        if (nr > 1) {
            for (uint32_t g = tid; g < d.lut_size; g += blockDim.x) {
                const uint64_t v = (uint64_t)g << d.lut_shift;
                uint32_t r = 0;
                while (r + 1 < nr && v >= d.reg_start[r + 1]) ++r;
                s_lut[g] = (uint8_t)r;
            }
        }
        t.lut = s_lut;
    }
    return t;
}

// The cell table entry of v (log_cell): the f32 bits of u = max((R1 - v) >> 8, 1)
// hold 16 (e + 127) + m above bit 19, so the entry's byte offset is bits 16 and
// up, less 8 (127 * 16), which cells_f has taken off already.
template <uint32_t HASH>
__device__ __forceinline__ uint2 cell_entry(uint32_t v, uint32_t R1, const Tables<HASH> &t) {
    uint32_t u = (R1 - v) >> 8;
    u = u > 1u ? u : 1u;
    return *reinterpret_cast<const uint2 *>(t.cells_f + ((__float_as_uint((float)u) >> 16) & ~7u));
}

// locate_log with the cell entry read as above.
template <uint32_t HASH>
__device__ __forceinline__ void locate_log_f(uint32_t v, uint32_t R1, const Tables<HASH> &t, uint32_t nb,
                                             uint32_t &bin, uint32_t &start) {
    const uint2 e = cell_entry<HASH>(v, R1, t);
    const uint32_t r = e.x + (v >= e.y ? 1u : 0u);
    const uint32_t y = v - t.regs[r][0];
    const uint32_t b = mul_u24(r, nb) + (uint32_t)(((uint64_t)y * t.regs[r][1]) >> 32);   // r < 64, nb <= 4096
    const uint32_t s0 = t.start[b], s1 = t.start[b + 1];
    const bool up = v >= s1;
    bin = b + (up ? 1u : 0u);
    start = up ? s1 : s0;
}

// Bin of a narrow permuted value (view, low; see permute_narrow) and its
// offset from the bin start.
template <uint32_t HASH, int LOC>
__device__ __forceinline__ void bin_of_narrow(uint32_t view, uint32_t low, const SketchDesc &d,
                                              const Tables<HASH> &t, uint32_t &b, uint32_t &off) {
    if constexpr (LOC == LOC_POW2) {
        // the power-of-two lookup needs R <= 2^32 - 1 (view = low)
        uint32_t u = (uint32_t)(d.R - 1) - view;
        u = u > 1u ? u : 1u;
        const uint4 e = t.pow2[clz32(u)];          // few distinct entries: mostly broadcast reads
        const uint32_t dl = view - e.x;
        b = e.z + (dl >> e.y);
        off = dl & e.w;
    } else {
        uint32_t start;
        if constexpr (LOC == LOC_EST) {
            const uint32_t e = bin_estimate(view, d.est_mul, d.est_shift);
            const uint32_t s0 = t.start[e], s1 = t.start[e + 1];
            const bool up = view >= s1;
            b = e + (up ? 1u : 0u);
            start = up ? s1 : s0;
        } else if constexpr (LOC == LOC_LOG) {
            locate_log_f(view, narrow_r1(d.R), t, d.nb, b, start);
        } else {
            locate_narrow(view, t.lut, d.lut_shift, t.rstart, t.rmag, d.n_regions, d.nb, t.start, b, start);
        }
        off = low - start;                             // below 2^32 (the bin's width)
    }
}

// Bin of a table value v (64-bit starts) and its offset from the bin start.
template <int LOC>
__device__ __forceinline__ void bin_of_wide(uint64_t v, const SketchDesc &d, const Tables<HOPH_HASH_TABLE> &t,
                                            uint32_t &b, uint32_t &off) {
    uint64_t start;
    if constexpr (LOC == LOC_EST) locate_est(v, d.est_mul, d.est_shift, t.start, b, start);
    else locate(v, t.lut, d.lut_shift, t.reg, d.n_regions, d.nb, t.start, b, start);
    off = (uint32_t)(v - start);
}

// Hash, bin and fold into the LDS signature the elements base + lane + 64 u,
// u < kUnroll (FULL: all of them are below hi).  Ids are clamped to the
// universe (and table values to the range) so that every lookup stays in its
// table; the largest id and table value are kept per lane and an
// out-of-range one raises the range error once per wavefront (the signature of
// such a set is then unspecified).  In the last batch of a set, lanes past hi
// fold EMPTY into a bin of their own (bin lane mod k: no two such lanes of a
// wavefront hit one word), which changes nothing, and element groups with no
// element at all are skipped by a wave-uniform test; the path has no per-lane
// branch, and the groups' LDS reads are issued before any LDS minimum.
template <uint32_t HASH, int LOC, bool FULL>
__device__ __forceinline__ void add_elements(const SketchDesc &d, const Tables<HASH> &t, uint32_t *sig,
                                             const uint32_t (&x)[kUnroll], uint64_t base, uint64_t hi,
                                             uint32_t lane, uint32_t umax, uint32_t &xmax, uint64_t &vmax) {
    // every bin lookup before the first LDS minimum: the tables and the
    // signature share the workgroup's LDS, so a lookup written after a minimum
    // would wait for it
    uint32_t b[kUnroll], off[kUnroll];
    if constexpr (kNarrow<HASH>) {
        uint32_t view[kUnroll], low[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (!FULL && base + 64u * u >= hi) break;
            xmax = max(xmax, x[u]);
            permute_narrow<HASH>(x[u], umax, d, view[u], low[u]);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (!FULL && base + 64u * u >= hi) break;
            bin_of_narrow<HASH, LOC>(view[u], low[u], d, t, b[u], off[u]);
        }
    } else {
        uint64_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (!FULL && base + 64u * u >= hi) break;
            xmax = max(xmax, x[u]);
            v[u] = d.perm[min(x[u], umax)];
            vmax = max(vmax, v[u]);
            v[u] = min(v[u], d.R - 1);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (!FULL && base + 64u * u >= hi) break;
            bin_of_wide<LOC>(v[u], d, t, b[u], off[u]);
        }
    }
    if constexpr (FULL) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) atomicMin(&sig[b[u]], off[u]);
    } else {
        const uint32_t idle_bin = lane < d.k ? lane : lane % d.k;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (base + 64u * u >= hi) break;
            const bool in = base + lane + 64u * u < hi;
            atomicMin(&sig[in ? b[u] : idle_bin], in ? off[u] : HOPH_EMPTY);
        }
    }
}

// Range errors seen by a lane (the largest id, and table value, it folded).
template <uint32_t HASH>
__device__ __forceinline__ uint32_t range_error(const SketchDesc &d, uint32_t xmax, uint64_t vmax) {
    uint32_t e = (uint64_t)xmax >= d.universe ? kErrRange : 0u;
    if constexpr (HASH == HOPH_HASH_TABLE) e |= vmax >= d.R ? kErrRange : 0u;
    return e;
}

// The code planes of the first cu code units (ub bins each) of a finished LDS
// signature: one lane per bin, one ballot per code bit gives the plane words
// of 32 bins (the low and high halves: two units of ub <= 32 bins, or both
// words of one unit of up to 64 bins); lane 0 stores each unit's PW words.
// Bins past ub are 0.
__device__ __forceinline__ void sketch_code_planes(const uint32_t *sig, const CodeSink &cs, uint64_t set,
                                                   uint32_t lane) {
    const uint64_t row = cs.first + set;
    const uint64_t tile_off = (row >> 6) * 64 + (row & 63);
    const uint32_t ub = cs.ub;
    if (ub <= 32) {
        for (uint32_t g0 = 0; g0 < cs.cu; g0 += 2) {
            const uint32_t g = g0 + (lane >> 5), i = lane & 31;
            const bool in = g < cs.cu && i < ub;
            const uint32_t c = in ? bin_code(sig[g * ub + i]) : 0u;
            uint32_t lo[kCodeBits], hi[kCodeBits];
#pragma unroll
            for (int p = 0; p < (int)kCodeBits; ++p) {
                const uint64_t m = __ballot((c >> p) & 1u);
                lo[p] = (uint32_t)m;
                hi[p] = (uint32_t)(m >> 32);
            }
            if (lane == 0) {
                uint4 *d0 = reinterpret_cast<uint4 *>(cs.codes + ((uint64_t)g0 * cs.ctiles * 64 + tile_off) * 8);
                d0[0] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
                d0[1] = make_uint4(lo[4], lo[5], lo[6], lo[7]);
                if (g0 + 1 < cs.cu) {
                    uint4 *d1 =
                        reinterpret_cast<uint4 *>(cs.codes + ((uint64_t)(g0 + 1) * cs.ctiles * 64 + tile_off) * 8);
                    d1[0] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
                    d1[1] = make_uint4(hi[4], hi[5], hi[6], hi[7]);
                }
            }
        }
    } else {
        for (uint32_t g = 0; g < cs.cu; ++g) {
            const bool in = lane < ub;
            const uint32_t c = in ? bin_code(sig[g * ub + lane]) : 0u;
            uint32_t pl[2 * kCodeBits];
#pragma unroll
            for (int p = 0; p < (int)kCodeBits; ++p) {
                const uint64_t m = __ballot((c >> p) & 1u);
                pl[2 * p] = (uint32_t)m;
                pl[2 * p + 1] = (uint32_t)(m >> 32);
            }
            if (lane == 0) {
                uint4 *d = reinterpret_cast<uint4 *>(cs.codes + ((uint64_t)g * cs.ctiles * 64 + tile_off) * 16);
#pragma unroll
                for (int j = 0; j < 4; ++j) d[j] = make_uint4(pl[4 * j], pl[4 * j + 1], pl[4 * j + 2], pl[4 * j + 3]);
            }
        }
    }
}

// Orders one wavefront's LDS accesses (the signature is private to the wavefront).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// A batch of ids: the 64 kUnroll ids from p (wave-uniform), lane byte offsets
// off[u] = 4 (lane + 64 u) clamped to the range's last id (`last4` = 4 (n - 1),
// n >= 1 ids left from p): one load site with one clamp per load, so that the
// loads of the next batch stay in flight while the current batch is processed.
__device__ __forceinline__ void load_batch_at(const uint32_t *__restrict__ p, uint32_t last4,
                                              const uint32_t (&off)[kUnroll], uint32_t (&x)[kUnroll]) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(p);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) x[u] = *reinterpret_cast<const uint32_t *>(b + min(off[u], last4));
}

__device__ __forceinline__ uint32_t last_byte(uint64_t from, uint64_t end) {
    const uint64_t n = end - from;
    return (uint32_t)(n < 64u * kUnroll ? n - 1 : 64u * kUnroll - 1) * 4u;
}

// The elements [lo, hi) into the LDS signature.  x holds the first batch of
// [lo, hi) on entry; the next batch is read while the current one is
// processed, and during the last batch the first batch of the next set's range
// [nlo, nhi) (or, with none, this batch again) is read into x.
template <uint32_t HASH, int LOC>
__device__ __forceinline__ void sketch_range(const SketchDesc &d, const Tables<HASH> &t,
                                             const uint32_t *__restrict__ ids, uint64_t lo, uint64_t hi,
                                             uint64_t nlo, uint64_t nhi, const uint32_t (&off)[kUnroll],
                                             uint32_t (&x)[kUnroll], uint32_t *sig, uint32_t lane, uint32_t umax,
                                             uint32_t &xmax, uint64_t &vmax) {
    constexpr uint32_t B = 64u * kUnroll;
    if (hi <= lo) {
        if (nlo < nhi) load_batch_at(ids + nlo, last_byte(nlo, nhi), off, x);
        return;
    }
    for (uint64_t base = lo; base < hi; base += B) {
        const uint64_t next = base + B;
        const bool more = next < hi, ahead = nlo < nhi;
        const uint64_t src = more ? next : (ahead ? nlo : base);
        const uint64_t end = more ? hi : (ahead ? nhi : hi);
        uint32_t xn[kUnroll];
        load_batch_at(ids + src, last_byte(src, end), off, xn);
        if (base + B <= hi) add_elements<HASH, LOC, true>(d, t, sig, x, base, hi, lane, umax, xmax, vmax);
        else add_elements<HASH, LOC, false>(d, t, sig, x, base, hi, lane, umax, xmax, vmax);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) x[u] = xn[u];
    }
}

template <uint32_t HASH, int LOC, bool CODES>
__global__ __launch_bounds__(256) void sketch_kernel(SketchDesc d, const uint32_t *__restrict__ ids,
                                                     const uint64_t *__restrict__ offsets, uint64_t n_sets,
                                                     uint32_t *__restrict__ sigs, uint32_t *__restrict__ err_flag,
                                                     const CodeSink cs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t k = d.k;
    const uint32_t waves = blockDim.x >> 6;
    const SketchLds L = sketch_lds(k, d.n_regions, d.lut_size, waves, kNarrow<HASH>, LOC);
    const Tables<HASH> t = build_tables<HASH, LOC>(d, smem, L);
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *sig = reinterpret_cast<uint32_t *>(smem + L.sigs + L.sig_stride * wib);
    const bool vec_out = (k & 3u) == 0 && (reinterpret_cast<uintptr_t>(sigs) & 15u) == 0;
    uint32_t err = 0, xmax = 0;
    uint64_t vmax = 0;
    const uint32_t umax = (uint32_t)(d.universe - 1);
    const uint64_t wstride = (uint64_t)gridDim.x * waves;
    uint32_t off[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) off[u] = 4u * (lane + 64u * u);
    uint64_t set = (uint64_t)blockIdx.x * waves + wib, lo = 0, hi = 0;
    uint32_t x[kUnroll];
    if (set < n_sets) {
        lo = offsets[set];
        hi = offsets[set + 1];
        if (lo < hi) load_batch_at(ids + lo, last_byte(lo, hi), off, x);
    }
    for (; set < n_sets; set += wstride) {
        const uint64_t nset = set + wstride;
        uint64_t nlo = 0, nhi = 0;
        if (nset < n_sets) {
            nlo = offsets[nset];
            nhi = offsets[nset + 1];
        }
        for (uint32_t b = lane; b < k; b += 64) sig[b] = HOPH_EMPTY;
        wave_lds_fence();
        if (hi <= lo) err |= hi == lo ? kErrEmptySet : kErrBadRange;   // a decreasing range reads nothing
        sketch_range<HASH, LOC>(d, t, ids, lo, hi, nlo, nhi, off, x, sig, lane, umax, xmax, vmax);
        wave_lds_fence();
        uint32_t *out = sigs + set * k;
        if (vec_out) {
            const uint4 *src = reinterpret_cast<const uint4 *>(sig);
            uint4 *dst = reinterpret_cast<uint4 *>(out);
            for (uint32_t i = lane; i < k / 4; i += 64) dst[i] = src[i];
        } else {
            for (uint32_t i = lane; i < k; i += 64) out[i] = sig[i];
        }
        if constexpr (CODES) sketch_code_planes(sig, cs, set, lane);
        wave_lds_fence();
        lo = nlo;
        hi = nhi;
    }
    err |= range_error<HASH>(d, xmax, vmax);
    if (err) atomicOr(err_flag, err);
}

// Chunk counts of the sets of a batch: prefix[i] = chunks of sets [0, i),
// a set of m ids has ceil(m / chunk) chunks (at least 1).  One workgroup.
// A set's id range, clamped to the staged ids [0, max_ids); a malformed range
// (decreasing, or past the staged ids) is empty.
__device__ __forceinline__ void set_range(const uint64_t *offsets, uint64_t i, uint64_t max_ids, uint64_t &lo,
                                          uint64_t &hi) {
    lo = offsets[i];
    hi = offsets[i + 1];
    if (hi < lo || hi > max_ids) hi = lo = 0;
}

__global__ __launch_bounds__(1024) void chunk_prefix_kernel(const uint64_t *__restrict__ offsets,
                                                           const uint64_t *__restrict__ desc, uint32_t chunk,
                                                           uint64_t max_ids, uint64_t *__restrict__ prefix) {
    __shared__ uint64_t s_part[1024];
    __shared__ uint64_t s_carry;
    const uint32_t n = (uint32_t)desc[0];
    const uint32_t t = threadIdx.x;
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + t;
        uint64_t v = 0;
        if (i < n) {
            uint64_t lo, hi;
            set_range(offsets, i, max_ids, lo, hi);
            const uint64_t m = hi - lo;
            v = m == 0 ? 1 : (m + chunk - 1) / chunk;
        }
        s_part[t] = v;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            const uint64_t add = t >= d ? s_part[t - d] : 0;
            __syncthreads();
            s_part[t] += add;
            __syncthreads();
        }
        if (i < n) prefix[i] = s_carry + s_part[t] - v;
        __syncthreads();
        if (t == 1023) s_carry += s_part[t];
        __syncthreads();
    }
    if (t == 0) prefix[n] = s_carry;
}

__global__ __launch_bounds__(256) void fill_sigs_kernel(uint32_t *__restrict__ sigs, const uint64_t *__restrict__ desc,
                                                       uint32_t k) {
    const uint64_t n = desc[0] * (uint64_t)k;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) sigs[i] = HOPH_EMPTY;
}

// Persistent sketch of a batch whose size is read from desc[0]: work items are
// chunks of sets (prefix from chunk_prefix_kernel); a wavefront sketches its
// chunk into an LDS signature and merges it into the global signature with
// atomicMin (the sketch of a union is the elementwise minimum of the sketches).
// The global signatures must be EMPTY beforehand (fill_sigs_kernel).
template <uint32_t HASH, int LOC>
__global__ __launch_bounds__(256) void sketch_chunked_kernel(SketchDesc d, const uint32_t *__restrict__ ids,
                                                             const uint64_t *__restrict__ offsets,
                                                             const uint64_t *__restrict__ desc,
                                                             const uint64_t *__restrict__ prefix, uint32_t chunk,
                                                             uint64_t max_ids, uint32_t *__restrict__ sigs,
                                                             uint32_t *__restrict__ err_flag) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t k = d.k;
    const uint32_t waves = blockDim.x >> 6;
    const SketchLds L = sketch_lds(k, d.n_regions, d.lut_size, waves, kNarrow<HASH>, LOC);
    const Tables<HASH> t = build_tables<HASH, LOC>(d, smem, L);
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *sig = reinterpret_cast<uint32_t *>(smem + L.sigs + L.sig_stride * wib);
    const uint64_t n_sets = desc[0];
    const uint64_t n_items = prefix[n_sets];
    uint32_t err = 0, xmax = 0;
    uint64_t vmax = 0;
    const uint32_t umax = (uint32_t)(d.universe - 1);
    const uint64_t wstride = (uint64_t)gridDim.x * waves;
    for (uint64_t item = (uint64_t)blockIdx.x * waves + wib; item < n_items; item += wstride) {
        // the set holding this item: the last set whose prefix is <= item
        uint64_t lo_s = 0, hi_s = n_sets;
        while (hi_s - lo_s > 1) {
            const uint64_t mid = (lo_s + hi_s) >> 1;
            if (prefix[mid] <= item) lo_s = mid; else hi_s = mid;
        }
        const uint64_t set = lo_s;
        const uint64_t c = item - prefix[set];
        uint64_t s_lo, s_hi;
        set_range(offsets, set, max_ids, s_lo, s_hi);
        if (s_hi == s_lo) {
            err |= kErrEmptySet;
            continue;
        }
        const uint64_t lo = s_lo + c * chunk;
        const uint64_t hi = min(s_hi, lo + chunk);
        for (uint32_t b = lane; b < k; b += 64) sig[b] = HOPH_EMPTY;
        wave_lds_fence();
        uint32_t off[kUnroll], x[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) off[u] = 4u * (lane + 64u * u);
        if (lo < hi) load_batch_at(ids + lo, last_byte(lo, hi), off, x);
        sketch_range<HASH, LOC>(d, t, ids, lo, hi, 0, 0, off, x, sig, lane, umax, xmax, vmax);
        wave_lds_fence();
        uint32_t *out = sigs + set * k;
        for (uint32_t b = lane; b < k; b += 64) {
            const uint32_t v = sig[b];
            if (v != HOPH_EMPTY) atomicMin(&out[b], v);
        }
        wave_lds_fence();
    }
    err |= range_error<HASH>(d, xmax, vmax);
    if (err) atomicOr(err_flag, err);
}

// Waves per workgroup (LDS at most 48 KB per workgroup) and its LDS bytes.
template <uint32_t HASH, int LOC>
void sketch_shape(const SketchDesc &d, uint32_t &waves, size_t &lds) {
    waves = 4;
    auto bytes = [&](uint32_t w) {
        return sketch_lds(d.k, d.n_regions, d.lut_size, w, kNarrow<HASH>, LOC).total;
    };
    while (waves > 1 && bytes(waves) > 48 * 1024) waves >>= 1;
    lds = bytes(waves);
}

template <typename K>
hipError_t allow_lds(K kern, size_t lds) {
    if (lds > 64 * 1024)
        return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    return hipSuccess;
}

template <uint32_t HASH, int LOC>
hipError_t launch_t(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets, uint64_t n_sets,
                    uint32_t *sigs, uint32_t *err_flag, hipStream_t st, const CodeSink &cs) {
    uint32_t waves;
    size_t lds;
    sketch_shape<HASH, LOC>(d, waves, lds);
    const uint64_t want_waves = (uint64_t)device_cu_count() * 32;
    uint64_t grid = (n_sets + waves - 1) / waves;
    if (grid > want_waves / waves) grid = want_waves / waves;
    if (grid == 0) grid = 1;
    auto kern = cs.codes ? sketch_kernel<HASH, LOC, true> : sketch_kernel<HASH, LOC, false>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(64 * waves), lds, st, d, ids, offsets, n_sets, sigs,
                       err_flag, cs);
    return hipGetLastError();
}

template <uint32_t HASH, int LOC>
hipError_t launch_chunked_t(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets, const uint64_t *desc,
                            const uint64_t *prefix, uint32_t chunk, uint64_t max_ids, uint32_t *sigs,
                            uint32_t *err_flag, uint32_t waves_per_cu, hipStream_t st) {
    uint32_t waves;
    size_t lds;
    sketch_shape<HASH, LOC>(d, waves, lds);
    const uint32_t grid = (uint32_t)((uint64_t)device_cu_count() * (waves_per_cu ? waves_per_cu : 16) / waves);
    auto kern = sketch_chunked_kernel<HASH, LOC>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid ? grid : 1), dim3(64 * waves), lds, st, d, ids, offsets, desc, prefix, chunk,
                       max_ids, sigs, err_flag);
    return hipGetLastError();
}

// Whether the (a x + b) mod (2^32 + 15) coefficients fit psi_p32_narrow.
bool p32_small(const SketchDesc &d) { return (d.ha >> 32) == 0 && (d.hb >> 32) == 0; }

}  // namespace

hipError_t launch_sketch_chunked(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets,
                                 const uint64_t *desc, uint64_t *prefix, uint32_t chunk, uint32_t max_sets,
                                 uint64_t max_ids, uint32_t *sigs, uint32_t *err_flag, uint32_t waves_per_cu,
                                 hipStream_t st) {
    hipLaunchKernelGGL(chunk_prefix_kernel, dim3(1), dim3(1024), 0, st, offsets, desc, chunk, max_ids, prefix);
    uint64_t fill_blocks = ((uint64_t)max_sets * d.k + 255) / 256;
    if (fill_blocks > 4096) fill_blocks = 4096;
    if (fill_blocks == 0) fill_blocks = 1;
    hipLaunchKernelGGL(fill_sigs_kernel, dim3((uint32_t)fill_blocks), dim3(256), 0, st, sigs, desc, d.k);
#define HOPH_SKC(H, LOC) \
    launch_chunked_t<H, LOC>(d, ids, offsets, desc, prefix, chunk, max_ids, sigs, err_flag, waves_per_cu, st)
    const bool est = d.est_ok != 0;
    switch (d.hash) {
    case HOPH_HASH_TABLE: return est ? HOPH_SKC(HOPH_HASH_TABLE, LOC_EST) : HOPH_SKC(HOPH_HASH_TABLE, LOC_REGION);
    case HOPH_HASH_MODP31:
        return d.pow2_ok ? HOPH_SKC(HOPH_HASH_MODP31, LOC_POW2)
               : est     ? HOPH_SKC(HOPH_HASH_MODP31, LOC_EST)
               : d.log_ok ? HOPH_SKC(HOPH_HASH_MODP31, LOC_LOG)
                          : HOPH_SKC(HOPH_HASH_MODP31, LOC_REGION);
    default:
        if (p32_small(d))
            return est        ? HOPH_SKC(kHashP32Small, LOC_EST)
                   : d.log_ok ? HOPH_SKC(kHashP32Small, LOC_LOG)
                              : HOPH_SKC(kHashP32Small, LOC_REGION);
        return est        ? HOPH_SKC(HOPH_HASH_MODP32P15, LOC_EST)
               : d.log_ok ? HOPH_SKC(HOPH_HASH_MODP32P15, LOC_LOG)
                          : HOPH_SKC(HOPH_HASH_MODP32P15, LOC_REGION);
    }
#undef HOPH_SKC
}

hipError_t launch_sketch(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets, uint64_t n_sets,
                         uint32_t *sigs, uint32_t *err_flag, hipStream_t st, const CodeSink &cs) {
    if (n_sets == 0) return hipSuccess;
    if (cs.codes && (cs.cu == 0 || cs.ub == 0 || cs.ub > 64 || (uint64_t)cs.cu * cs.ub > d.k))
        return hipErrorInvalidValue;
    const bool est = d.est_ok != 0;
#define HOPH_SK(H, LOC) launch_t<H, LOC>(d, ids, offsets, n_sets, sigs, err_flag, st, cs)
    switch (d.hash) {
    case HOPH_HASH_TABLE: return est ? HOPH_SK(HOPH_HASH_TABLE, LOC_EST) : HOPH_SK(HOPH_HASH_TABLE, LOC_REGION);
    case HOPH_HASH_MODP31:
        return d.pow2_ok ? HOPH_SK(HOPH_HASH_MODP31, LOC_POW2)
               : est     ? HOPH_SK(HOPH_HASH_MODP31, LOC_EST)
               : d.log_ok ? HOPH_SK(HOPH_HASH_MODP31, LOC_LOG)
                          : HOPH_SK(HOPH_HASH_MODP31, LOC_REGION);
    default:
        if (p32_small(d))
            return est        ? HOPH_SK(kHashP32Small, LOC_EST)
                   : d.log_ok ? HOPH_SK(kHashP32Small, LOC_LOG)
                              : HOPH_SK(kHashP32Small, LOC_REGION);
        return est        ? HOPH_SK(HOPH_HASH_MODP32P15, LOC_EST)
               : d.log_ok ? HOPH_SK(HOPH_HASH_MODP32P15, LOC_LOG)
                          : HOPH_SK(HOPH_HASH_MODP32P15, LOC_REGION);
    }
#undef HOPH_SK
}

}  // namespace hoph
