// Index storage.  The signature words are kept row-major, one row of k words
// per set, word (set s, bin b) at slab[s * k + b]: a set is sketched straight
// into its row, and the per-pair pass reads one group of one row as a
// contiguous run.  The coarse pass reads the narrowed code planes of the
// first cg groups instead, in code units of pk whole groups (ub = pk k' bins,
// code_pack), tiled so that a wavefront (one set per lane) reads them
// coalesced: PW = code_words(k') words per (set, unit u), plane p of the
// unit's bins [32 w, 32 w + 32) at word p * W + w (W = PW / 8),
//   codes[((u * (capacity / 64) + s / 64) * 64 + s % 64) * PW + p * W + w].
// The writers below take the unit as a group of ub bins.
#include "hoph_internal.h"

namespace hoph {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t value) {
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        p[i] = value;
}

// Reads p[0 .. n) (16-byte words) and keeps nothing: a measurement helper that
// replaces the caches' contents with clean lines.  The store below happens only
// when the words' XOR equals `never`, which the caller picks so that it does not
// (it keeps the loads from being removed).
__global__ __launch_bounds__(kThreads) void read_sweep_kernel(const uint4 *p, uint64_t n, uint32_t never,
                                                               uint32_t *sink) {
    uint32_t acc = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads) {
        const uint4 v = p[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == never) sink[blockIdx.x * kThreads + threadIdx.x] = acc;
}

// 8 x 8 bit transpose of a 64-bit word (byte r = row r, bit c = column c):
// three exchanges of off-diagonal blocks of 1, 2 and 4 bits.  Byte p of the
// result holds bit p of each of the eight input bytes.
__device__ __forceinline__ uint64_t transpose8x8(uint64_t x) {
    uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x = x ^ t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x = x ^ t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    return x ^ t ^ (t << 28);
}

// Code planes of the KP bins v[0..KP), written as PW contiguous words (bins
// past KP in a plane word are 0).  KP <= 32: the codes are packed as bytes,
// eight bins to a 64-bit word, and one bit transpose per word gives the eight
// plane bytes of those bins, which are then gathered into the plane words.
template <int KP>
__device__ __forceinline__ void store_code_planes(const uint32_t (&v)[KP], uint32_t *__restrict__ dst) {
    constexpr int W = KP > 32 ? 2 : 1;
    uint32_t pl[kCodeBits * W];
    if constexpr (KP <= 32) {
        uint32_t half[8];                    // plane bytes: half[2 j] bits 0..31, half[2 j + 1] bits 32..63 of word j
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (8 * j + b < KP) lo |= bin_code(v[8 * j + b]) << (8 * b);
                if (8 * j + 4 + b < KP) hi |= bin_code(v[8 * j + 4 + b]) << (8 * b);
            }
            const uint64_t x = (8 * j < KP) ? transpose8x8(((uint64_t)hi << 32) | lo) : 0ull;
            half[2 * j] = (uint32_t)x;
            half[2 * j + 1] = (uint32_t)(x >> 32);
        }
#pragma unroll
        for (int p = 0; p < (int)kCodeBits; ++p) {
            const int h = p >> 2, sh = 8 * (p & 3);
            pl[p] = ((half[h] >> sh) & 0xFFu) | (((half[2 + h] >> sh) & 0xFFu) << 8) |
                    (((half[4 + h] >> sh) & 0xFFu) << 16) | (((half[6 + h] >> sh) & 0xFFu) << 24);
        }
    } else {
#pragma unroll
        for (int j = 0; j < (int)kCodeBits * W; ++j) pl[j] = 0;
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            const uint32_t c = bin_code(v[i]);
#pragma unroll
            for (int p = 0; p < (int)kCodeBits; ++p) pl[p * W + (i >> 5)] |= ((c >> p) & 1u) << (i & 31);
        }
    }
    uint4 *d4 = reinterpret_cast<uint4 *>(dst);
#pragma unroll
    for (int j = 0; j < 2 * W; ++j) d4[j] = make_uint4(pl[4 * j], pl[4 * j + 1], pl[4 * j + 2], pl[4 * j + 3]);
}

// Code planes for an even unit width KP with k even: one thread per (row,
// unit < cg), the units of a row in consecutive lanes, so that a wavefront
// reads contiguous runs of the rows it covers (ordering the threads unit-major
// instead read 128 bytes of each 2 KB row per pass, at 0.45 against 0.29 ms
// for 10^6 rows of 9 units); a unit of a row is read as 16-byte loads (QUAD:
// KP and k multiples of 4) or 8-byte loads.  sigs row r is index row first + r.
template <int KP, bool QUAD>
__global__ __launch_bounds__(kThreads) void row_codes_vec_kernel(const uint32_t *__restrict__ sigs, uint64_t n_new,
                                                                uint64_t first, uint32_t k, uint64_t capacity,
                                                                uint32_t cg, uint32_t *__restrict__ codes) {
    static_assert(!QUAD || KP % 4 == 0, "16-byte loads need k' a multiple of 4");
    constexpr uint32_t PW = kCodeBits * (KP > 32 ? 2 : 1);
    const uint64_t total = n_new * cg;
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kThreads) {
        const uint64_t r = i / cg;           // the units of one row are adjacent threads: a wavefront
        const uint32_t g = (uint32_t)(i - r * cg);    // reads whole runs of each row it touches
        const uint64_t s = first + r;
        const uint32_t *row = sigs + r * k + (uint64_t)g * KP;
        uint32_t v[KP];
        if constexpr (QUAD) {
            const uint4 *src = reinterpret_cast<const uint4 *>(row);
#pragma unroll
            for (int u = 0; u < KP / 4; ++u) {
                const uint4 q = src[u];
                v[4 * u] = q.x;
                v[4 * u + 1] = q.y;
                v[4 * u + 2] = q.z;
                v[4 * u + 3] = q.w;
            }
        } else {
            const uint2 *src = reinterpret_cast<const uint2 *>(row);
#pragma unroll
            for (int u = 0; u < KP / 2; ++u) {
                const uint2 q = src[u];
                v[2 * u] = q.x;
                v[2 * u + 1] = q.y;
            }
        }
        store_code_planes<KP>(v, codes + (((uint64_t)g * (capacity / 64) + (s >> 6)) * 64 + (s & 63)) * PW);
    }
}

template <int KP>
void launch_row_codes(dim3 grid, dim3 block, hipStream_t st, const uint32_t *rows, uint64_t n_new, uint64_t first,
                      uint32_t k, uint64_t capacity, uint32_t cg, uint32_t *codes) {
    if constexpr (KP % 4 == 0) {
        if ((k & 3u) == 0) {
            hipLaunchKernelGGL((row_codes_vec_kernel<KP, true>), grid, block, 0, st, rows, n_new, first, k, capacity,
                               cg, codes);
            return;
        }
    }
    hipLaunchKernelGGL((row_codes_vec_kernel<KP, false>), grid, block, 0, st, rows, n_new, first, k, capacity, cg,
                       codes);
}

// Code planes of rows [first, first + n_new) from their signature rows (sigs
// row r is index row first + r), any unit width: one thread per (set, unit < cg),
// the units of a row in consecutive threads.
__global__ __launch_bounds__(kThreads) void index_codes_kernel(const uint32_t *__restrict__ sigs, uint64_t n_new,
                                                              uint64_t first, uint32_t k, uint32_t kp,
                                                              uint64_t capacity, uint32_t cg,
                                                              uint32_t *__restrict__ codes) {
    const uint32_t W = code_plane_words(kp), PW = code_words(kp);
    const uint64_t total = n_new * cg;
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kThreads) {
        const uint64_t r = i / cg;           // units of one row in adjacent threads
        const uint32_t g = (uint32_t)(i - r * cg);
        const uint64_t s = first + r;
        const uint32_t *row = sigs + r * k + (uint64_t)g * kp;
        uint32_t lo[kCodeBits], hi[kCodeBits];
#pragma unroll
        for (int p = 0; p < (int)kCodeBits; ++p) lo[p] = hi[p] = 0;
        for (uint32_t b = 0; b < kp; ++b) {
            const uint32_t c = bin_code(row[b]), bit = b & 31;
            if (b < 32) {
#pragma unroll
                for (int p = 0; p < (int)kCodeBits; ++p) lo[p] |= ((c >> p) & 1u) << bit;
            } else {
#pragma unroll
                for (int p = 0; p < (int)kCodeBits; ++p) hi[p] |= ((c >> p) & 1u) << bit;
            }
        }
        uint32_t *dst = codes + (((uint64_t)g * (capacity / 64) + (s >> 6)) * 64 + (s & 63)) * PW;
#pragma unroll
        for (int p = 0; p < (int)kCodeBits; ++p) {
            dst[p * W] = lo[p];
            if (W == 2) dst[p * W + 1] = hi[p];
        }
    }
}

// One wavefront per pair, one lane per bin: per-group (m, e) under a policy.
__global__ __launch_bounds__(kThreads) void pair_counts_kernel(const uint32_t *__restrict__ slab, uint64_t capacity,
                                                              uint64_t n_sets, uint32_t kpad, uint32_t kp, uint32_t L,
                                                              uint32_t k, const uint32_t *__restrict__ qsigs,
                                                              uint32_t n_q, const uint32_t *__restrict__ pairs,
                                                              uint64_t n_pairs, uint32_t policy,
                                                              uint32_t *__restrict__ mo, uint32_t *__restrict__ eo) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * (kThreads / 64);
    for (uint64_t p = (blockIdx.x * (uint64_t)kThreads + threadIdx.x) >> 6; p < n_pairs; p += nw) {
        const uint64_t q = pairs[2 * p], s = pairs[2 * p + 1];
        if (q >= n_q || s >= n_sets) {
            for (uint32_t g = lane; g < L; g += 64) {
                mo[p * L + g] = 0xFFFFFFFFu;
                eo[p * L + g] = 0xFFFFFFFFu;
            }
            continue;
        }
        for (uint32_t g = 0; g < L; ++g) {
            const bool in = lane < kp;
            uint32_t sw = 0, qv = 0;
            if (in) {
                sw = slab[s * k + (uint64_t)g * kp + lane];
                qv = qsigs[q * k + (uint64_t)g * kp + lane];
            }
            const uint64_t eqb = __ballot(in && sw == qv);
            const uint64_t qe = __ballot(in && qv == HOPH_EMPTY);
            const uint64_t se = __ballot(in && sw == HOPH_EMPTY);
            const uint32_t ej = __popcll(qe & se), ee = __popcll(qe | se);
            const uint32_t m = __popcll(eqb & ~qe);
            if (lane == 0) {
                mo[p * L + g] = m;
                eo[p * L + g] = policy == HOPH_EMPTY_JOINT ? ej : policy == HOPH_EMPTY_EITHER ? ee : 0u;
            }
        }
    }
}

__global__ void set_desc_kernel(uint64_t *desc, uint64_t a, uint64_t b) {
    desc[0] = a;
    desc[1] = b;
}

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap = 65536) {
    uint64_t g = (work + per_block - 1) / per_block;
    if (g == 0) g = 1;
    return (uint32_t)(g < cap ? g : cap);
}

}  // namespace

int device_cu_count() {
    static int cached[64] = {};
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev]) return cached[dev];
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cached[dev] = cus;
    return cus;
}

hipError_t launch_set_desc(uint64_t *desc, uint64_t a, uint64_t b, hipStream_t st) {
    hipLaunchKernelGGL(set_desc_kernel, dim3(1), dim3(1), 0, st, desc, a, b);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t value, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, kThreads, 4096)), dim3(kThreads), 0, st, p, n, value);
    return hipGetLastError();
}

hipError_t launch_read_sweep(const void *p, uint64_t bytes, uint32_t *sink, hipStream_t st) {
    const uint64_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(read_sweep_kernel, dim3(4096), dim3(kThreads), 0, st, static_cast<const uint4 *>(p), n,
                       0x9E3779B9u, sink);
    return hipGetLastError();
}

hipError_t launch_index_store(const uint32_t *sigs, uint64_t n_new, uint64_t first, uint32_t k, uint64_t capacity,
                              uint32_t *slab, uint32_t *codes, uint32_t ub, uint32_t cu, hipStream_t st) {
    if (n_new == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(slab + first * k, sigs, n_new * k * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    return launch_codes_from_slab(slab, capacity, k, ub, first, n_new, codes, cu, st);
}

bool codes_have_row_kernel(uint32_t k, uint32_t kp) { return (k % 2) == 0 && (kp % 2) == 0 && kp <= 64; }

hipError_t launch_codes_from_slab(const uint32_t *slab, uint64_t capacity, uint32_t k, uint32_t kp, uint64_t first,
                                  uint64_t n_new, uint32_t *codes, uint32_t cg, hipStream_t st) {
    if (n_new == 0 || cg == 0 || !codes) return hipSuccess;
    const dim3 grid(grid_for(n_new * cg, kThreads)), block(kThreads);
    const uint32_t *rows = slab + first * k;
    if (codes_have_row_kernel(k, kp)) {
        switch (kp) {
#define HOPH_ROW_CODES(KP)                                                                                      \
    case KP: launch_row_codes<KP>(grid, block, st, rows, n_new, first, k, capacity, cg, codes); break;
            HOPH_ROW_CODES(2) HOPH_ROW_CODES(4) HOPH_ROW_CODES(6) HOPH_ROW_CODES(8) HOPH_ROW_CODES(10)
            HOPH_ROW_CODES(12) HOPH_ROW_CODES(14) HOPH_ROW_CODES(16) HOPH_ROW_CODES(18) HOPH_ROW_CODES(20)
            HOPH_ROW_CODES(22) HOPH_ROW_CODES(24) HOPH_ROW_CODES(26) HOPH_ROW_CODES(28) HOPH_ROW_CODES(30)
            HOPH_ROW_CODES(32) HOPH_ROW_CODES(34) HOPH_ROW_CODES(36) HOPH_ROW_CODES(38) HOPH_ROW_CODES(40)
            HOPH_ROW_CODES(42) HOPH_ROW_CODES(44) HOPH_ROW_CODES(46) HOPH_ROW_CODES(48) HOPH_ROW_CODES(50)
            HOPH_ROW_CODES(52) HOPH_ROW_CODES(54) HOPH_ROW_CODES(56) HOPH_ROW_CODES(58) HOPH_ROW_CODES(60)
            HOPH_ROW_CODES(62) HOPH_ROW_CODES(64)
#undef HOPH_ROW_CODES
        default: return hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(index_codes_kernel, grid, block, 0, st, rows, n_new, first, k, kp, capacity, cg, codes);
    }
    return hipGetLastError();
}

hipError_t launch_pair_counts(const uint32_t *slab, uint64_t capacity, uint64_t n_sets, uint32_t kpad, uint32_t kp,
                              uint32_t L, uint32_t k, const uint32_t *qsigs, uint32_t n_q, const uint32_t *pairs,
                              uint64_t n_pairs, uint32_t policy, uint32_t *m, uint32_t *e, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(pair_counts_kernel, dim3(grid_for(n_pairs, kThreads / 64, 4096)), dim3(kThreads), 0, st,
                       slab, capacity, n_sets, kpad, kp, L, k, qsigs, n_q, pairs, n_pairs, policy, m, e);
    return hipGetLastError();
}

}  // namespace hoph
