// Canonical output: accepted (query, set) pairs as 64-bit keys
// (query << 32 | set) are sorted with a bitonic network, then turned into a
// per-query CSR (offsets by binary search, set ids by truncation).  The order
// of appends in the scan is not deterministic; the sorted output is.
#include "hoph_internal.h"

namespace hoph {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kSeg = 4096;        // keys sorted inside one workgroup (32 KiB of LDS)

__device__ __forceinline__ void cswap(uint64_t &x, uint64_t &y, bool up) {
    if ((x > y) == up) {
        const uint64_t t = x;
        x = y;
        y = t;
    }
}

__global__ __launch_bounds__(kThreads) void fill_u32_kernel_for_seg(uint32_t *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads) p[i] = 0;
}

// Pad [n, N) with the largest key.
__global__ __launch_bounds__(kThreads) void pad_kernel(uint64_t *keys, uint64_t n, uint64_t N) {
    for (uint64_t i = n + blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < N; i += (uint64_t)gridDim.x * kThreads)
        keys[i] = ~0ull;
}

// Stages of size <= kSeg (or, with k_fixed, the substages j < kSeg of stage
// k_fixed) inside one workgroup's segment.
__global__ __launch_bounds__(kThreads) void bitonic_local(uint64_t *keys, uint64_t k_fixed) {
    __shared__ uint64_t s[kSeg];
    const uint64_t base = (uint64_t)blockIdx.x * kSeg;
    for (uint32_t i = threadIdx.x; i < kSeg; i += kThreads) s[i] = keys[base + i];
    __syncthreads();
    const uint64_t k_lo = k_fixed ? k_fixed : 2, k_hi = k_fixed ? k_fixed : kSeg;
    for (uint64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (uint32_t j = (uint32_t)((k_fixed ? kSeg : k) >> 1); j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < kSeg / 2; t += kThreads) {
                const uint32_t i = 2 * t - (t & (j - 1));    // lower index of the pair
                const uint64_t gi = base + i;
                cswap(s[i], s[i + j], (gi & k) == 0);
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < kSeg; i += kThreads) keys[base + i] = s[i];
}

// One substage j >= kSeg of stage k over the whole array.
__global__ __launch_bounds__(kThreads) void bitonic_global(uint64_t *keys, uint64_t N, uint64_t k, uint64_t j) {
    for (uint64_t t = blockIdx.x * (uint64_t)kThreads + threadIdx.x; t < N / 2; t += (uint64_t)gridDim.x * kThreads) {
        const uint64_t i = 2 * t - (t & (j - 1));
        uint64_t x = keys[i], y = keys[i + j];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
            keys[i] = y;
            keys[i + j] = x;
        }
    }
}

__global__ __launch_bounds__(kThreads) void results_kernel(const uint64_t *__restrict__ keys, uint64_t n, uint32_t n_q,
                                                          uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids) {
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    const uint64_t t0 = blockIdx.x * (uint64_t)kThreads + threadIdx.x;
    for (uint64_t q = t0; q <= n_q; q += stride) {
        // first position whose query is >= q
        uint64_t lo = 0, hi = n;
        const uint64_t target = q << 32;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (keys[mid] < target) lo = mid + 1; else hi = mid;
        }
        offsets[q] = lo;
    }
    for (uint64_t i = t0; i < n; i += stride) ids[i] = (uint32_t)(keys[i] & 0xFFFFFFFFull);
}

uint32_t grid_for(uint64_t work) {
    uint64_t g = (work + kThreads - 1) / kThreads;
    if (g == 0) g = 1;
    return (uint32_t)(g < 16384 ? g : 16384);
}

}  // namespace

uint64_t sort_capacity(uint64_t n) {
    uint64_t N = kSeg;
    while (N < n) N <<= 1;
    return N;
}

hipError_t launch_sort_keys(uint64_t *keys, uint64_t n, uint64_t N, hipStream_t st) {
    if (n <= 1) return hipSuccess;
    hipLaunchKernelGGL(pad_kernel, dim3(grid_for(N - n)), dim3(kThreads), 0, st, keys, n, N);
    hipLaunchKernelGGL(bitonic_local, dim3((uint32_t)(N / kSeg)), dim3(kThreads), 0, st, keys, 0ull);
    for (uint64_t k = 2ull * kSeg; k <= N; k <<= 1) {
        for (uint64_t j = k >> 1; j >= kSeg; j >>= 1)
            hipLaunchKernelGGL(bitonic_global, dim3(grid_for(N / 2)), dim3(kThreads), 0, st, keys, N, k, j);
        hipLaunchKernelGGL(bitonic_local, dim3((uint32_t)(N / kSeg)), dim3(kThreads), 0, st, keys, k);
    }
    return hipGetLastError();
}

hipError_t launch_results(const uint64_t *keys, uint64_t n, uint32_t n_q, uint64_t *offsets, uint32_t *set_ids,
                          hipStream_t st) {
    hipLaunchKernelGGL(results_kernel, dim3(grid_for((n > n_q ? n : n_q) + 1)), dim3(kThreads), 0, st, keys, n, n_q,
                       offsets, set_ids);
    return hipGetLastError();
}

}  // namespace hoph

// ---------------------------------------------------------------------------
// Per-query output without a global sort (usable with no host
// synchronisation, e.g. inside a captured graph): count the accepted keys of
// every query, scan the counts into CSR offsets, scatter the set ids, then sort
// each query's ids in LDS (at most seg_max <= kSegMaxLimit ids per query, a
// power of two chosen by the caller).  A query with more than seg_max ids, or a
// total above the output capacity, raises a flag so the caller can take the
// global-sort path instead.
// ---------------------------------------------------------------------------
namespace hoph {

namespace {

constexpr uint32_t kSegMaxLimit = 16384;   // 64 KB of LDS
constexpr int kScanThreads = 1024;

__device__ __forceinline__ uint64_t count_of(const uint64_t *counters, uint64_t cap) {
    const uint64_t c = counters[1];
    return c < cap ? c : cap;
}

__device__ __forceinline__ uint32_t nq_of(const uint64_t *desc, uint32_t n_q) {
    return desc ? (uint32_t)desc[0] : n_q;
}

__global__ __launch_bounds__(kThreads) void seg_count_kernel(const uint64_t *__restrict__ keys,
                                                            const uint64_t *__restrict__ counters, uint64_t keys_cap,
                                                            uint32_t *__restrict__ qcount) {
    const uint64_t n = count_of(counters, keys_cap);
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        atomicAdd(&qcount[keys[i] >> 32], 1u);
}

// One workgroup: exclusive scan of qcount[0..n_q) into offsets[0..n_q] and
// cursor[0..n_q); flags bit 0: a query has more than seg_max ids; bit 1: the
// total exceeds out_cap.  counters[2] receives the total.  Chunks of
// 4 kScanThreads counts: each thread reads four consecutive counts (one 16-byte
// load where the chunk is whole), a wavefront scans its threads' sums with
// shuffles, and the wavefront totals are combined through LDS (two barriers
// per chunk).
__global__ __launch_bounds__(kScanThreads) void seg_scan_kernel(const uint32_t *__restrict__ qcount,
                                                               const uint64_t *__restrict__ desc, uint32_t n_q_arg,
                                                               uint64_t *__restrict__ offsets,
                                                               uint64_t *__restrict__ cursor, uint64_t out_cap,
                                                               uint64_t *__restrict__ counters, uint32_t seg_max) {
    constexpr uint32_t kW = kScanThreads / 64;
    __shared__ uint64_t s_w[kW];
    __shared__ uint32_t s_big;
    const uint32_t n_q = nq_of(desc, n_q_arg);
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) s_big = 0;
    uint64_t carry = 0;
    uint32_t big = 0;
    for (uint64_t base = 0; base < n_q; base += 4ull * kScanThreads) {
        const uint64_t q0 = base + 4ull * t;
        uint32_t a[4] = {0, 0, 0, 0};
        if (q0 + 4 <= n_q) {
            const uint4 v = *reinterpret_cast<const uint4 *>(qcount + q0);   // qcount is 16-byte aligned
            a[0] = v.x;
            a[1] = v.y;
            a[2] = v.z;
            a[3] = v.w;
        } else {
            for (uint32_t i = 0; i < 4; ++i)
                if (q0 + i < n_q) a[i] = qcount[q0 + i];
        }
        uint64_t tsum = 0;
        for (uint32_t i = 0; i < 4; ++i) {
            big |= a[i] > seg_max ? 1u : 0u;
            tsum += a[i];
        }
        uint64_t inc = tsum;                                  // inclusive scan over the wavefront
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t o = __shfl_up(inc, d, 64);
            if (lane >= d) inc += o;
        }
        if (lane == 63) s_w[wv] = inc;
        __syncthreads();
        uint64_t before = 0, chunk = 0;
        for (uint32_t w = 0; w < kW; ++w) {
            const uint64_t x = s_w[w];
            before += w < wv ? x : 0;
            chunk += x;
        }
        uint64_t run = carry + before + inc - tsum;
        for (uint32_t i = 0; i < 4; ++i) {
            if (q0 + i < n_q) {
                offsets[q0 + i] = run;
                cursor[q0 + i] = run;
            }
            run += a[i];
        }
        carry += chunk;
        __syncthreads();                                      // s_w is rewritten by the next chunk
    }
    if (big) atomicOr(&s_big, 1u);
    __syncthreads();
    if (t == 0) {
        offsets[n_q] = carry;
        counters[2] = carry;
        counters[3] = (s_big ? 1ull : 0ull) | (carry > out_cap ? 2ull : 0ull);
    }
}

__global__ __launch_bounds__(kThreads) void seg_scatter_kernel(const uint64_t *__restrict__ keys,
                                                              const uint64_t *__restrict__ counters, uint64_t keys_cap,
                                                              unsigned long long *__restrict__ cursor,
                                                              uint32_t *__restrict__ ids, uint64_t out_cap) {
    const uint64_t n = count_of(counters, keys_cap);
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads) {
        const uint64_t key = keys[i];
        const uint64_t pos = atomicAdd(&cursor[key >> 32], 1ull);
        if (pos < out_cap) ids[pos] = (uint32_t)(key & 0xFFFFFFFFull);
    }
}

// One workgroup per query (grid-stride): bitonic sort of the query's ids in LDS.
__global__ __launch_bounds__(kThreads) void seg_sort_kernel(const uint64_t *__restrict__ offsets,
                                                           const uint64_t *__restrict__ desc, uint32_t n_q_arg,
                                                           uint32_t *__restrict__ ids, uint64_t out_cap,
                                                           uint32_t seg_max) {
    extern __shared__ uint32_t s[];          // seg_max words
    const uint32_t n_q = nq_of(desc, n_q_arg);
    for (uint32_t q = blockIdx.x; q < n_q; q += gridDim.x) {
        const uint64_t lo = offsets[q], hi = offsets[q + 1];
        const uint64_t len = hi - lo;
        if (len <= 1 || len > seg_max || hi > out_cap) continue;     // uniform per workgroup
        uint32_t N = 2;
        while (N < len) N <<= 1;
        for (uint32_t i = threadIdx.x; i < N; i += kThreads) s[i] = i < len ? ids[lo + i] : 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t k = 2; k <= N; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t t = threadIdx.x; t < N / 2; t += kThreads) {
                    const uint32_t i = 2 * t - (t & (j - 1));
                    const uint32_t x = s[i], y = s[i + j];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        s[i] = y;
                        s[i + j] = x;
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < len; i += kThreads) ids[lo + i] = s[i];
        __syncthreads();
    }
}

// One workgroup: the whole output stage of a batch with at most kSmallOutKeys
// accepted keys (query row << 32 | set id): the keys sorted in LDS (bitonic),
// which orders them by row and then by set id, each row's offset found by a
// binary search for its first key, the ids written in that order, and
// counters[2] = the total, counters[3] = 2 when it exceeds out_cap.  More
// keys (or more than keys_cap) write nothing but counters[3] = 4, and the
// caller runs the general stage.
__global__ __launch_bounds__(kScanThreads) void seg_small_kernel(const uint64_t *__restrict__ keys,
                                                                uint64_t *__restrict__ counters, uint64_t keys_cap,
                                                                const uint64_t *__restrict__ desc, uint32_t n_q_arg,
                                                                uint64_t *__restrict__ offsets,
                                                                uint32_t *__restrict__ ids, uint64_t out_cap) {
    __shared__ uint64_t s[kSmallOutKeys];
    const uint32_t t = threadIdx.x;
    const uint32_t n_q = nq_of(desc, n_q_arg);
    const uint64_t acc = counters[1];
    if (acc > kSmallOutKeys || acc > keys_cap) {         // uniform: every thread reads the same count
        if (t == 0) counters[3] = 4;
        return;
    }
    const uint32_t A = (uint32_t)acc;
    uint32_t N = 2;
    while (N < A) N <<= 1;
    for (uint32_t i = t; i < N; i += kScanThreads) s[i] = i < A ? keys[i] : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t u = t; u < N / 2; u += kScanThreads) {
                const uint32_t i = 2 * u - (u & (j - 1));
                const uint64_t x = s[i], y = s[i + j];
                if ((x > y) == ((i & k) == 0)) {
                    s[i] = y;
                    s[i + j] = x;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t q = t; q <= n_q; q += kScanThreads) {
        const uint64_t first = (uint64_t)q << 32;          // row q's first key is the first >= this
        uint32_t lo = 0, hi = A;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s[mid] < first) lo = mid + 1;
            else hi = mid;
        }
        offsets[q] = lo;
    }
    for (uint32_t i = t; i < A && i < out_cap; i += kScanThreads) ids[i] = (uint32_t)(s[i] & 0xFFFFFFFFull);
    if (t == 0) {
        counters[2] = A;
        counters[3] = A > out_cap ? 2ull : 0ull;
    }
}

}  // namespace

hipError_t launch_small_output(const uint64_t *keys, uint64_t *counters, uint64_t keys_cap, const uint64_t *desc,
                               uint32_t n_q, uint64_t *offsets, uint32_t *ids, uint64_t out_cap, hipStream_t st) {
    hipLaunchKernelGGL(seg_small_kernel, dim3(1), dim3(kScanThreads), 0, st, keys, counters, keys_cap, desc, n_q,
                       offsets, ids, out_cap);
    return hipGetLastError();
}

hipError_t launch_segmented_output(const uint64_t *keys, const uint64_t *counters_ro, uint64_t keys_cap,
                                   uint32_t *qcount, const uint64_t *desc, uint32_t n_q, uint64_t *offsets,
                                   uint64_t *cursor, uint32_t *ids, uint64_t out_cap, uint64_t *counters,
                                   uint32_t max_queries, uint64_t max_keys, uint32_t seg_max, hipStream_t st) {
    if (seg_max < 2 || seg_max > kSegMaxLimit || (seg_max & (seg_max - 1))) return hipErrorInvalidValue;
    // counts
    const uint64_t nqc = (uint64_t)max_queries + 1;
    hipLaunchKernelGGL(fill_u32_kernel_for_seg, dim3(grid_for(nqc)), dim3(kThreads), 0, st, qcount, nqc);
    hipLaunchKernelGGL(seg_count_kernel, dim3(grid_for(max_keys)), dim3(kThreads), 0, st, keys, counters_ro, keys_cap,
                       qcount);
    hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, qcount, desc, n_q, offsets, cursor, out_cap,
                       counters, seg_max);
    hipLaunchKernelGGL(seg_scatter_kernel, dim3(grid_for(max_keys)), dim3(kThreads), 0, st, keys, counters_ro, keys_cap,
                       reinterpret_cast<unsigned long long *>(cursor), ids, out_cap);
    uint32_t blocks = max_queries < 4096 ? (max_queries ? max_queries : 1) : 4096;
    hipLaunchKernelGGL(seg_sort_kernel, dim3(blocks), dim3(kThreads), (size_t)seg_max * 4, st, offsets, desc, n_q, ids,
                       out_cap, seg_max);
    return hipGetLastError();
}

}  // namespace hoph
