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
