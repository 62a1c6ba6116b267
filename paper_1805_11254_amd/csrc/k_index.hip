// Index build: signatures (row-major, one row of k words per set) are stored
// group by group (the comparison order of Sec. 3.3 / Sec. 4.1) in slabs whose
// tiles hold 64 sets -- one wavefront -- with the words of a bin quad of the 64
// sets contiguous:
//   word (set s, group g, bin i) at
//   slab[g * capacity * kpad + (s / 64) * kpad * 64 + (i / 4) * 256 + (s % 64) * 4 + i % 4]
// so that a wavefront reads a tile's group with fully coalesced 16-byte loads,
// one set per lane.  kpad = k' rounded up to 4; pad words hold EMPTY and are
// never compared.
#include "hoph_internal.h"

namespace hoph {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t value) {
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        p[i] = value;
}

// 16-byte path: k' and k multiples of 4, source 16-byte aligned.
// thread -> (group g, tile t, quad qd, lane): writes one 16-byte chunk.
__global__ __launch_bounds__(kThreads) void index_store_vec(const uint32_t *__restrict__ sigs, uint64_t n_new,
                                                           uint64_t first, uint32_t k, uint32_t kp, uint32_t L,
                                                           uint64_t capacity, uint64_t tile0, uint64_t ntiles,
                                                           uint32_t *__restrict__ slab) {
    const uint32_t nq = kp / 4;
    const uint64_t total = (uint64_t)L * ntiles * nq * 64;
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kThreads) {
        const uint32_t lane = (uint32_t)(i & 63);
        uint64_t rest = i >> 6;
        const uint32_t qd = (uint32_t)(rest % nq);
        rest /= nq;
        const uint64_t t = tile0 + rest % ntiles;
        const uint32_t g = (uint32_t)(rest / ntiles);
        const uint64_t s = t * 64 + lane;
        if (s < first || s >= first + n_new) continue;
        const uint4 v = *reinterpret_cast<const uint4 *>(sigs + (s - first) * k + (uint64_t)g * kp + qd * 4);
        uint4 *dst = reinterpret_cast<uint4 *>(slab + (uint64_t)g * capacity * kp + t * kp * 64 + qd * 256 + lane * 4);
        *dst = v;
    }
}

// word path for any k'
__global__ __launch_bounds__(kThreads) void index_store_word(const uint32_t *__restrict__ sigs, uint64_t n_new,
                                                            uint64_t first, uint32_t k, uint32_t kp, uint32_t kpad,
                                                            uint32_t L, uint64_t capacity, uint64_t tile0,
                                                            uint64_t ntiles, uint32_t *__restrict__ slab) {
    const uint64_t total = (uint64_t)L * ntiles * kpad * 64;
    for (uint64_t i = blockIdx.x * (uint64_t)kThreads + threadIdx.x; i < total; i += (uint64_t)gridDim.x * kThreads) {
        const uint32_t w = (uint32_t)(i & 3);
        const uint32_t lane = (uint32_t)((i >> 2) & 63);
        uint64_t rest = i >> 8;
        const uint32_t qd = (uint32_t)(rest % (kpad / 4));
        rest /= (kpad / 4);
        const uint64_t t = tile0 + rest % ntiles;
        const uint32_t g = (uint32_t)(rest / ntiles);
        const uint64_t s = t * 64 + lane;
        if (s < first || s >= first + n_new) continue;
        const uint32_t bin = qd * 4 + w;
        const uint32_t v = bin < kp ? sigs[(s - first) * k + (uint64_t)g * kp + bin] : HOPH_EMPTY;
        slab[(uint64_t)g * capacity * kpad + t * kpad * 64 + qd * 256 + lane * 4 + w] = v;
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
                sw = slab[(uint64_t)g * capacity * kpad + (s / 64) * kpad * 64 + (lane / 4) * 256 + (s % 64) * 4 + lane % 4];
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

hipError_t launch_index_store(const uint32_t *sigs, uint64_t n_new, uint64_t first, uint32_t k, uint32_t kp,
                              uint32_t L, uint32_t kpad, uint64_t capacity, uint32_t *slab, hipStream_t st) {
    if (n_new == 0) return hipSuccess;
    const uint64_t tile0 = first / 64, tile1 = (first + n_new - 1) / 64;
    const uint64_t ntiles = tile1 - tile0 + 1;
    const bool vec = (kp % 4 == 0) && (k % 4 == 0) && ((reinterpret_cast<uintptr_t>(sigs) & 15u) == 0);
    if (vec) {
        const uint64_t total = (uint64_t)L * ntiles * (kp / 4) * 64;
        hipLaunchKernelGGL(index_store_vec, dim3(grid_for(total, kThreads)), dim3(kThreads), 0, st, sigs, n_new,
                           first, k, kp, L, capacity, tile0, ntiles, slab);
    } else {
        const uint64_t total = (uint64_t)L * ntiles * kpad * 64;
        hipLaunchKernelGGL(index_store_word, dim3(grid_for(total, kThreads)), dim3(kThreads), 0, st, sigs, n_new,
                           first, k, kp, kpad, L, capacity, tile0, ntiles, slab);
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
