// MinWise comparator (Sec. 1-2): k independent hashes (a_i x + b_i) mod p per
// element, each slot keeps its minimum; two sets are compared on all k slots.
// Sketch: one workgroup per set (persistent), a thread owns k / 256 slots and
// keeps their minima in registers while the set's ids are broadcast through LDS.
// Scan: one wavefront per indexed set, a lane owns k / 64 slots; equal slots
// are counted with ballots.
#include "hoph_internal.h"

namespace hoph {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxSlotsPerThread = 16;     // k <= 4096
constexpr int kChunk = 256;

template <uint32_t HASH, int SLOTS>
__global__ __launch_bounds__(kThreads) void minwise_sketch_kernel(uint32_t k, uint64_t universe,
                                                                  const uint64_t *__restrict__ ha,
                                                                  const uint64_t *__restrict__ hb,
                                                                  const uint32_t *__restrict__ ids,
                                                                  const uint64_t *__restrict__ offsets,
                                                                  uint64_t n_sets, uint64_t *__restrict__ sigs,
                                                                  uint32_t *__restrict__ err_flag) {
    __shared__ uint32_t s_ids[kChunk];
    __shared__ uint32_t s_n;
    const uint32_t tid = threadIdx.x;
    uint64_t a[SLOTS], b[SLOTS];
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
        const uint32_t h = tid + u * kThreads;
        a[u] = h < k ? ha[h] : 1;
        b[u] = h < k ? hb[h] : 0;
    }
    uint32_t err = 0;
    for (uint64_t set = blockIdx.x; set < n_sets; set += gridDim.x) {
        uint64_t mn[SLOTS];
#pragma unroll
        for (int u = 0; u < SLOTS; ++u) mn[u] = ~0ull;
        const uint64_t lo = offsets[set], hi = offsets[set + 1];
        if (hi == lo) err |= kErrEmptySet;
        for (uint64_t base = lo; base < hi; base += kChunk) {
            const uint32_t cnt = (uint32_t)min<uint64_t>(kChunk, hi - base);
            __syncthreads();
            if (tid < cnt) {
                const uint32_t x = ids[base + tid];
                if ((uint64_t)x >= universe) err |= kErrRange;
                s_ids[tid] = x;
            }
            if (tid == 0) s_n = cnt;
            __syncthreads();
            const uint32_t n = s_n;
            for (uint32_t j = 0; j < n; ++j) {
                const uint64_t x = s_ids[j];
                if (x >= universe) continue;
#pragma unroll
                for (int u = 0; u < SLOTS; ++u) {
                    const uint64_t v = HASH == HOPH_HASH_MODP31 ? psi_p31(x, a[u], b[u]) : psi_p32(x, a[u], b[u]);
                    mn[u] = v < mn[u] ? v : mn[u];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < SLOTS; ++u) {
            const uint32_t h = tid + u * kThreads;
            if (h < k) sigs[set * k + h] = mn[u];
        }
    }
    if (err) atomicOr(err_flag, err);
}

// One wavefront per indexed set; lane l owns slots l, l + 64, ...  The query
// rows [q0, q1) are compared in turn with the set's row held in registers.
template <int PER>
__global__ __launch_bounds__(kThreads) void minwise_scan_kernel(uint32_t k, const uint64_t *__restrict__ sigs,
                                                               uint64_t n_sets, const uint64_t *__restrict__ qsigs,
                                                               uint32_t q0, uint32_t q1, uint32_t tn, uint32_t td,
                                                               uint64_t *__restrict__ keys, uint64_t keys_cap,
                                                               uint64_t *__restrict__ counters) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * (kThreads / 64);
    for (uint64_t s = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) >> 6; s < n_sets; s += nw) {
        uint64_t row[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t h = lane + 64 * u;
            row[u] = h < k ? sigs[s * k + h] : 0;
        }
        for (uint32_t q = q0; q < q1; ++q) {
            uint32_t eq = 0;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t h = lane + 64 * u;
                const bool e = h < k && row[u] == qsigs[(uint64_t)q * k + h];
                eq += __popcll(__ballot(e));
            }
            if ((uint64_t)eq * td >= (uint64_t)tn * k && lane == 0) {
                const uint64_t slot = atomicAdd((unsigned long long *)(counters + 1), 1ull);
                if (slot < keys_cap) keys[slot] = ((uint64_t)q << 32) | s;
            }
        }
    }
}

template <uint32_t HASH>
hipError_t sketch_h(uint32_t k, uint64_t universe, const uint64_t *ha, const uint64_t *hb, const uint32_t *ids,
                    const uint64_t *offsets, uint64_t n_sets, uint64_t *sigs, uint32_t *err_flag, hipStream_t st,
                    uint32_t grid) {
    const uint32_t slots = (k + kThreads - 1) / kThreads;
#define HOPH_MW(S)                                                                                            \
    if (slots <= S) {                                                                                         \
        hipLaunchKernelGGL((minwise_sketch_kernel<HASH, S>), dim3(grid), dim3(kThreads), 0, st, k, universe, ha, \
                           hb, ids, offsets, n_sets, sigs, err_flag);                                         \
        return hipGetLastError();                                                                             \
    }
    HOPH_MW(1) HOPH_MW(2) HOPH_MW(4) HOPH_MW(8) HOPH_MW(16)
#undef HOPH_MW
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_minwise_sketch(uint32_t k, uint32_t hash, uint64_t universe, const uint64_t *ha, const uint64_t *hb,
                                 const uint32_t *ids, const uint64_t *offsets, uint64_t n_sets, uint64_t *sigs,
                                 uint32_t *err_flag, hipStream_t st) {
    if (n_sets == 0) return hipSuccess;
    const int cus = device_cu_count();
    const uint64_t want = (uint64_t)(cus > 0 ? cus : 256) * 8;
    const uint32_t grid = (uint32_t)(n_sets < want ? n_sets : want);
    if (hash == HOPH_HASH_MODP31)
        return sketch_h<HOPH_HASH_MODP31>(k, universe, ha, hb, ids, offsets, n_sets, sigs, err_flag, st, grid);
    return sketch_h<HOPH_HASH_MODP32P15>(k, universe, ha, hb, ids, offsets, n_sets, sigs, err_flag, st, grid);
}

hipError_t launch_minwise_scan(uint32_t k, const uint64_t *sigs, uint64_t n_sets, const uint64_t *qsigs, uint32_t q0,
                               uint32_t q1, hoph_ratio T, uint64_t *keys, uint64_t keys_cap, uint64_t *counters,
                               hipStream_t st) {
    if (n_sets == 0 || q1 <= q0) return hipSuccess;
    uint64_t blocks = (n_sets + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    const uint32_t per = (k + 63) / 64;
#define HOPH_MWS(P)                                                                                              \
    if (per <= P) {                                                                                              \
        hipLaunchKernelGGL((minwise_scan_kernel<P>), dim3((uint32_t)blocks), dim3(kThreads), 0, st, k, sigs, n_sets, \
                           qsigs, q0, q1, T.num, T.den, keys, keys_cap, counters);                               \
        return hipGetLastError();                                                                                \
    }
    HOPH_MWS(1) HOPH_MWS(2) HOPH_MWS(4) HOPH_MWS(8) HOPH_MWS(16) HOPH_MWS(32) HOPH_MWS(64)
#undef HOPH_MWS
    return hipErrorInvalidValue;
}

}  // namespace hoph
