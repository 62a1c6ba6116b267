// OPH / HOPH sketching (Sec. 3.2, Sec. 4.1): every element goes through the
// one shared permutation, lands in one of k contiguous bins of the permuted
// range, and each bin keeps its smallest offset from the bin start.
//
// One wavefront per set, persistent over sets (no workgroup barrier inside the
// set loop).  The bin-start table, the region table and the region lookup
// table are built once per workgroup in LDS; each wavefront owns a k-word LDS
// signature updated with ds_min (the minimum is order-free, so the order of
// lanes does not matter) and written back with 16-byte stores.  Element ids
// are read with unconditional (clamped) coalesced loads, four per lane in
// flight.
#include "hoph_internal.h"

namespace hoph {

namespace {

constexpr int kUnroll = 4;

template <uint32_t HASH>
__device__ __forceinline__ uint64_t permute(uint64_t x, const SketchDesc &d) {
    if constexpr (HASH == HOPH_HASH_TABLE) {
        return d.perm[x];
    } else if constexpr (HASH == HOPH_HASH_MODP31) {
        return psi_p31(x, d.ha, d.hb);
    } else {
        return psi_p32(x, d.ha, d.hb);
    }
}

// LDS layout of one workgroup (byte offsets, all 16-byte aligned).
struct SketchLds {
    uint32_t starts, reg, lut, sigs, sig_stride, total;
};

__host__ __device__ inline SketchLds sketch_lds(uint32_t k, uint32_t nr, uint32_t lut_size, uint32_t waves) {
    SketchLds l;
    l.starts = 0;
    l.reg = (8u * (k + 1) + 15u) & ~15u;
    l.lut = l.reg + 16u * (nr + 1);
    l.sigs = (l.lut + (nr > 1 ? lut_size : 0u) + 15u) & ~15u;
    l.sig_stride = (4u * k + 15u) & ~15u;
    l.total = l.sigs + l.sig_stride * waves;
    return l;
}

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <uint32_t HASH, bool HIER>
__global__ __launch_bounds__(256) void sketch_kernel(SketchDesc d, const uint32_t *__restrict__ ids,
                                                     const uint64_t *__restrict__ offsets, uint64_t n_sets,
                                                     uint32_t *__restrict__ sigs, uint32_t *__restrict__ err_flag) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t k = d.k, nr = d.n_regions, nb = d.nb;
    const uint32_t waves = blockDim.x >> 6;
    const SketchLds L = sketch_lds(k, nr, d.lut_size, waves);
    uint64_t *s_start = reinterpret_cast<uint64_t *>(smem + L.starts);
    RegionEntry *s_reg = reinterpret_cast<RegionEntry *>(smem + L.reg);
    uint8_t *s_lut = smem + L.lut;
    const uint32_t tid = threadIdx.x;

    for (uint32_t r = tid; r <= nr; r += blockDim.x)
        s_reg[r] = RegionEntry{d.reg_start[r], r < nr ? d.reg_magic[r] : 0ull};
    for (uint32_t b = tid; b < k; b += blockDim.x) {
        const uint32_t r = b / nb, t = b - r * nb;
        const uint64_t z = d.reg_start[r + 1] - d.reg_start[r];
        s_start[b] = d.reg_start[r] + ((uint64_t)t * z + nb - 1) / nb;
    }
    if (tid == 0) s_start[k] = d.R;
    if constexpr (HIER) {
        for (uint32_t g = tid; g < d.lut_size; g += blockDim.x) {
            const uint64_t v = (uint64_t)g << d.lut_shift;
            uint32_t r = 0;
            while (r + 1 < nr && v >= d.reg_start[r + 1]) ++r;
            s_lut[g] = (uint8_t)r;
        }
    }
    __syncthreads();

    const uint32_t lane = tid & 63;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(tid >> 6);
    uint32_t *sig = reinterpret_cast<uint32_t *>(smem + L.sigs + L.sig_stride * wib);
    const bool vec_out = (k & 3u) == 0 && (reinterpret_cast<uintptr_t>(sigs) & 15u) == 0;
    uint32_t err = 0;
    const uint64_t wstride = (uint64_t)gridDim.x * waves;
    for (uint64_t set = (uint64_t)blockIdx.x * waves + wib; set < n_sets; set += wstride) {
        for (uint32_t b = lane; b < k; b += 64) sig[b] = HOPH_EMPTY;
        wave_lds_fence();
        const uint64_t lo = offsets[set], hi = offsets[set + 1];
        if (hi == lo) err |= kErrEmptySet;
        for (uint64_t base = lo; base < hi; base += 64 * kUnroll) {
            uint32_t x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t j = base + lane + 64u * u;
                x[u] = ids[j < hi ? j : hi - 1];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t j = base + lane + 64u * u;
                if (j >= hi) continue;
                if ((uint64_t)x[u] >= d.universe) { err |= kErrRange; continue; }
                const uint64_t v = permute<HASH>(x[u], d);
                if constexpr (HASH == HOPH_HASH_TABLE) {
                    if (v >= d.R) { err |= kErrRange; continue; }
                }
                uint32_t b;
                uint64_t start;
                locate(v, s_lut, d.lut_shift, s_reg, HIER ? nr : 1u, nb, s_start, b, start);
                atomicMin(&sig[b], (uint32_t)(v - start));
            }
        }
        wave_lds_fence();
        uint32_t *out = sigs + set * k;
        if (vec_out) {
            const uint4 *src = reinterpret_cast<const uint4 *>(sig);
            uint4 *dst = reinterpret_cast<uint4 *>(out);
            for (uint32_t i = lane; i < k / 4; i += 64) dst[i] = src[i];
        } else {
            for (uint32_t i = lane; i < k; i += 64) out[i] = sig[i];
        }
        wave_lds_fence();
    }
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
template <uint32_t HASH, bool HIER>
__global__ __launch_bounds__(256) void sketch_chunked_kernel(SketchDesc d, const uint32_t *__restrict__ ids,
                                                             const uint64_t *__restrict__ offsets,
                                                             const uint64_t *__restrict__ desc,
                                                             const uint64_t *__restrict__ prefix, uint32_t chunk,
                                                             uint64_t max_ids, uint32_t *__restrict__ sigs,
                                                             uint32_t *__restrict__ err_flag) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t k = d.k, nr = d.n_regions, nb = d.nb;
    const uint32_t waves = blockDim.x >> 6;
    const SketchLds L = sketch_lds(k, nr, d.lut_size, waves);
    uint64_t *s_start = reinterpret_cast<uint64_t *>(smem + L.starts);
    RegionEntry *s_reg = reinterpret_cast<RegionEntry *>(smem + L.reg);
    uint8_t *s_lut = smem + L.lut;
    const uint32_t tid = threadIdx.x;
    for (uint32_t r = tid; r <= nr; r += blockDim.x)
        s_reg[r] = RegionEntry{d.reg_start[r], r < nr ? d.reg_magic[r] : 0ull};
    for (uint32_t b = tid; b < k; b += blockDim.x) {
        const uint32_t r = b / nb, t = b - r * nb;
        const uint64_t z = d.reg_start[r + 1] - d.reg_start[r];
        s_start[b] = d.reg_start[r] + ((uint64_t)t * z + nb - 1) / nb;
    }
    if (tid == 0) s_start[k] = d.R;
    if constexpr (HIER) {
        for (uint32_t g = tid; g < d.lut_size; g += blockDim.x) {
            const uint64_t v = (uint64_t)g << d.lut_shift;
            uint32_t r = 0;
            while (r + 1 < nr && v >= d.reg_start[r + 1]) ++r;
            s_lut[g] = (uint8_t)r;
        }
    }
    __syncthreads();

    const uint32_t lane = tid & 63;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(tid >> 6);
    uint32_t *sig = reinterpret_cast<uint32_t *>(smem + L.sigs + L.sig_stride * wib);
    const uint64_t n_sets = desc[0];
    const uint64_t n_items = prefix[n_sets];
    uint32_t err = 0;
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
        for (uint64_t base = lo; base < hi; base += 64 * kUnroll) {
            uint32_t x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t j = base + lane + 64u * u;
                x[u] = ids[j < hi ? j : hi - 1];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint64_t j = base + lane + 64u * u;
                if (j >= hi) continue;
                if ((uint64_t)x[u] >= d.universe) { err |= kErrRange; continue; }
                const uint64_t v = permute<HASH>(x[u], d);
                if constexpr (HASH == HOPH_HASH_TABLE) {
                    if (v >= d.R) { err |= kErrRange; continue; }
                }
                uint32_t b;
                uint64_t start;
                locate(v, s_lut, d.lut_shift, s_reg, HIER ? nr : 1u, nb, s_start, b, start);
                atomicMin(&sig[b], (uint32_t)(v - start));
            }
        }
        wave_lds_fence();
        uint32_t *out = sigs + set * k;
        for (uint32_t b = lane; b < k; b += 64) {
            const uint32_t v = sig[b];
            if (v != HOPH_EMPTY) atomicMin(&out[b], v);
        }
        wave_lds_fence();
    }
    if (err) atomicOr(err_flag, err);
}

template <uint32_t HASH, bool HIER>
hipError_t launch_t(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets, uint64_t n_sets,
                    uint32_t *sigs, uint32_t *err_flag, hipStream_t st, uint32_t threads, size_t lds,
                    uint32_t grid) {
    auto kern = sketch_kernel<HASH, HIER>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, d, ids, offsets, n_sets, sigs, err_flag);
    return hipGetLastError();
}

template <uint32_t HASH, bool HIER>
hipError_t launch_chunked_t(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets, const uint64_t *desc,
                            const uint64_t *prefix, uint32_t chunk, uint64_t max_ids, uint32_t *sigs,
                            uint32_t *err_flag, hipStream_t st, uint32_t threads, size_t lds, uint32_t grid) {
    auto kern = sketch_chunked_kernel<HASH, HIER>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, st, d, ids, offsets, desc, prefix, chunk, max_ids, sigs,
                       err_flag);
    return hipGetLastError();
}

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
    const bool hier = d.n_regions > 1;
    uint32_t waves = 4;
    while (waves > 1 && sketch_lds(d.k, d.n_regions, d.lut_size, waves).total > 48 * 1024) waves >>= 1;
    const size_t lds = sketch_lds(d.k, d.n_regions, d.lut_size, waves).total;
    const uint32_t grid = (uint32_t)((uint64_t)device_cu_count() * (waves_per_cu ? waves_per_cu : 16) / waves);
    const uint32_t threads = 64 * waves;
#define HOPH_SKC(H, HI) \
    launch_chunked_t<H, HI>(d, ids, offsets, desc, prefix, chunk, max_ids, sigs, err_flag, st, threads, lds, grid)
    switch (d.hash) {
    case HOPH_HASH_TABLE: return hier ? HOPH_SKC(HOPH_HASH_TABLE, true) : HOPH_SKC(HOPH_HASH_TABLE, false);
    case HOPH_HASH_MODP31: return hier ? HOPH_SKC(HOPH_HASH_MODP31, true) : HOPH_SKC(HOPH_HASH_MODP31, false);
    default: return hier ? HOPH_SKC(HOPH_HASH_MODP32P15, true) : HOPH_SKC(HOPH_HASH_MODP32P15, false);
    }
#undef HOPH_SKC
}

hipError_t launch_sketch(const SketchDesc &d, const uint32_t *ids, const uint64_t *offsets, uint64_t n_sets,
                         uint32_t *sigs, uint32_t *err_flag, hipStream_t st) {
    if (n_sets == 0) return hipSuccess;
    const bool hier = d.n_regions > 1;
    // four wavefronts per workgroup unless the signatures are large
    uint32_t waves = 4;
    while (waves > 1 && sketch_lds(d.k, d.n_regions, d.lut_size, waves).total > 48 * 1024) waves >>= 1;
    const size_t lds = sketch_lds(d.k, d.n_regions, d.lut_size, waves).total;
    const uint64_t want_waves = (uint64_t)device_cu_count() * 32;
    uint64_t grid = (n_sets + waves - 1) / waves;
    if (grid > want_waves / waves) grid = want_waves / waves;
    if (grid == 0) grid = 1;
    const uint32_t threads = 64 * waves;
    switch (d.hash) {
    case HOPH_HASH_TABLE:
        return hier ? launch_t<HOPH_HASH_TABLE, true>(d, ids, offsets, n_sets, sigs, err_flag, st, threads, lds, grid)
                    : launch_t<HOPH_HASH_TABLE, false>(d, ids, offsets, n_sets, sigs, err_flag, st, threads, lds, grid);
    case HOPH_HASH_MODP31:
        return hier ? launch_t<HOPH_HASH_MODP31, true>(d, ids, offsets, n_sets, sigs, err_flag, st, threads, lds, grid)
                    : launch_t<HOPH_HASH_MODP31, false>(d, ids, offsets, n_sets, sigs, err_flag, st, threads, lds, grid);
    default:
        return hier ? launch_t<HOPH_HASH_MODP32P15, true>(d, ids, offsets, n_sets, sigs, err_flag, st, threads, lds, grid)
                    : launch_t<HOPH_HASH_MODP32P15, false>(d, ids, offsets, n_sets, sigs, err_flag, st, threads, lds,
                                                           grid);
    }
}

}  // namespace hoph
