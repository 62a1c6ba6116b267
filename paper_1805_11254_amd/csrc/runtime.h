// Runtime internals shared by the C ABI translation units of libhoph
// (api.cpp, plan.cpp, server.cpp): the index object, the per-query workspace
// and error helpers.  Not part of the C ABI.
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include "hoph_internal.h"

namespace hoph {

uint32_t max_depth_for_kpad(uint32_t kpad);
uint64_t sort_capacity(uint64_t n);

// Record msg as the calling thread's last error and return st.
constexpr int kMaxDevices = 64;           // device ordinals the library keeps per-device state for
hoph_status fail(hoph_status st, const std::string &msg);
hoph_status hip_fail(hipError_t e, const char *what);
void clear_error();

#define HOPH_HIP(call, what)                      \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// The device error word of the current device (allocated on first use).
hoph_status device_err_word(uint32_t **out);

// Device buffers for one query at a time: survivors, accepted keys, counters.
// A fixed workspace is a view of memory someone else owns (the library's
// static scratch): its grow_* calls never allocate and report
// HOPH_E_CAPACITY when a request exceeds what the view holds, and it has no
// events (no timing).
struct Workspace {
    bool fixed = false;
    Survivor *surv = nullptr;
    uint64_t surv_cap = 0;
    uint64_t *keys = nullptr;
    uint64_t keys_cap = 0;        // a power of two >= 4096
    uint64_t *counters = nullptr; // device [0] survivors, [1] accepted
    uint64_t *qmasks = nullptr;   // per (query, group) empty-bin masks
    uint64_t qmask_cap = 0;
    uint32_t *qcodes = nullptr;   // per (query, code group) code planes
    uint64_t qcode_cap = 0;
    uint32_t *qcount = nullptr;   // per-query accepted counts (output stage)
    uint64_t *cursor = nullptr;   // per-query scatter cursors
    uint64_t seg_cap = 0;
    uint64_t *h_counters = nullptr; // pinned host mirror
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t aev[3] = {nullptr, nullptr, nullptr};   // around the last append of sets
    bool aev_recorded = false;
    float last_ms[3] = {0, 0, 0};
    uint64_t last_counts[2] = {0, 0};   // survivors of the coarse pass, accepted pairs
    uint32_t last_nq = 0;                // queries of that batch
    uint32_t last_plan[4] = {0, 0, 0, 0};   // the coarse pass's shape (hoph_coarse_plan)
    void release() {
        if (fixed) return;                 // a view: nothing of its own to free
        for (auto &e : ev)
            if (e) { (void)hipEventDestroy(e); e = nullptr; }
        for (auto &e : aev)
            if (e) { (void)hipEventDestroy(e); e = nullptr; }
        aev_recorded = false;
        if (surv) (void)hipFree(surv);
        if (keys) (void)hipFree(keys);
        if (counters) (void)hipFree(counters);
        if (qmasks) (void)hipFree(qmasks);
        if (qcodes) (void)hipFree(qcodes);
        if (qcount) (void)hipFree(qcount);
        if (cursor) (void)hipFree(cursor);
        if (h_counters) (void)hipHostFree(h_counters);
        qmasks = nullptr;
        qmask_cap = 0;
        qcodes = nullptr;
        qcode_cap = 0;
        qcount = nullptr;
        cursor = nullptr;
        seg_cap = 0;
        surv = nullptr;
        keys = nullptr;
        counters = nullptr;
        h_counters = nullptr;
        surv_cap = keys_cap = 0;
    }
    hoph_status init(uint64_t surv_records, uint64_t keys_records) {
        HOPH_HIP(hipMalloc(&counters, 64), "hipMalloc(counters)");
        HOPH_HIP(hipHostMalloc(&h_counters, 64, hipHostMallocDefault), "hipHostMalloc(counters)");
        for (auto &e : ev) HOPH_HIP(hipEventCreate(&e), "hipEventCreate");
        for (auto &e : aev) HOPH_HIP(hipEventCreate(&e), "hipEventCreate");
        hoph_status st = grow_surv(surv_records);
        if (st) return st;
        return grow_keys(keys_records);
    }
    hoph_status grow_surv(uint64_t n) {
        if (n <= surv_cap) return HOPH_OK;
        if (fixed) return fail(HOPH_E_CAPACITY, "survivor records exceed the fixed scratch");
        if (surv) (void)hipFree(surv);
        surv = nullptr;
        surv_cap = 0;
        if (hipMalloc(&surv, n * sizeof(Survivor)) != hipSuccess) return fail(HOPH_E_NOMEM, "survivor buffer");
        surv_cap = n;
        return HOPH_OK;
    }
    hoph_status grow_qmasks(uint64_t n) {
        if (n <= qmask_cap) return HOPH_OK;
        if (fixed) return fail(HOPH_E_CAPACITY, "query masks exceed the fixed scratch");
        if (qmasks) (void)hipFree(qmasks);
        qmasks = nullptr;
        qmask_cap = 0;
        uint64_t want = 4096;
        while (want < n) want <<= 1;
        if (hipMalloc(&qmasks, want * sizeof(uint64_t)) != hipSuccess) return fail(HOPH_E_NOMEM, "query mask buffer");
        qmask_cap = want;
        return HOPH_OK;
    }
    hoph_status grow_qcodes(uint64_t n) {
        if (n <= qcode_cap) return HOPH_OK;
        if (fixed) return fail(HOPH_E_CAPACITY, "query code records exceed the fixed scratch");
        if (qcodes) (void)hipFree(qcodes);
        qcodes = nullptr;
        qcode_cap = 0;
        uint64_t want = 1 << 16;
        while (want < n) want <<= 1;
        if (hipMalloc(&qcodes, want * sizeof(uint32_t)) != hipSuccess) return fail(HOPH_E_NOMEM, "query code buffer");
        qcode_cap = want;
        return HOPH_OK;
    }
    hoph_status grow_seg(uint64_t n) {
        if (n <= seg_cap) return HOPH_OK;
        if (fixed) return fail(HOPH_E_CAPACITY, "per-query output counters exceed the fixed scratch");
        if (qcount) (void)hipFree(qcount);
        if (cursor) (void)hipFree(cursor);
        qcount = nullptr;
        cursor = nullptr;
        seg_cap = 0;
        uint64_t want = 1024;
        while (want < n) want <<= 1;
        if (hipMalloc(&qcount, want * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&cursor, want * sizeof(uint64_t)) != hipSuccess)
            return fail(HOPH_E_NOMEM, "output stage buffers");
        seg_cap = want;
        return HOPH_OK;
    }
    hoph_status grow_keys(uint64_t n) {
        const uint64_t want = sort_capacity(n);
        if (want <= keys_cap) return HOPH_OK;
        if (fixed)
            return fail(HOPH_E_CAPACITY, std::to_string(n) + " accepted pairs exceed the fixed scratch's " +
                                             std::to_string(keys_cap) + " keys");
        if (keys) (void)hipFree(keys);
        keys = nullptr;
        keys_cap = 0;
        if (hipMalloc(&keys, want * sizeof(uint64_t)) != hipSuccess) return fail(HOPH_E_NOMEM, "key buffer");
        keys_cap = want;
        return HOPH_OK;
    }
};

inline uint32_t round4(uint32_t x) { return (x + 3u) & ~3u; }

bool valid_ratio_T(hoph_ratio T);
bool valid_ratio_eps(hoph_ratio e);
hoph_status check_results(const hoph_results *r, uint32_t n_q);

enum class QueryKind { GOPH, HOPH, OPH_FULL };

// Queries per wavefront so that a pass has enough (tile group, query chunk) items
// to fill the device; tiles_per_wave as coarse_tiles_per_wave reports.
uint32_t pick_q_per_wave(uint64_t n_sets, uint32_t n_q, uint32_t tiles_per_wave, bool tri = false);
hoph_status copy_counters(Workspace &ws, hipStream_t st);
hoph_status write_output(Workspace &ws, uint64_t accepted, uint32_t n_q, hoph_results *res, hipStream_t s);

}  // namespace hoph

namespace hoph {
// Decision tables of one (T, eps, empty policy, weights) for an index's layout.
struct TabEntry {
    hoph_ratio T{}, eps{};
    uint32_t policy = 0, goph = 0;
    ScanTab tab{};
    // phase-1 keep rates of the first-group pass sampled from the index rows
    // (sample_keep_rates), and the index size they were sampled at (0: none)
    double keep_rate[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t keep_n = 0;
};
constexpr size_t kTabCache = 16;
}  // namespace hoph

struct hoph_index {
    int device = 0;
    hoph_sketch_params params{};
    hoph::LayoutInfo lay;
    uint32_t kpad = 0;
    uint64_t n = 0;
    uint64_t capacity = 0;        // slab capacity in sets, a multiple of 64
    uint64_t max_sets = 0;        // the capacity the caller asked for
    uint32_t *slab = nullptr;
    uint32_t *codes = nullptr;    // code planes of the first cg groups (coarse pass on codes)
    uint32_t cg = 0;
    hoph::Workspace ws;
    // the exact tables of the last kTabCache query parameter sets (reserved at
    // build, replaced oldest first), so that a repeated query does not rebuild
    // them on the host (about 30 us at k' = 32)
    std::vector<hoph::TabEntry> tabs;
    size_t tab_next = 0;
    std::mutex mu;
};

namespace hoph {
// Sketch n_sets sets straight into index rows [first, first + n_sets) (slabs and
// code planes), asynchronously on s; the caller checks capacity and owns idx->n.
hipError_t append_sets_async(hoph_index *idx, const uint32_t *d_ids, const uint64_t *d_offsets, uint64_t n_sets,
                             uint64_t first, uint32_t *err_word, hipStream_t s, bool timed);
// GOPH / HOPH / plain-OPH query through the index's own workspace (host-synchronised),
// against the index rows below min(index size, n_limit): a batch that a plan
// dispatched against a snapshot of the size and then redoes here keeps it.
hoph_status run_query(const hoph_index *cidx, const uint32_t *d_qsigs, uint32_t n_q, const hoph_query_params *qp,
                      hoph_results *res, void *stream, QueryKind kind, bool self_join = false,
                      uint64_t n_limit = ~0ull);
// The same with a caller-supplied workspace (a fixed view: nothing is allocated).
hoph_status run_query_in(const hoph_index *cidx, Workspace &ws, const uint32_t *d_qsigs, uint32_t n_q,
                         const hoph_query_params *qp, hoph_results *res, void *stream, QueryKind kind);
// The coarse pass alone, reps launches back to back between two events (hoph_scan_timing).
hoph_status scan_timing(const hoph_index *cidx, const uint32_t *d_qsigs, uint32_t n_q, const hoph_query_params *qp,
                        uint32_t reps, void *d_flush, uint64_t flush_bytes, float *ms, void *stream);
// The scan tables for qp on idx's layout, from the index's cache (caller holds idx->mu).
hoph_status cached_scan_tab(hoph_index *idx, const hoph_query_params &qp, bool goph, ScanTab &out,
                            TabEntry **entry = nullptr);
// The results of a plan's last batch copied to host buffers with one stream
// synchronisation in the usual case: the counters, the CSR offsets (n_q + 1)
// and the first `pre` ids are read together; more ids are read only when the
// batch returned more than `pre`, or when it took the host-synchronised
// fallback.  h_ids holds the plan's max_results ids; pre <= max_results.
hoph_status plan_results_to_host(hoph_plan *p, uint64_t *h_offsets, uint32_t *h_ids, uint64_t pre,
                                 uint64_t *n_results, hipStream_t st);
// Survivor records a plan holds: the index capacity (at least 2^20) per 1,024
// queries of its batch capacity.
uint64_t plan_survivor_capacity(uint64_t index_capacity, uint32_t max_queries);
// Takes the tile shapes another plan tuned (from may be null: keep the
// defaults) and captures this plan's graph now (if it uses one), so that its
// first batch starts without tuning or capture.
hoph_status plan_adopt_and_capture(hoph_plan *p, const hoph_plan *from);
}  // namespace hoph
