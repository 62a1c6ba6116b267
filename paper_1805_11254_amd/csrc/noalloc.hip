// query_hoph_noalloc: query_hoph (Alg. 2 over a resident index) for callers
// that cannot allocate.  Every buffer the query path needs beyond its inputs
// and outputs (counters, per-query empty masks and code records, survivors,
// accepted keys, output-stage counts and cursors) lives in one file-scope
// device array of kScratchBytes, which each device holds from the library's
// load until the process ends.  The host side reaches that array only through
// the address hipGetSymbolAddress gives for the current device; the array's
// own name is never passed to a kernel or a copy.
#include <mutex>

#include "runtime.h"

namespace hoph {
namespace {

constexpr uint64_t kScratchBytes = 64ull << 20;       // 64 MiB per device
constexpr uint32_t kNoallocMaxQueries = 4096;

// Regions of the scratch array (byte offsets; each a multiple of 256).
constexpr uint64_t kOffCounters = 0;                  // 8 x u64
constexpr uint64_t kOffQmasks = 256;                  // u64 per (query, group)
constexpr uint64_t kQmaskWords = 4096ull * 64;        // 2 MiB
constexpr uint64_t kOffQcodes = kOffQmasks + kQmaskWords * 8;
constexpr uint64_t kQcodeWords = 5ull << 18;          // 5 MiB of u32 query code records
constexpr uint64_t kOffQcount = kOffQcodes + kQcodeWords * 4;
constexpr uint64_t kSegEntries = 8192;                // >= kNoallocMaxQueries + 1
constexpr uint64_t kOffCursor = kOffQcount + kSegEntries * 4;
constexpr uint64_t kOffKeys = kOffCursor + kSegEntries * 8;
constexpr uint64_t kKeyWords = 1ull << 20;            // accepted pairs of one call (a power of two)
constexpr uint64_t kOffSurv = kOffKeys + kKeyWords * 8;
constexpr uint64_t kSurvRecords = (kScratchBytes - kOffSurv) / sizeof(Survivor);
static_assert(kOffQcodes % 256 == 0 && kOffQcount % 256 == 0 && kOffCursor % 256 == 0 && kOffKeys % 256 == 0 &&
                  kOffSurv % 256 == 0,
              "scratch regions must stay 256-byte aligned");
static_assert(kSurvRecords >= (1u << 20), "survivor region too small");

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Per device: the array's device address (set up once, with that device
// current), a host mirror of the counters, and a lock that serialises calls
// on the device (each call ends with a stream synchronisation, so a call
// holding the lock has finished with the array when it releases it).
std::mutex g_setup_mu;
uint8_t *g_scratch[kMaxDevices] = {};
alignas(64) uint64_t g_host_counters[kMaxDevices][8];
std::mutex g_call_mu[kMaxDevices];

hoph_status scratch_address(int dev, uint8_t **out) {
    std::lock_guard<std::mutex> lk(g_setup_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(HOPH_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch[dev];
    return HOPH_OK;
}

}  // namespace
}  // namespace hoph

using namespace hoph;

extern "C" hoph_status query_hoph_noalloc(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                                          const hoph_query_params *qp, hoph_results *results, void *hip_stream) {
    clear_error();
    if (!index) return fail(HOPH_E_INVAL, "index is NULL");
    if (n_q > kNoallocMaxQueries)
        return fail(HOPH_E_CAPACITY, "query_hoph_noalloc takes at most " + std::to_string(kNoallocMaxQueries) +
                                         " queries per call (" + std::to_string(n_q) + " given)");
    const int dev = index->device;
    if (dev < 0 || dev >= kMaxDevices) return fail(HOPH_E_DEVICE, "device ordinal out of range");
    DeviceGuard dg(dev);
    if (!dg.ok) return fail(HOPH_E_DEVICE, "cannot select the index device");
    uint8_t *base = nullptr;
    hoph_status st = scratch_address(dev, &base);
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_call_mu[dev]);
    Workspace ws;
    ws.fixed = true;
    ws.counters = reinterpret_cast<uint64_t *>(base + kOffCounters);
    ws.h_counters = g_host_counters[dev];
    ws.qmasks = reinterpret_cast<uint64_t *>(base + kOffQmasks);
    ws.qmask_cap = kQmaskWords;
    ws.qcodes = reinterpret_cast<uint32_t *>(base + kOffQcodes);
    ws.qcode_cap = kQcodeWords;
    ws.qcount = reinterpret_cast<uint32_t *>(base + kOffQcount);
    ws.cursor = reinterpret_cast<uint64_t *>(base + kOffCursor);
    ws.seg_cap = kSegEntries;
    ws.keys = reinterpret_cast<uint64_t *>(base + kOffKeys);
    ws.keys_cap = kKeyWords;
    ws.surv = reinterpret_cast<Survivor *>(base + kOffSurv);
    ws.surv_cap = kSurvRecords;
    return run_query_in(index, ws, d_qsigs, n_q, qp, results, hip_stream, QueryKind::HOPH);
}
