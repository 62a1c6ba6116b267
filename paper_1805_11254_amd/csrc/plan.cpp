// Batched execution (hoph_plan_*): a fixed-capacity pipeline whose kernels
// read the batch size from a device descriptor, so that one captured hipGraph
// replays every batch; tile shapes come from timing candidates on the first
// batch (cached per shape class, optionally in the file named by
// HOPH_TUNE_CACHE).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.h"

namespace hoph {

namespace {

struct PlanShape {
    uint32_t q_per_wave = 16, coarse_wpc = 16, chunk = 1024, sketch_wpc = 16;
};

// Tuning results of this process, keyed by shape class.
std::mutex g_tune_mu;
std::map<std::string, std::pair<PlanShape, float>> g_tune;
bool g_tune_loaded = false;

void load_tune_cache() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("HOPH_TUNE_CACHE");
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream is(line);
        std::string key;
        PlanShape s;
        float ms = 0;
        if (is >> key >> s.q_per_wave >> s.coarse_wpc >> s.chunk >> s.sketch_wpc >> ms) g_tune[key] = {s, ms};
    }
}

void store_tune_cache(const std::string &key, const PlanShape &s, float ms) {
    g_tune[key] = {s, ms};
    const char *path = std::getenv("HOPH_TUNE_CACHE");
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << s.q_per_wave << " " << s.coarse_wpc << " " << s.chunk << " " << s.sketch_wpc << " " << ms
        << "\n";
}

uint32_t log2_bucket(uint64_t x) {
    uint32_t b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

}  // namespace

}  // namespace hoph

using namespace hoph;

struct hoph_plan {
    hoph_index *idx = nullptr;
    hoph_sketch_params params{};
    hoph_query_params qp{};
    hoph_plan_config cfg{};
    QueryKind kind = QueryKind::HOPH;
    SketchDesc sd{};
    ScanTab tab{};
    uint32_t depth = 1;
    // device buffers
    uint32_t *q_ids = nullptr;
    uint64_t *q_offsets = nullptr, *desc = nullptr, *prefix = nullptr, *q_masks = nullptr;
    uint32_t *q_sigs = nullptr, *q_codes = nullptr;
    bool codes = false;           // coarse pass on code planes
    Survivor *surv = nullptr;
    uint64_t surv_cap = 0;
    uint64_t *keys = nullptr;
    uint64_t keys_cap = 0;
    uint64_t *counters = nullptr, *cursor = nullptr, *out_offsets = nullptr;
    uint32_t *qcount = nullptr, *out_ids = nullptr;
    uint64_t *h_counters = nullptr;
    uint32_t *err_word = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // state
    PlanShape shape;
    bool tuned = false;
    float tune_ms = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t last_nq = 0;
    uint64_t last_nsets = 0;      // index size the last batch was dispatched against
    bool pending = false;
    uint32_t fallbacks = 0;
    uint32_t fallback_causes = 0;  // hoph_plan_info.fallback_causes
    std::mutex mu;

    // the causes of a batch that must be redone, from its device counters
    void note_fallback(uint64_t surv, uint64_t acc, uint64_t flags) {
        ++fallbacks;
        fallback_causes |= (surv > surv_cap ? 1u : 0u) | (acc > keys_cap ? 2u : 0u) | ((flags & 3ull) ? 4u : 0u);
    }

    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        void *bufs[] = {q_ids, q_offsets, desc, prefix, q_masks, q_sigs, q_codes, surv, keys, counters, cursor,
                        out_offsets, qcount, out_ids};
        for (void *p : bufs)
            if (p) (void)hipFree(p);
        if (h_counters) (void)hipHostFree(h_counters);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace hoph {
namespace {

std::string shape_key(const hoph_plan *p, uint64_t n_sets, uint32_t n_q) {
    std::ostringstream os;
    os << "k" << p->params.k << "_kp" << p->params.k_group << "_lay" << p->params.layout << "_hash" << p->params.hash
       << "_d" << p->depth << (p->codes ? "c" : "w") << "_kind" << (p->kind == QueryKind::GOPH ? 0 : 1) << "_n"
       << log2_bucket(n_sets) << "_q"
       << log2_bucket(n_q);
    return os.str();
}

ScanLaunch scan_launch(const hoph_plan *p, const PlanShape &s) {
    const hoph_index *idx = p->idx;
    ScanLaunch l{};
    l.slab = idx->slab;
    l.capacity = idx->capacity;
    l.n_sets = 0;                      // from desc
    l.kpad = idx->kpad;
    l.kp = idx->lay.kp;
    l.L = idx->lay.L;
    l.k = idx->lay.k;
    l.qsigs = p->q_sigs;
    l.qmasks = p->q_masks;
    l.codes = p->codes ? idx->codes : nullptr;
    l.qcodes = p->q_codes;
    l.cg = idx->cg;
    l.q0 = 0;
    l.q1 = p->cfg.max_queries;
    l.depth = p->depth;
    l.q_per_wave = s.q_per_wave;
    l.surv = p->surv;
    l.surv_cap = p->surv_cap;
    l.keys = p->keys;
    l.keys_cap = p->keys_cap;
    l.counters = p->counters;
    l.desc = p->desc;
    l.waves_per_cu = s.coarse_wpc;
    return l;
}

hoph_status enqueue_sketch(hoph_plan *p, const PlanShape &s, hipStream_t st) {
    HOPH_HIP(launch_sketch_chunked(p->sd, p->q_ids, p->q_offsets, p->desc, p->prefix, s.chunk, p->cfg.max_queries,
                                   p->cfg.max_query_ids, p->q_sigs, p->err_word, s.sketch_wpc, st),
             "batch sketch launch");
    const LayoutInfo &lay = p->idx->lay;
    CodeThr thr{};
    std::memcpy(thr.dthr, p->tab.dthr0, sizeof(thr.dthr));
    LinTab lin;
    const bool with_lin = p->codes && lin_records(scan_launch(p, s), p->tab, &lin);
    HOPH_HIP(launch_query_masks(p->q_sigs, p->cfg.max_queries, p->desc, lay.k, lay.kp, lay.L, p->q_masks,
                                p->codes ? p->q_codes : nullptr, p->idx->cg, &thr, st, with_lin ? &lin : nullptr,
                                p->counters, 4),
             "query mask launch");
    return HOPH_OK;
}

// fill: zero the counters first (the sketch stage's record launch already
// zeroes them in the pipeline; the tuner runs passes on their own)
hoph_status enqueue_scan(hoph_plan *p, const PlanShape &s, hipStream_t st, bool with_fine, bool fill) {
    if (fill) HOPH_HIP(launch_fill_u64(p->counters, 4, 0, st), "fill counters");
    const ScanLaunch l = scan_launch(p, s);
    HOPH_HIP(launch_scan_coarse(l, p->tab, st), "coarse scan launch");
    if (with_fine) HOPH_HIP(launch_scan_fine(l, p->tab, st), "fine scan launch");
    return HOPH_OK;
}

// The general output stage (counts, scan, scatter, per-query sort).
hoph_status enqueue_general_output(hoph_plan *p, hipStream_t st) {
    HOPH_HIP(launch_segmented_output(p->keys, p->counters, p->keys_cap, p->qcount, p->desc, p->cfg.max_queries,
                                     p->out_offsets, p->cursor, p->out_ids, p->cfg.max_results, p->counters,
                                     p->cfg.max_queries, p->keys_cap, kSegMaxPlan, st),
             "output launch");
    return HOPH_OK;
}

// Plans of up to kSmallOutQueries queries end with the one-workgroup output
// stage; a batch that accepted more pairs than it sorts leaves counters[3] = 4
// and gets the general stage when its results are read (finish_output).
hoph_status enqueue_output(hoph_plan *p, hipStream_t st) {
    if (p->cfg.max_queries > kSmallOutQueries) return enqueue_general_output(p, st);
    HOPH_HIP(launch_small_output(p->keys, p->counters, p->keys_cap, p->desc, p->cfg.max_queries, p->out_offsets,
                                 p->out_ids, p->cfg.max_results, st),
             "output launch");
    return HOPH_OK;
}

// After the counters of a batch were read into h_counters: when the
// one-workgroup stage left the output to the general stage and nothing
// overflowed, run it and read counters[2..3] again (synchronises st); true
// when it ran.
hoph_status finish_output(hoph_plan *p, hipStream_t st, bool &ran) {
    ran = false;
    const uint64_t surv = p->h_counters[0], acc = p->h_counters[1];
    if (!(p->h_counters[3] & 4ull) || surv > p->surv_cap || acc > p->keys_cap) return HOPH_OK;
    hoph_status r = enqueue_general_output(p, st);
    if (r) return r;
    HOPH_HIP(hipMemcpyAsync(p->h_counters + 2, p->counters + 2, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, st),
             "read counters");
    HOPH_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    ran = true;
    return HOPH_OK;
}

hoph_status enqueue_pipeline(hoph_plan *p, const PlanShape &s, hipStream_t st) {
    hoph_status r = enqueue_sketch(p, s, st);
    if (r) return r;
    r = enqueue_scan(p, s, st, true, false);
    if (r) return r;
    return enqueue_output(p, st);
}

// Time candidate shapes on the batch already staged in the plan (descriptor set).
hoph_status tune(hoph_plan *p, hipStream_t st, uint64_t n_sets, uint32_t n_q) {
    const std::string key = shape_key(p, n_sets, n_q);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_cache();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            p->shape = it->second.first;
            p->tune_ms = it->second.second;
            p->tuned = true;
            return HOPH_OK;
        }
    }
    auto time_it = [&](auto &&enqueue) -> float {
        float best = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {           // first run warms caches and code objects
            if (hipEventRecord(p->ev[0], st) != hipSuccess) return 1e30f;
            if (enqueue() != HOPH_OK) return 1e30f;
            if (hipEventRecord(p->ev[1], st) != hipSuccess) return 1e30f;
            if (hipEventSynchronize(p->ev[1]) != hipSuccess) return 1e30f;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, p->ev[0], p->ev[1]);
            if (rep) best = std::min(best, ms);
        }
        return best;
    };
    PlanShape best = p->shape;
    float sk_best = 1e30f;
    for (uint32_t chunk : {256u, 1024u, 4096u}) {
        for (uint32_t wpc : {16u, 32u}) {
            PlanShape s = best;
            s.chunk = chunk;
            s.sketch_wpc = wpc;
            const float ms = time_it([&] { return enqueue_sketch(p, s, st); });
            if (ms < sk_best) {
                sk_best = ms;
                best.chunk = chunk;
                best.sketch_wpc = wpc;
            }
        }
    }
    hoph_status r = enqueue_sketch(p, best, st);      // signatures for the scan candidates
    if (r) return r;
    float sc_best = 1e30f;
    for (uint32_t qpw : {4u, 8u, 16u, 32u, 64u, 128u, 256u}) {
        for (uint32_t wpc : {8u, 16u, 32u}) {
            PlanShape s = best;
            s.q_per_wave = qpw;
            s.coarse_wpc = wpc;
            const float ms = time_it([&] { return enqueue_scan(p, s, st, false, true); });
            if (ms < sc_best) {
                sc_best = ms;
                best.q_per_wave = qpw;
                best.coarse_wpc = wpc;
            }
        }
    }
    p->shape = best;
    p->tune_ms = sk_best + sc_best;
    p->tuned = true;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    store_tune_cache(key, best, p->tune_ms);
    return HOPH_OK;
}

hoph_status capture(hoph_plan *p) {
    hipStream_t cs = nullptr;
    HOPH_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate(capture)");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    hoph_status r = enqueue_pipeline(p, p->shape, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    p->graph = g;
    p->exec = x;
    return HOPH_OK;
}

template <typename T>
hoph_status dalloc(T **p, uint64_t n, const char *what) {
    if (hipMalloc(reinterpret_cast<void **>(p), std::max<uint64_t>(n, 1) * sizeof(T)) != hipSuccess)
        return fail(HOPH_E_NOMEM, what);
    return HOPH_OK;
}

}  // namespace
}  // namespace hoph

extern "C" {

hoph_status hoph_plan_create(hoph_index *idx, const hoph_sketch_params *params, const hoph_query_params *qp,
                             const hoph_plan_config *cfg, hoph_plan **out) {
    clear_error();
    if (!idx || !params || !qp || !cfg || !out) return fail(HOPH_E_INVAL, "NULL argument");
    *out = nullptr;
    if (cfg->kind > 1) return fail(HOPH_E_INVAL, "kind must be 0 (GOPH) or 1 (HOPH)");
    if (cfg->max_queries == 0 || cfg->max_query_ids == 0) return fail(HOPH_E_INVAL, "empty plan capacities");
    if (cfg->kind == 0 && idx->params.layout != HOPH_LAYOUT_OPH) return fail(HOPH_E_INVAL, "GOPH needs an OPH index");
    if (cfg->kind == 1 && idx->params.layout != HOPH_LAYOUT_HIER) return fail(HOPH_E_INVAL, "HOPH needs a HIER index");
    if (params->layout != idx->params.layout || params->k != idx->params.k ||
        params->k_group != idx->params.k_group || params->hash != idx->params.hash ||
        params->universe != idx->params.universe || params->hash_a != idx->params.hash_a ||
        params->hash_b != idx->params.hash_b || params->ratio_a != idx->params.ratio_a ||
        params->ratio_b != idx->params.ratio_b)
        return fail(HOPH_E_INVAL, "sketch parameters differ from the index's");
    if (!valid_ratio_T(qp->T) || !valid_ratio_eps(qp->eps)) return fail(HOPH_E_INVAL, "T or eps out of range");
    if (qp->empty_policy > HOPH_EMPTY_EITHER) return fail(HOPH_E_INVAL, "unknown empty policy");
    if (qp->coarse_filter > HOPH_COARSE_WORDS) return fail(HOPH_E_INVAL, "unknown coarse filter");
    std::unique_ptr<hoph_plan> p(new (std::nothrow) hoph_plan());
    if (!p) return fail(HOPH_E_NOMEM, "host allocation");
    p->idx = idx;
    p->params = *params;
    p->qp = *qp;
    p->cfg = *cfg;
    p->kind = cfg->kind == 0 ? QueryKind::GOPH : QueryKind::HOPH;
    DeviceGuard dg(idx->device);
    fill_sketch_desc(*params, idx->lay, p->sd);
    hoph_decision_tables t;
    std::string err;
    hoph_status st = build_tables(idx->lay, *qp, cfg->kind == 0, t, err);
    if (st) return fail(st, err);
    to_scan_tab(t, p->tab);
    p->codes = qp->coarse_filter == HOPH_COARSE_CODES && idx->codes;
    const uint32_t maxd = p->codes ? idx->cg : std::min(max_depth_for_kpad(idx->kpad), idx->lay.L);
    p->depth = default_coarse_depth(p->tab, qp->coarse_depth, maxd, p->codes ? code_pack(idx->lay.kp, idx->lay.L) : 1u);
    const uint64_t Q = cfg->max_queries, k = params->k, L = idx->lay.L;
    p->surv_cap = plan_survivor_capacity(idx->capacity, cfg->max_queries);
    p->keys_cap = sort_capacity(std::max<uint64_t>(cfg->max_results, 1));
    auto cleanup = [&](hoph_status s) {
        p->release();
        return s;
    };
    if ((st = dalloc(&p->q_ids, cfg->max_query_ids, "plan query ids")) ||
        (st = dalloc(&p->q_offsets, Q + 1, "plan query offsets")) || (st = dalloc(&p->desc, 2, "plan descriptor")) ||
        (st = dalloc(&p->prefix, Q + 1, "plan chunk prefix")) || (st = dalloc(&p->q_sigs, Q * k, "plan signatures")) ||
        (st = dalloc(&p->q_masks, Q * L, "plan query masks")) ||
        (st = dalloc(&p->q_codes, (Q + 1) * idx->cg * code_rec_words(idx->lay.kp), "plan query codes")) ||
        (st = dalloc(&p->surv, p->surv_cap, "plan survivors")) ||
        (st = dalloc(&p->keys, p->keys_cap, "plan keys")) || (st = dalloc(&p->counters, 8, "plan counters")) ||
        (st = dalloc(&p->cursor, Q + 1, "plan cursors")) || (st = dalloc(&p->out_offsets, Q + 1, "plan offsets")) ||
        (st = dalloc(&p->qcount, Q + 1, "plan counts")) ||
        (st = dalloc(&p->out_ids, std::max<uint64_t>(cfg->max_results, 1), "plan results")))
        return cleanup(st);
    if (hipHostMalloc(&p->h_counters, 64, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(HOPH_E_NOMEM, "pinned counters"));
    for (auto &e : p->ev)
        if (hipEventCreate(&e) != hipSuccess) return cleanup(fail(HOPH_E_DEVICE, "hipEventCreate"));
    if ((st = device_err_word(&p->err_word))) return cleanup(st);
    *out = p.release();
    return HOPH_OK;
}

hoph_status hoph_plan_run(hoph_plan *p, const uint32_t *d_ids, const uint64_t *d_offsets, uint32_t n_q, uint64_t n_ids,
                          void *hip_stream) {
    clear_error();
    if (!p) return fail(HOPH_E_INVAL, "plan is NULL");
    if (n_q > p->cfg.max_queries || n_ids > p->cfg.max_query_ids)
        return fail(HOPH_E_CAPACITY, "batch larger than the plan (queries or ids)");
    if ((n_ids && !d_ids) || !d_offsets) return fail(HOPH_E_INVAL, "NULL device pointer");
    std::lock_guard<std::mutex> lk(p->mu);
    DeviceGuard dg(p->idx->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (n_ids) HOPH_HIP(hipMemcpyAsync(p->q_ids, d_ids, n_ids * 4, hipMemcpyDeviceToDevice, st), "stage ids");
    HOPH_HIP(hipMemcpyAsync(p->q_offsets, d_offsets, ((uint64_t)n_q + 1) * 8, hipMemcpyDeviceToDevice, st),
             "stage offsets");
    uint64_t n_sets;
    {
        std::lock_guard<std::mutex> il(p->idx->mu);
        n_sets = p->idx->n;
    }
    HOPH_HIP(launch_set_desc(p->desc, n_q, n_sets, st), "descriptor");
    if (p->cfg.tune && !p->tuned && n_q) {
        hoph_status r = tune(p, st, n_sets, n_q);
        if (r) return r;
    }
    if (p->cfg.use_graph) {
        if (!p->exec) {
            hoph_status r = capture(p);
            if (r) return r;
        }
        HOPH_HIP(hipGraphLaunch(p->exec, st), "hipGraphLaunch");
    } else {
        hoph_status r = enqueue_pipeline(p, p->shape, st);
        if (r) return r;
    }
    p->last_nq = n_q;
    p->last_nsets = n_sets;
    p->pending = true;
    return HOPH_OK;
}

hoph_status hoph_plan_results(hoph_plan *p, const uint64_t **d_offsets, const uint32_t **d_set_ids, uint64_t *n_results,
                              void *hip_stream) {
    clear_error();
    if (!p || !d_offsets || !d_set_ids || !n_results) return fail(HOPH_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->pending) return fail(HOPH_E_INVAL, "no batch has been run");
    DeviceGuard dg(p->idx->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HOPH_HIP(hipMemcpyAsync(p->h_counters, p->counters, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, st),
             "read counters");
    HOPH_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    bool general = false;
    hoph_status fo = finish_output(p, st, general);
    if (fo) return fo;
    const uint64_t surv = p->h_counters[0], acc = p->h_counters[1], total = p->h_counters[2], flags = p->h_counters[3];
    *n_results = total;
    const bool exact = surv <= p->surv_cap && acc <= p->keys_cap && (flags & 7ull) == 0;
    if (!exact) {
        // redo on the host-synchronised path with the batch's signatures
        p->note_fallback(surv, acc, flags);
        hoph_results r{p->out_offsets, p->out_ids, p->cfg.max_results, 0};
        hoph_status s = run_query(p->idx, p->q_sigs, p->last_nq, &p->qp, &r, hip_stream, p->kind, false,
                                  p->last_nsets);
        *n_results = r.needed;
        if (s) return s;
    }
    *d_offsets = p->out_offsets;
    *d_set_ids = p->out_ids;
    return HOPH_OK;
}

hoph_status hoph_plan_query_sigs(const hoph_plan *p, const uint32_t **d_qsigs, uint32_t *n_q) {
    clear_error();
    if (!p || !d_qsigs || !n_q) return fail(HOPH_E_INVAL, "NULL argument");
    if (!p->pending) return fail(HOPH_E_INVAL, "no batch has been run");
    *d_qsigs = p->q_sigs;
    *n_q = p->last_nq;
    return HOPH_OK;
}

hoph_status hoph_plan_get_info(const hoph_plan *p, hoph_plan_info *info) {
    clear_error();
    if (!p || !info) return fail(HOPH_E_INVAL, "NULL argument");
    info->q_per_wave = p->shape.q_per_wave;
    info->coarse_waves_per_cu = p->shape.coarse_wpc;
    info->sketch_chunk = p->shape.chunk;
    info->sketch_waves_per_cu = p->shape.sketch_wpc;
    info->depth = p->depth;
    info->graph = p->exec ? 1u : 0u;
    info->tuned = p->tuned ? 1u : 0u;
    info->fallbacks = p->fallbacks;
    info->fallback_causes = p->fallback_causes;
    info->reserved = 0;
    info->tune_ms = p->tune_ms;
    return HOPH_OK;
}

void hoph_plan_free(hoph_plan *p) {
    if (!p) return;
    {
        DeviceGuard dg(p->idx->device);
        (void)hipDeviceSynchronize();
        p->release();
    }
    delete p;
}

}  // extern "C"

namespace hoph {

uint64_t plan_survivor_capacity(uint64_t index_capacity, uint32_t max_queries) {
    // first-pass survivors grow with the batch: the index capacity per 1,024 queries
    return std::max<uint64_t>(index_capacity, 1u << 20) * std::max<uint64_t>(1, (max_queries + 1023) / 1024);
}

hoph_status plan_adopt_and_capture(hoph_plan *p, const hoph_plan *from) {
    if (!p) return fail(HOPH_E_INVAL, "plan is NULL");
    std::lock_guard<std::mutex> lk(p->mu);
    DeviceGuard dg(p->idx->device);
    if (from) {
        p->shape = from->shape;
        p->tuned = from->tuned;
        p->tune_ms = from->tune_ms;
    }
    if (p->cfg.use_graph && !p->exec) return capture(p);
    return HOPH_OK;
}

hoph_status plan_results_to_host(hoph_plan *p, uint64_t *h_offsets, uint32_t *h_ids, uint64_t pre,
                                 uint64_t *n_results, hipStream_t st) {
    if (!p || !h_offsets || !h_ids || !n_results) return fail(HOPH_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(p->mu);
    if (!p->pending) return fail(HOPH_E_INVAL, "no batch has been run");
    DeviceGuard dg(p->idx->device);
    const uint32_t n_q = p->last_nq;
    pre = std::min<uint64_t>(pre, p->cfg.max_results);
    HOPH_HIP(hipMemcpyAsync(p->h_counters, p->counters, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, st),
             "read counters");
    HOPH_HIP(hipMemcpyAsync(h_offsets, p->out_offsets, ((uint64_t)n_q + 1) * 8, hipMemcpyDeviceToHost, st),
             "read result offsets");
    if (pre) HOPH_HIP(hipMemcpyAsync(h_ids, p->out_ids, pre * 4, hipMemcpyDeviceToHost, st), "read result ids");
    HOPH_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    bool general = false;
    hoph_status fo = finish_output(p, st, general);
    if (fo) return fo;
    const uint64_t surv = p->h_counters[0], acc = p->h_counters[1], total = p->h_counters[2], flags = p->h_counters[3];
    uint64_t n = total, have = general ? 0 : pre;     // ids read early are stale once the general stage ran
    if (general)
        HOPH_HIP(hipMemcpyAsync(h_offsets, p->out_offsets, ((uint64_t)n_q + 1) * 8, hipMemcpyDeviceToHost, st),
                 "read result offsets");
    if (!(surv <= p->surv_cap && acc <= p->keys_cap && (flags & 7ull) == 0)) {
        // redo on the host-synchronised path with the batch's signatures
        p->note_fallback(surv, acc, flags);
        hoph_results r{p->out_offsets, p->out_ids, p->cfg.max_results, 0};
        hoph_status s = run_query(p->idx, p->q_sigs, n_q, &p->qp, &r, st, p->kind, false, p->last_nsets);
        if (s) return s;
        n = r.needed;
        HOPH_HIP(hipMemcpyAsync(h_offsets, p->out_offsets, ((uint64_t)n_q + 1) * 8, hipMemcpyDeviceToHost, st),
                 "read result offsets");
        have = 0;
    }
    if (n > p->cfg.max_results) return fail(HOPH_E_CAPACITY, "batch results exceed the plan's max_results");
    if (n > have)
        HOPH_HIP(hipMemcpyAsync(h_ids + have, p->out_ids + have, (n - have) * 4, hipMemcpyDeviceToHost, st),
                 "read result ids");
    if (n > have || have == 0) HOPH_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    *n_results = n;
    return HOPH_OK;
}

}  // namespace hoph
