// The C ABI of libhoph (include/hoph.h): host validation, ownership of the
// index and its workspace, and the order of kernel launches for each call.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "runtime.h"


using namespace hoph;

namespace hoph {

thread_local std::string g_last_error;

void clear_error() { g_last_error.clear(); }

hoph_status fail(hoph_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

hoph_status hip_fail(hipError_t e, const char *what) {
    return fail(HOPH_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// One 32-bit device error word per device, allocated on first use.
std::mutex g_err_mu;
uint32_t *g_err[kMaxDevices] = {};

hoph_status device_err_word(uint32_t **out) {
    int dev = 0;
    HOPH_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(HOPH_E_DEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_err_mu);
    if (!g_err[dev]) {
        uint32_t *p = nullptr;
        HOPH_HIP(hipMalloc(&p, 256), "hipMalloc(error word)");
        HOPH_HIP(hipMemset(p, 0, 256), "hipMemset(error word)");
        g_err[dev] = p;
    }
    *out = g_err[dev];
    return HOPH_OK;
}



bool valid_ratio_T(hoph_ratio T) { return T.den != 0 && T.num != 0 && T.num <= T.den; }
bool valid_ratio_eps(hoph_ratio e) { return e.den != 0 && e.num < e.den; }

hoph_status check_results(const hoph_results *r, uint32_t n_q) {
    if (!r) return fail(HOPH_E_INVAL, "results is NULL");
    if (!r->d_offsets) return fail(HOPH_E_INVAL, "results->d_offsets is NULL");
    if (r->capacity && !r->d_set_ids) return fail(HOPH_E_INVAL, "results->d_set_ids is NULL");
    (void)n_q;
    return HOPH_OK;
}


// Pick queries per wavefront so that the grid has enough wavefronts to fill
// the device (about 32 per CU) without splitting the query batch further, and
// into at most one chunk per kChunkQueries queries (each chunk reads the
// index's planes again).
uint32_t pick_q_per_wave(uint64_t n_sets, uint32_t n_q, uint32_t tiles_per_wave, bool tri) {
    const uint64_t per_wave = 64ull * std::max<uint32_t>(1, tiles_per_wave);
    const uint64_t ntiles = std::max<uint64_t>(1, (n_sets + per_wave - 1) / per_wave);
    // about four rounds of items; the self-join keeps about half of its items
    // (the upper triangle) and takes about eight rounds of those, so that the
    // last round's stragglers cost little
    const uint64_t rounds = tri ? 16 : 4;
    uint64_t want_chunks = (rounds * 8192ull + ntiles - 1) / ntiles;
    want_chunks = std::min<uint64_t>(want_chunks, std::max<uint64_t>(1, n_q / kChunkQueries));
    if (want_chunks == 0) want_chunks = 1;
    return (uint32_t)((n_q + want_chunks - 1) / want_chunks);
}

hoph_status copy_counters(Workspace &ws, hipStream_t st) {
    HOPH_HIP(hipMemcpyAsync(ws.h_counters, ws.counters, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, st),
             "hipMemcpyAsync(counters)");
    HOPH_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    return HOPH_OK;
}

// Accepted keys -> per-query ascending CSR in the caller's buffers: counting,
// scan, scatter and a per-query LDS sort of up to seg_max ids, seg_max the
// total's power of two up to 16384, so that below that total no query can
// exceed it and no flag has to be read back; above it the device reports a
// larger query in counters[3] and the global bitonic sort takes over.
hoph_status write_output(Workspace &ws, uint64_t accepted, uint32_t n_q, hoph_results *res, hipStream_t s) {
    hoph_status st = ws.grow_seg((uint64_t)n_q + 1);
    if (st) return st;
    uint32_t seg_max = 2;
    while (seg_max < accepted && seg_max < 16384) seg_max <<= 1;
    HOPH_HIP(launch_segmented_output(ws.keys, ws.counters, ws.keys_cap, ws.qcount, nullptr, n_q, res->d_offsets,
                                     ws.cursor, res->d_set_ids, res->capacity, ws.counters, n_q, accepted, seg_max, s),
             "output launch");
    if (accepted > seg_max) {
        HOPH_HIP(hipMemcpyAsync(ws.h_counters + 2, ws.counters + 2, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s),
                 "hipMemcpyAsync(flags)");
        HOPH_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (ws.h_counters[3] & 1ull) {
            HOPH_HIP(launch_sort_keys(ws.keys, accepted, sort_capacity(accepted), s), "sort launch");
            HOPH_HIP(launch_results(ws.keys, accepted, n_q, res->d_offsets, res->d_set_ids, s), "results launch");
        }
    }
    return HOPH_OK;
}

hipError_t append_sets_async(hoph_index *idx, const uint32_t *d_ids, const uint64_t *d_offsets, uint64_t n_sets,
                             uint64_t first, uint32_t *err_word, hipStream_t s, bool timed) {
    SketchDesc d;
    fill_sketch_desc(idx->params, idx->lay, d);
    hipError_t e = hipSuccess;
    // code planes of the new rows: the row kernel where it reads a group with
    // vector loads, else the sketch writes them from its LDS signature (then
    // aev[1]..aev[2] spans no work)
    const uint32_t ub = code_unit_bins(idx->lay.kp, idx->lay.L), cu = code_units(idx->cg, idx->lay.kp, idx->lay.L);
    const bool fused = idx->codes && !codes_have_row_kernel(idx->lay.k, ub);
    const CodeSink sink = fused ? CodeSink{idx->codes, first, idx->capacity / 64, cu, ub} : CodeSink{};
    if (timed && (e = hipEventRecord(idx->ws.aev[0], s)) != hipSuccess) return e;
    e = launch_sketch(d, d_ids, d_offsets, n_sets, idx->slab + first * idx->lay.k, err_word, s, sink);
    if (e != hipSuccess) return e;
    if (timed && (e = hipEventRecord(idx->ws.aev[1], s)) != hipSuccess) return e;
    if (!fused) {
        e = launch_codes_from_slab(idx->slab, idx->capacity, idx->lay.k, ub, first, n_sets, idx->codes, cu, s);
        if (e != hipSuccess) return e;
    }
    if (timed && (e = hipEventRecord(idx->ws.aev[2], s)) != hipSuccess) return e;
    if (timed) idx->ws.aev_recorded = true;
    return hipSuccess;
}

hoph_status cached_scan_tab(hoph_index *idx, const hoph_query_params &qp, bool goph, ScanTab &out,
                            TabEntry **entry) {
    for (TabEntry &e : idx->tabs) {
        if (e.T.num == qp.T.num && e.T.den == qp.T.den && e.eps.num == qp.eps.num && e.eps.den == qp.eps.den &&
            e.policy == qp.empty_policy && e.goph == (goph ? 1u : 0u)) {
            out = e.tab;
            if (entry) *entry = &e;
            return HOPH_OK;
        }
    }
    hoph_decision_tables t;
    std::string err;
    hoph_status st = build_tables(idx->lay, qp, goph, t, err);
    if (st) return fail(st, err);
    TabEntry e;
    e.T = qp.T;
    e.eps = qp.eps;
    e.policy = qp.empty_policy;
    e.goph = goph ? 1u : 0u;
    to_scan_tab(t, e.tab);
    out = e.tab;
    TabEntry *slot;
    if (idx->tabs.size() < kTabCache) {
        idx->tabs.push_back(e);                  // within the capacity reserved at build
        slot = &idx->tabs.back();
    } else {
        slot = &idx->tabs[idx->tab_next];
        *slot = e;
        idx->tab_next = (idx->tab_next + 1) % kTabCache;
    }
    if (entry) *entry = slot;
    return HOPH_OK;
}

// The first-group pass's keep rates for these tables (ent), sampled from the
// first n_sets index rows when none were taken yet or the index has since
// grown or shrunk more than twofold, and when sampling is allowed (it reads a
// few rows back to the host and synchronises s); false when there are none.
hoph_status index_keep_rates(hoph_index *idx, TabEntry &ent, uint64_t n_sets, hipStream_t s, bool may_sample,
                             double rate[8], bool &have) {
    have = false;
    const bool stale = ent.keep_n == 0 || n_sets > 2 * ent.keep_n || 2 * n_sets < ent.keep_n;
    if (stale && may_sample && n_sets >= 2) {
        HOPH_HIP(sample_keep_rates(idx->codes, n_sets, idx->lay.kp, ent.tab.dthr0, ent.keep_rate, s),
                 "sample_keep_rates");
        ent.keep_n = n_sets;
    }
    if (ent.keep_n == 0) return HOPH_OK;
    std::memcpy(rate, ent.keep_rate, sizeof(ent.keep_rate));
    have = true;
    return HOPH_OK;
}

namespace {

// time_reps > 0: a measurement run instead of a query -- the coarse pass alone,
// time_reps launches back to back between two events, the mean written to
// *time_ms; no output is written (res may be a dummy).  With flush_bytes > 0 a
// read of flush[0 .. flush_bytes) precedes every timed pass, so that each pass
// starts with the index's planes out of the caches (which then hold clean
// lines only), and the time of the same reads alone is taken off.
hoph_status run_query_impl(const hoph_index *cidx, Workspace *ws_in, const uint32_t *d_qsigs, uint32_t n_q,
                           const hoph_query_params *qp, hoph_results *res, void *stream, QueryKind kind,
                           bool self_join, uint64_t n_limit, uint32_t time_reps = 0, float *time_ms = nullptr,
                           uint32_t *flush = nullptr, uint64_t flush_bytes = 0) {
    if (!cidx) return fail(HOPH_E_INVAL, "index is NULL");
    if (!qp) return fail(HOPH_E_INVAL, "query params are NULL");
    if (self_join) {
        // the queries are the index rows themselves; only set id > row is reported
        if (kind == QueryKind::OPH_FULL) return fail(HOPH_E_UNSUPPORTED, "self-join of the plain OPH comparator");
        d_qsigs = cidx->slab;
        n_q = (uint32_t)cidx->n;
    }
    if (n_q && !d_qsigs) return fail(HOPH_E_INVAL, "d_qsigs is NULL");
    if (!valid_ratio_T(qp->T)) return fail(HOPH_E_INVAL, "T must be an exact ratio in (0, 1]");
    if (kind != QueryKind::OPH_FULL && !valid_ratio_eps(qp->eps)) return fail(HOPH_E_INVAL, "eps must be in [0, 1)");
    if (qp->empty_policy > HOPH_EMPTY_EITHER) return fail(HOPH_E_INVAL, "unknown empty policy");
    if (qp->coarse_filter > HOPH_COARSE_WORDS) return fail(HOPH_E_INVAL, "unknown coarse filter");
    hoph_status st = check_results(res, n_q);
    if (st) return st;
    hoph_index *idx = const_cast<hoph_index *>(cidx);
    if (kind == QueryKind::GOPH && idx->params.layout != HOPH_LAYOUT_OPH)
        return fail(HOPH_E_INVAL, "query_goph needs an index built with HOPH_LAYOUT_OPH");
    if (kind == QueryKind::HOPH && idx->params.layout != HOPH_LAYOUT_HIER)
        return fail(HOPH_E_INVAL, "query_hoph needs an index built with HOPH_LAYOUT_HIER");
    std::lock_guard<std::mutex> lk(idx->mu);
    DeviceGuard dg(idx->device);
    if (!dg.ok) return fail(HOPH_E_DEVICE, "cannot select the index device");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const LayoutInfo &lay = idx->lay;
    const uint64_t n_sets = std::min(idx->n, n_limit);   // rows this call compares against
    Workspace &ws = ws_in ? *ws_in : idx->ws;
    const bool timed_ev = ws.ev[0] != nullptr;       // a fixed workspace has no events

    ScanTab tab{};
    TabEntry *tab_entry = nullptr;
    uint32_t depth = 0, maxd = 0;
    const bool use_codes = kind != QueryKind::OPH_FULL && qp->coarse_filter == HOPH_COARSE_CODES && idx->codes;
    if (kind != QueryKind::OPH_FULL) {
        st = cached_scan_tab(idx, *qp, kind == QueryKind::GOPH, tab, &tab_entry);
        if (st) return st;
        maxd = use_codes ? idx->cg : std::min(max_depth_for_kpad(idx->kpad), lay.L);
        depth = default_coarse_depth(tab, qp->coarse_depth, maxd, use_codes ? code_pack(lay.kp, lay.L) : 1u);
    }

    ScanLaunch a{};
    a.slab = idx->slab;
    a.capacity = idx->capacity;
    a.n_sets = n_sets;
    a.kpad = idx->kpad;
    a.kp = lay.kp;
    a.L = lay.L;
    a.k = lay.k;
    a.qsigs = d_qsigs;
    a.depth = depth;
    a.tri = self_join;
    a.counters = ws.counters;
    a.codes = use_codes ? idx->codes : nullptr;
    a.cg = idx->cg;
    bool counters_zeroed = false;                    // by the query-record launch (no fill launch needed)
    if (kind != QueryKind::OPH_FULL && n_q && n_sets) {
        st = ws.grow_qmasks((uint64_t)n_q * lay.L);
        if (st) return st;
        CodeThr thr{};
        LinTab lin;
        bool with_lin = false;
        if (use_codes) {
            st = ws.grow_qcodes(((uint64_t)n_q + 1) * idx->cg * code_rec_words(lay.kp));  // + a padding record
            if (st) return st;
            std::memcpy(thr.dthr, tab.dthr0, sizeof(thr.dthr));
            with_lin = lin_records(a, tab, &lin);
        }
        HOPH_HIP(launch_query_masks(d_qsigs, n_q, nullptr, lay.k, lay.kp, lay.L, ws.qmasks,
                                    use_codes ? ws.qcodes : nullptr, idx->cg, &thr, s, with_lin ? &lin : nullptr,
                                    ws.counters, 4),
                 "query mask launch");
        counters_zeroed = true;
    }
    a.qmasks = ws.qmasks;
    a.qcodes = ws.qcodes;
    // A self-join's first-group pass picks its kernel and plane count with keep
    // rates measured on sampled pairs of index rows, taken once per index size
    // and parameters.  (Query batches keep the binomial rates: on bag-of-words
    // sets, where background pairs agree on more bins, 1,024 queries over 10^6
    // sets still ran fastest at the plane count those give, 0.139 ms at 2
    // planes against 0.175 ms at the 3 the sampled rates pick.)
    double keep_rate[8];
    if (self_join && use_codes && tab_entry && depth == 1 && tab.policy != HOPH_EMPTY_EITHER &&
        code_plane_words(lay.kp) == 1 && n_q && n_sets >= 2) {
        bool have = false;
        st = index_keep_rates(idx, *tab_entry, n_sets, s, ws_in == nullptr, keep_rate, have);
        if (st) return st;
        if (have) a.keep_rate = keep_rate;
    }

    // one pass over queries [q0, q1) (coarse, then per-survivor), events ev[0..2]
    uint32_t plan[4] = {0, HOPH_PLAN_NONE, 0, 0};
    auto pass = [&](uint32_t q0, uint32_t q1) -> hoph_status {
        a.q0 = q0;
        a.q1 = q1;
        a.q_per_wave = pick_q_per_wave(n_sets, q1 - q0, coarse_tiles_per_wave(a, tab), a.tri);
        if (kind == QueryKind::OPH_FULL) {
            plan[0] = 0;
            plan[1] = HOPH_PLAN_OPH_FULL;
            plan[2] = 0;
            plan[3] = 1;
        } else {
            describe_coarse(a, tab, plan);
        }
        if (timed_ev) HOPH_HIP(hipEventRecord(ws.ev[0], s), "hipEventRecord");
        if (kind == QueryKind::OPH_FULL) {
            HOPH_HIP(launch_oph_full(a, qp->T, qp->empty_policy, s), "oph_full launch");
            if (timed_ev) HOPH_HIP(hipEventRecord(ws.ev[1], s), "hipEventRecord");
        } else {
            HOPH_HIP(launch_scan_coarse(a, tab, s), "coarse scan launch");
            if (timed_ev) HOPH_HIP(hipEventRecord(ws.ev[1], s), "hipEventRecord");
            HOPH_HIP(launch_scan_fine(a, tab, s), "fine scan launch");
        }
        if (timed_ev) HOPH_HIP(hipEventRecord(ws.ev[2], s), "hipEventRecord");
        return HOPH_OK;
    };
    if (time_reps) {
        if (!timed_ev || kind == QueryKind::OPH_FULL) return fail(HOPH_E_INVAL, "coarse-pass timing needs the index workspace");
        *time_ms = 0.f;
        if (!n_q || !n_sets) return HOPH_OK;
        a.surv = ws.surv;
        a.surv_cap = ws.surv_cap;
        a.keys = ws.keys;
        a.keys_cap = ws.keys_cap;
        a.q0 = 0;
        a.q1 = n_q;
        a.q_per_wave = pick_q_per_wave(n_sets, n_q, coarse_tiles_per_wave(a, tab), a.tri);
        HOPH_HIP(launch_fill_u64(ws.counters, 4, 0, s), "fill counters");
        HOPH_HIP(launch_scan_coarse(a, tab, s), "coarse scan launch");    // warm: code object, caches
        if (flush_bytes) HOPH_HIP(launch_read_sweep(flush, flush_bytes, flush, s), "flush read");   // warm it
        HOPH_HIP(hipEventRecord(ws.ev[0], s), "hipEventRecord");
        // survivors past the buffer are counted, not written, so repeated passes stay in bounds
        for (uint32_t r = 0; r < time_reps; ++r) {
            if (flush_bytes) HOPH_HIP(launch_read_sweep(flush, flush_bytes, flush, s), "flush read");
            HOPH_HIP(launch_scan_coarse(a, tab, s), "coarse scan launch");
        }
        HOPH_HIP(hipEventRecord(ws.ev[1], s), "hipEventRecord");
        if (flush_bytes) {
            HOPH_HIP(hipEventRecord(ws.ev[2], s), "hipEventRecord");
            for (uint32_t r = 0; r < time_reps; ++r)
                HOPH_HIP(launch_read_sweep(flush, flush_bytes, flush, s), "flush read");
            HOPH_HIP(hipEventRecord(ws.ev[3], s), "hipEventRecord");
        }
        HOPH_HIP(hipEventSynchronize(flush_bytes ? ws.ev[3] : ws.ev[1]), "hipEventSynchronize");
        describe_coarse(a, tab, ws.last_plan);
        float ms = 0.f, flush_ms = 0.f;
        HOPH_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[1]), "hipEventElapsedTime");
        if (flush_bytes) HOPH_HIP(hipEventElapsedTime(&flush_ms, ws.ev[2], ws.ev[3]), "hipEventElapsedTime");
        *time_ms = std::max(0.f, ms - flush_ms) / (float)time_reps;
        return HOPH_OK;
    }
    auto record_timing = [&]() {
        if (!timed_ev) return;
        (void)hipEventElapsedTime(&ws.last_ms[0], ws.ev[0], ws.ev[1]);
        (void)hipEventElapsedTime(&ws.last_ms[1], ws.ev[1], ws.ev[2]);
        (void)hipEventElapsedTime(&ws.last_ms[2], ws.ev[2], ws.ev[3]);
    };

    if (n_q && n_sets) {
        // Optimistic path, one read-back: the pass and the output stage (which takes
        // its counts from the device) back to back, then the counters and flags.  It
        // stands when no buffer overflowed and no query holds more ids than the
        // per-query sort takes; otherwise the careful path below redoes the query.
        st = ws.grow_seg((uint64_t)n_q + 1);
        if (st) return st;
        a.surv = ws.surv;
        a.surv_cap = ws.surv_cap;
        a.keys = ws.keys;
        a.keys_cap = ws.keys_cap;
        if (!counters_zeroed) HOPH_HIP(launch_fill_u64(ws.counters, 4, 0, s), "fill counters");
        st = pass(0, n_q);
        if (st) return st;
        // a batch of up to kSmallOutQueries queries tries the one-workgroup output
        // stage first (one launch instead of five); it leaves counters[3] = 4 when
        // more keys were accepted than it sorts, and the general stage follows
        auto general_output = [&]() {
            return launch_segmented_output(ws.keys, ws.counters, ws.keys_cap, ws.qcount, nullptr, n_q,
                                           res->d_offsets, ws.cursor, res->d_set_ids, res->capacity, ws.counters,
                                           n_q, ws.keys_cap, kSegMaxPlan, s);
        };
        // (skipped when the workspace's last batch, scaled to this one, accepted
        // more pairs than it sorts: that saves a second read-back)
        const uint64_t expect = ws.last_nq ? ws.last_counts[1] * n_q / ws.last_nq : 0;
        if (n_q <= kSmallOutQueries && expect <= kSmallOutKeys) {
            HOPH_HIP(launch_small_output(ws.keys, ws.counters, ws.keys_cap, nullptr, n_q, res->d_offsets,
                                         res->d_set_ids, res->capacity, s),
                     "output launch");
        } else {
            HOPH_HIP(general_output(), "output launch");
        }
        if (timed_ev) HOPH_HIP(hipEventRecord(ws.ev[3], s), "hipEventRecord");
        HOPH_HIP(hipMemcpyAsync(ws.h_counters, ws.counters, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, s),
                 "hipMemcpyAsync(counters)");
        HOPH_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        const uint64_t surv = ws.h_counters[0], acc = ws.h_counters[1];
        const bool fits = surv <= ws.surv_cap && acc <= ws.keys_cap && acc <= res->capacity;
        if (fits && (ws.h_counters[3] & 4ull)) {
            HOPH_HIP(general_output(), "output launch");
            if (timed_ev) HOPH_HIP(hipEventRecord(ws.ev[3], s), "hipEventRecord");
            HOPH_HIP(hipMemcpyAsync(ws.h_counters + 2, ws.counters + 2, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                    s),
                     "hipMemcpyAsync(flags)");
            HOPH_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        const uint64_t flags = ws.h_counters[3];
        if (fits && (flags & 7ull) == 0) {
            res->needed = acc;
            ws.last_counts[0] = surv;
            ws.last_counts[1] = acc;
            ws.last_nq = n_q;
            std::memcpy(ws.last_plan, plan, sizeof(plan));
            record_timing();
            return HOPH_OK;
        }
        // survivors overflowed at the library's depth: walk every group that can be
        // walked before splitting the batch (a deeper pass keeps fewer pairs)
        if (surv > ws.surv_cap && qp->coarse_depth == 0 && a.depth < maxd) a.depth = maxd;
    }

    uint64_t accepted = 0, survivors = 0;
    float pass_ms[2] = {0, 0};
    for (int attempt = 0; attempt < 2; ++attempt) {
        a.surv = ws.surv;
        a.surv_cap = ws.surv_cap;
        a.keys = ws.keys;
        a.keys_cap = ws.keys_cap;
        HOPH_HIP(launch_fill_u64(ws.counters, 2, 0, s), "fill counters");
        bool fresh = false;                 // h_counters hold this attempt's device counters
        if (n_q && n_sets) {
            // one pass over the whole batch; on survivor overflow, redo in sub-batches
            st = pass(0, n_q);
            if (st) return st;
            st = copy_counters(ws, s);
            if (st) return st;
            if (timed_ev) {
                (void)hipEventElapsedTime(&pass_ms[0], ws.ev[0], ws.ev[1]);
                (void)hipEventElapsedTime(&pass_ms[1], ws.ev[1], ws.ev[2]);
            }
            survivors = ws.h_counters[0];
            if (ws.h_counters[0] > ws.surv_cap) {
                const uint64_t seen = ws.h_counters[0];
                HOPH_HIP(launch_fill_u64(ws.counters, 2, 0, s), "fill counters");
                uint64_t acc_before = 0;
                uint32_t sub = (uint32_t)std::max<uint64_t>(1, (uint64_t)n_q * ws.surv_cap / seen / 2);
                uint32_t q = 0;
                while (q < n_q) {
                    const uint32_t q1 = (uint32_t)std::min<uint64_t>(n_q, (uint64_t)q + sub);
                    HOPH_HIP(launch_fill_u64(ws.counters, 1, 0, s), "fill counters");
                    st = pass(q, q1);
                    if (st) return st;
                    st = copy_counters(ws, s);
                    if (st) return st;
                    if (ws.h_counters[0] > ws.surv_cap) {
                        if (sub == 1)
                            return fail(ws.fixed ? HOPH_E_CAPACITY : HOPH_E_NOMEM,
                                        "one query keeps more survivors than the survivor buffer holds");
                        sub = std::max<uint32_t>(1, sub / 2);
                        HOPH_HIP(launch_fill_u64(ws.counters + 1, 1, acc_before, s), "fill counters");
                        continue;
                    }
                    acc_before = ws.h_counters[1];
                    q = q1;
                }
            }
            fresh = true;
        }
        if (!fresh) {
            ws.h_counters[0] = ws.h_counters[1] = 0;     // nothing was scanned
        }
        accepted = ws.h_counters[1];
        if (accepted <= ws.keys_cap) break;
        if (accepted > res->capacity) break;      // reported below; no need to keep every key
        st = ws.grow_keys(accepted);
        if (st) return st;
    }
    res->needed = accepted;
    if (accepted > res->capacity) {
        return fail(HOPH_E_CAPACITY, "results capacity " + std::to_string(res->capacity) + " < " +
                                         std::to_string(accepted) + " accepted pairs");
    }
    const bool timed = n_q && n_sets;
    if (timed && timed_ev) HOPH_HIP(hipEventRecord(ws.ev[2], s), "hipEventRecord");
    st = write_output(ws, accepted, n_q, res, s);
    if (st) return st;
    if (timed && timed_ev) HOPH_HIP(hipEventRecord(ws.ev[3], s), "hipEventRecord");
    HOPH_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    ws.last_counts[0] = survivors;
    ws.last_counts[1] = accepted;
    ws.last_nq = n_q;
    std::memcpy(ws.last_plan, plan, sizeof(plan));
    ws.last_ms[0] = ws.last_ms[1] = ws.last_ms[2] = 0.f;
    if (timed && timed_ev) {
        ws.last_ms[0] = pass_ms[0];
        ws.last_ms[1] = pass_ms[1];
        (void)hipEventElapsedTime(&ws.last_ms[2], ws.ev[2], ws.ev[3]);
    }
    return HOPH_OK;
}

}  // namespace

hoph_status run_query(const hoph_index *cidx, const uint32_t *d_qsigs, uint32_t n_q, const hoph_query_params *qp,
                      hoph_results *res, void *stream, QueryKind kind, bool self_join, uint64_t n_limit) {
    return run_query_impl(cidx, nullptr, d_qsigs, n_q, qp, res, stream, kind, self_join, n_limit);
}

hoph_status scan_timing(const hoph_index *cidx, const uint32_t *d_qsigs, uint32_t n_q, const hoph_query_params *qp,
                        uint32_t reps, void *d_flush, uint64_t flush_bytes, float *ms, void *stream) {
    if (!cidx || !ms) return fail(HOPH_E_INVAL, "NULL argument");
    if (reps == 0) return fail(HOPH_E_INVAL, "reps must be >= 1");
    if (flush_bytes && !d_flush) return fail(HOPH_E_INVAL, "d_flush is NULL");
    if (reinterpret_cast<uintptr_t>(d_flush) % 16) return fail(HOPH_E_INVAL, "d_flush must be 16-byte aligned");
    if (flush_bytes && flush_bytes < kSweepSinkBytes)
        return fail(HOPH_E_INVAL, "flush_bytes must be 0 or at least 4 MiB");
    const QueryKind kind = cidx->params.layout == HOPH_LAYOUT_OPH ? QueryKind::GOPH : QueryKind::HOPH;
    uint64_t dummy_off = 0;
    hoph_results r{&dummy_off, nullptr, 0, 0};
    return run_query_impl(cidx, nullptr, d_qsigs, n_q, qp, &r, stream, kind, false, ~0ull, reps, ms,
                          static_cast<uint32_t *>(d_flush), flush_bytes / 16 * 16);
}

hoph_status run_query_in(const hoph_index *cidx, Workspace &ws, const uint32_t *d_qsigs, uint32_t n_q,
                         const hoph_query_params *qp, hoph_results *res, void *stream, QueryKind kind) {
    return run_query_impl(cidx, &ws, d_qsigs, n_q, qp, res, stream, kind, false, ~0ull);
}

// Workspace for MinWise queries, one per device.
std::mutex g_mw_mu;
Workspace *g_mw_ws[kMaxDevices] = {};

}  // namespace hoph

extern "C" {

const char *hoph_status_str(hoph_status s) {
    switch (s) {
    case HOPH_OK: return "HOPH_OK";
    case HOPH_E_INVAL: return "HOPH_E_INVAL";
    case HOPH_E_RANGE: return "HOPH_E_RANGE";
    case HOPH_E_CAPACITY: return "HOPH_E_CAPACITY";
    case HOPH_E_NOMEM: return "HOPH_E_NOMEM";
    case HOPH_E_UNSUPPORTED: return "HOPH_E_UNSUPPORTED";
    case HOPH_E_DEVICE: return "HOPH_E_DEVICE";
    }
    return "HOPH_E_UNKNOWN";
}

const char *hoph_last_error(void) { return g_last_error.c_str(); }

hoph_status sketch_oph(const hoph_sketch_params *params, const uint32_t *d_ids, const uint64_t *d_offsets,
                       uint64_t n_sets, uint32_t *d_sigs, void *hip_stream) {
    g_last_error.clear();
    if (!params) return fail(HOPH_E_INVAL, "params is NULL");
    LayoutInfo lay;
    std::string err;
    hoph_status st = build_layout(*params, lay, err);
    if (st) return fail(st, err);
    if (n_sets == 0) return HOPH_OK;
    if (!d_offsets || !d_sigs) return fail(HOPH_E_INVAL, "d_offsets / d_sigs is NULL");
    if (!d_ids) return fail(HOPH_E_INVAL, "d_ids is NULL");
    uint32_t *errw = nullptr;
    st = device_err_word(&errw);
    if (st) return st;
    SketchDesc d;
    fill_sketch_desc(*params, lay, d);
    HOPH_HIP(launch_sketch(d, d_ids, d_offsets, n_sets, d_sigs, errw, reinterpret_cast<hipStream_t>(hip_stream)),
             "sketch launch");
    return HOPH_OK;
}

hoph_status build_index(const hoph_sketch_params *params, const uint32_t *d_sigs, uint64_t n_sets, uint64_t capacity,
                        hoph_index **out, void *hip_stream) {
    g_last_error.clear();
    if (!params || !out) return fail(HOPH_E_INVAL, "params / out is NULL");
    *out = nullptr;
    if (n_sets && !d_sigs) return fail(HOPH_E_INVAL, "d_sigs is NULL");
    if (capacity < n_sets) return fail(HOPH_E_INVAL, "capacity < n_sets");
    if (capacity > 0xFFFFFFFFull) return fail(HOPH_E_INVAL, "capacity exceeds 2^32 sets (set ids are uint32)");
    std::unique_ptr<hoph_index> idx(new (std::nothrow) hoph_index());
    if (!idx) return fail(HOPH_E_NOMEM, "host allocation");
    std::string err;
    hoph_status st = build_layout(*params, idx->lay, err);
    if (st) return fail(st, err);
    HOPH_HIP(hipGetDevice(&idx->device), "hipGetDevice");
    idx->params = *params;
    idx->kpad = round4(params->k_group);
    idx->capacity = std::max<uint64_t>(64, (capacity + 63) / 64 * 64);
    idx->max_sets = capacity;
    const uint64_t words = idx->capacity * idx->lay.k;          // row-major signature words
    idx->cg = code_groups(idx->lay.kp, idx->lay.L, params->layout == HOPH_LAYOUT_HIER);
    const uint32_t ub = code_unit_bins(idx->lay.kp, idx->lay.L), cu = code_units(idx->cg, idx->lay.kp, idx->lay.L);
    const uint64_t code_words_total = idx->capacity * cu * code_words(idx->lay.kp);
    auto release = [&] {
        if (idx->slab) (void)hipFree(idx->slab);
        if (idx->codes) (void)hipFree(idx->codes);
        idx->slab = nullptr;
        idx->codes = nullptr;
        idx->ws.release();
    };
    if (hipMalloc(&idx->slab, words * sizeof(uint32_t)) != hipSuccess) return fail(HOPH_E_NOMEM, "index slabs");
    if (hipMalloc(&idx->codes, code_words_total * sizeof(uint32_t)) != hipSuccess) {
        release();
        return fail(HOPH_E_NOMEM, "index code planes");
    }
    st = idx->ws.init(std::max<uint64_t>(idx->capacity, 1u << 20), 1u << 16);
    if (st) {
        release();
        return st;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = launch_index_store(d_sigs, n_sets, 0, params->k, idx->capacity, idx->slab, idx->codes, ub, cu, s);
    if (e != hipSuccess) {
        release();
        return hip_fail(e, "index store launch");
    }
    idx->n = n_sets;
    idx->tabs.reserve(kTabCache);
    *out = idx.release();
    return HOPH_OK;
}

hoph_status index_append(hoph_index *idx, const uint32_t *d_sigs, uint64_t n_new, void *hip_stream) {
    g_last_error.clear();
    if (!idx) return fail(HOPH_E_INVAL, "index is NULL");
    if (n_new == 0) return HOPH_OK;
    if (!d_sigs) return fail(HOPH_E_INVAL, "d_sigs is NULL");
    std::lock_guard<std::mutex> lk(idx->mu);
    if (idx->n + n_new > idx->max_sets)
        return fail(HOPH_E_CAPACITY, "index capacity " + std::to_string(idx->max_sets) + " exceeded");
    DeviceGuard dg(idx->device);
    HOPH_HIP(launch_index_store(d_sigs, n_new, idx->n, idx->params.k, idx->capacity, idx->slab, idx->codes,
                                code_unit_bins(idx->lay.kp, idx->lay.L), code_units(idx->cg, idx->lay.kp, idx->lay.L),
                                reinterpret_cast<hipStream_t>(hip_stream)),
             "index store launch");
    idx->n += n_new;
    return HOPH_OK;
}

hoph_status index_append_sets(hoph_index *idx, const uint32_t *d_ids, const uint64_t *d_offsets, uint64_t n_sets,
                              void *hip_stream) {
    g_last_error.clear();
    if (!idx) return fail(HOPH_E_INVAL, "index is NULL");
    if (n_sets == 0) return HOPH_OK;
    if (!d_ids || !d_offsets) return fail(HOPH_E_INVAL, "d_ids / d_offsets is NULL");
    std::lock_guard<std::mutex> lk(idx->mu);
    if (idx->n + n_sets > idx->max_sets)
        return fail(HOPH_E_CAPACITY, "index capacity " + std::to_string(idx->max_sets) + " exceeded");
    DeviceGuard dg(idx->device);
    uint32_t *errw = nullptr;
    hoph_status st = device_err_word(&errw);
    if (st) return st;
    const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    HOPH_HIP(append_sets_async(idx, d_ids, d_offsets, n_sets, idx->n, errw, s, true), "sketch-into-index launch");
    idx->n += n_sets;
    return HOPH_OK;
}

uint64_t hoph_index_size(const hoph_index *idx) { return idx ? idx->n : 0; }

hoph_status hoph_index_code_planes(const hoph_index *idx, uint32_t *d_out, uint64_t out_words, uint64_t dims[3],
                                   void *hip_stream) {
    g_last_error.clear();
    if (!idx || !dims) return fail(HOPH_E_INVAL, "NULL argument");
    dims[0] = code_units(idx->cg, idx->lay.kp, idx->lay.L);
    dims[1] = idx->capacity;
    dims[2] = code_words(idx->lay.kp);
    const uint64_t words = dims[0] * dims[1] * dims[2];
    if (!idx->codes || words == 0) return HOPH_OK;
    if (out_words < words) return fail(HOPH_E_CAPACITY, "output smaller than the code planes");
    if (!d_out) return fail(HOPH_E_INVAL, "d_out is NULL");
    DeviceGuard dg(idx->device);
    if (!dg.ok) return fail(HOPH_E_DEVICE, "cannot select the index device");
    HOPH_HIP(hipMemcpyAsync(d_out, idx->codes, words * 4, hipMemcpyDeviceToDevice,
                            reinterpret_cast<hipStream_t>(hip_stream)),
             "hipMemcpyAsync(code planes)");
    return HOPH_OK;
}

hoph_status hoph_index_rows(const hoph_index *idx, uint64_t first, uint64_t n, uint32_t *d_out, void *hip_stream) {
    g_last_error.clear();
    if (!idx) return fail(HOPH_E_INVAL, "index is NULL");
    if (first > idx->n || n > idx->n - first) return fail(HOPH_E_RANGE, "rows past the index size");
    if (n == 0) return HOPH_OK;
    if (!d_out) return fail(HOPH_E_INVAL, "d_out is NULL");
    DeviceGuard dg(idx->device);
    if (!dg.ok) return fail(HOPH_E_DEVICE, "cannot select the index device");
    const uint64_t k = idx->lay.k;
    HOPH_HIP(hipMemcpyAsync(d_out, idx->slab + first * k, n * k * 4, hipMemcpyDeviceToDevice,
                            reinterpret_cast<hipStream_t>(hip_stream)),
             "hipMemcpyAsync(index rows)");
    return HOPH_OK;
}

hoph_status hoph_index_reset(hoph_index *idx) {
    g_last_error.clear();
    if (!idx) return fail(HOPH_E_INVAL, "index is NULL");
    std::lock_guard<std::mutex> lk(idx->mu);
    idx->n = 0;
    return HOPH_OK;
}

hoph_status hoph_query_timing(const hoph_index *idx, float ms[3]) {
    g_last_error.clear();
    if (!idx || !ms) return fail(HOPH_E_INVAL, "NULL argument");
    hoph_index *m = const_cast<hoph_index *>(idx);
    std::lock_guard<std::mutex> lk(m->mu);
    for (int i = 0; i < 3; ++i) ms[i] = m->ws.last_ms[i];
    return HOPH_OK;
}

hoph_status hoph_query_counts(const hoph_index *idx, uint64_t counts[2]) {
    g_last_error.clear();
    if (!idx || !counts) return fail(HOPH_E_INVAL, "NULL argument");
    hoph_index *m = const_cast<hoph_index *>(idx);
    std::lock_guard<std::mutex> lk(m->mu);
    counts[0] = m->ws.last_counts[0];
    counts[1] = m->ws.last_counts[1];
    return HOPH_OK;
}

hoph_status hoph_coarse_plan(const hoph_index *idx, uint32_t plan[4]) {
    g_last_error.clear();
    if (!idx || !plan) return fail(HOPH_E_INVAL, "NULL argument");
    hoph_index *m = const_cast<hoph_index *>(idx);
    std::lock_guard<std::mutex> lk(m->mu);
    std::memcpy(plan, m->ws.last_plan, sizeof(m->ws.last_plan));
    return HOPH_OK;
}

hoph_status hoph_scan_timing(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                             const hoph_query_params *qp, uint32_t reps, void *d_flush, uint64_t flush_bytes,
                             float *ms_per_launch, void *hip_stream) {
    g_last_error.clear();
    return scan_timing(index, d_qsigs, n_q, qp, reps, d_flush, flush_bytes, ms_per_launch, hip_stream);
}

hoph_status hoph_stream_timing(void *d_a, void *d_b, uint64_t bytes, uint32_t reps, float ms[3], void *hip_stream) {
    g_last_error.clear();
    if (!d_a || !d_b || !ms) return fail(HOPH_E_INVAL, "NULL argument");
    if (bytes < kSweepSinkBytes || reps == 0) return fail(HOPH_E_INVAL, "bytes must be at least 4 MiB, reps >= 1");
    if (reinterpret_cast<uintptr_t>(d_a) % 16 || reinterpret_cast<uintptr_t>(d_b) % 8)
        return fail(HOPH_E_INVAL, "d_a must be 16-byte and d_b 8-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    hipEvent_t e[2] = {nullptr, nullptr};
    for (auto &x : e)
        if (hipEventCreate(&x) != hipSuccess) return fail(HOPH_E_DEVICE, "hipEventCreate");
    hoph_status st = HOPH_OK;
    for (int kind = 0; kind < 3 && st == HOPH_OK; ++kind) {
        auto once = [&]() -> hipError_t {
            if (kind == 0) return launch_read_sweep(d_a, bytes / 16 * 16, static_cast<uint32_t *>(d_a), s);
            if (kind == 1) return launch_fill_u64(static_cast<uint64_t *>(d_b), bytes / 8, 1, s);
            return hipMemcpyAsync(d_b, d_a, bytes, hipMemcpyDeviceToDevice, s);
        };
        hipError_t err = once();                              // warm
        if (err == hipSuccess) err = hipEventRecord(e[0], s);
        for (uint32_t r = 0; r < reps && err == hipSuccess; ++r) err = once();
        if (err == hipSuccess) err = hipEventRecord(e[1], s);
        if (err == hipSuccess) err = hipEventSynchronize(e[1]);
        float t = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e[0], e[1]);
        if (err != hipSuccess) st = hip_fail(err, "stream timing");
        ms[kind] = t / (float)reps;
    }
    for (auto &x : e) (void)hipEventDestroy(x);
    return st;
}

hoph_status hoph_append_timing(const hoph_index *idx, float ms[2]) {
    g_last_error.clear();
    if (!idx || !ms) return fail(HOPH_E_INVAL, "NULL argument");
    hoph_index *m = const_cast<hoph_index *>(idx);
    std::lock_guard<std::mutex> lk(m->mu);
    ms[0] = ms[1] = 0.f;
    if (!m->ws.aev_recorded) return HOPH_OK;
    DeviceGuard dg(m->device);
    HOPH_HIP(hipEventSynchronize(m->ws.aev[2]), "hipEventSynchronize");
    (void)hipEventElapsedTime(&ms[0], m->ws.aev[0], m->ws.aev[1]);
    (void)hipEventElapsedTime(&ms[1], m->ws.aev[1], m->ws.aev[2]);
    return HOPH_OK;
}

void hoph_index_free(hoph_index *idx) {
    if (!idx) return;
    {
        DeviceGuard dg(idx->device);
        (void)hipDeviceSynchronize();
        if (idx->slab) (void)hipFree(idx->slab);
        if (idx->codes) (void)hipFree(idx->codes);
        idx->ws.release();
    }
    delete idx;
}

hoph_status query_goph(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q, const hoph_query_params *qp,
                       hoph_results *results, void *hip_stream) {
    g_last_error.clear();
    return run_query(index, d_qsigs, n_q, qp, results, hip_stream, QueryKind::GOPH);
}

hoph_status query_hoph(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q, const hoph_query_params *qp,
                       hoph_results *results, void *hip_stream) {
    g_last_error.clear();
    return run_query(index, d_qsigs, n_q, qp, results, hip_stream, QueryKind::HOPH);
}

hoph_status query_oph_full(const hoph_index *index, const uint32_t *d_qsigs, uint32_t n_q,
                           const hoph_query_params *qp, hoph_results *results, void *hip_stream) {
    g_last_error.clear();
    return run_query(index, d_qsigs, n_q, qp, results, hip_stream, QueryKind::OPH_FULL);
}

static hoph_status check_minwise(const hoph_minwise_params *p) {
    if (!p) return fail(HOPH_E_INVAL, "params is NULL");
    if (p->k == 0 || p->k > 4096) return fail(HOPH_E_INVAL, "k must be in [1, 4096]");
    if (p->hash != HOPH_HASH_MODP31 && p->hash != HOPH_HASH_MODP32P15)
        return fail(HOPH_E_INVAL, "MinWise needs HOPH_HASH_MODP31 or HOPH_HASH_MODP32P15");
    if (p->universe == 0 || p->universe > (1ull << 32)) return fail(HOPH_E_INVAL, "universe must be in [1, 2^32]");
    if (p->hash == HOPH_HASH_MODP31 && p->universe > kP31) return fail(HOPH_E_INVAL, "universe exceeds 2^31 - 1");
    if (!p->d_hash_a || !p->d_hash_b) return fail(HOPH_E_INVAL, "hash coefficient arrays are NULL");
    return HOPH_OK;
}

hoph_status minwise_sketch(const hoph_minwise_params *params, const uint32_t *d_ids, const uint64_t *d_offsets,
                           uint64_t n_sets, uint64_t *d_sigs, void *hip_stream) {
    g_last_error.clear();
    hoph_status st = check_minwise(params);
    if (st) return st;
    if (n_sets == 0) return HOPH_OK;
    if (!d_ids || !d_offsets || !d_sigs) return fail(HOPH_E_INVAL, "NULL device pointer");
    uint32_t *errw = nullptr;
    st = device_err_word(&errw);
    if (st) return st;
    HOPH_HIP(launch_minwise_sketch(params->k, params->hash, params->universe, params->d_hash_a, params->d_hash_b, d_ids,
                                   d_offsets, n_sets, d_sigs, errw, reinterpret_cast<hipStream_t>(hip_stream)),
             "minwise sketch launch");
    return HOPH_OK;
}

hoph_status minwise_query(const hoph_minwise_params *params, const uint64_t *d_sigs, uint64_t n_sets,
                          const uint64_t *d_qsigs, uint32_t n_q, hoph_ratio T, hoph_results *res, void *hip_stream) {
    g_last_error.clear();
    hoph_status st = check_minwise(params);
    if (st) return st;
    if (!valid_ratio_T(T)) return fail(HOPH_E_INVAL, "T must be an exact ratio in (0, 1]");
    st = check_results(res, n_q);
    if (st) return st;
    if ((n_sets && !d_sigs) || (n_q && !d_qsigs)) return fail(HOPH_E_INVAL, "NULL device pointer");
    if (n_sets > 0xFFFFFFFFull) return fail(HOPH_E_INVAL, "n_sets exceeds 2^32");
    int dev = 0;
    HOPH_HIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mw_mu);
    if (!g_mw_ws[dev]) {
        Workspace *w = new (std::nothrow) Workspace();
        if (!w) return fail(HOPH_E_NOMEM, "host allocation");
        st = w->init(1, 1u << 16);
        if (st) { w->release(); delete w; return st; }
        g_mw_ws[dev] = w;
    }
    Workspace &ws = *g_mw_ws[dev];
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    uint64_t accepted = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        HOPH_HIP(launch_fill_u64(ws.counters, 2, 0, s), "fill counters");
        HOPH_HIP(launch_minwise_scan(params->k, d_sigs, n_sets, d_qsigs, 0, n_q, T, ws.keys, ws.keys_cap, ws.counters, s),
                 "minwise scan launch");
        st = copy_counters(ws, s);
        if (st) return st;
        accepted = ws.h_counters[1];
        if (accepted <= ws.keys_cap || accepted > res->capacity) break;
        st = ws.grow_keys(accepted);
        if (st) return st;
    }
    res->needed = accepted;
    if (accepted > res->capacity) return fail(HOPH_E_CAPACITY, "results capacity too small");
    st = write_output(ws, accepted, n_q, res, s);
    if (st) return st;
    HOPH_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    return HOPH_OK;
}

hoph_status hoph_sync(void *hip_stream) {
    g_last_error.clear();
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    HOPH_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    uint32_t *errw = nullptr;
    hoph_status st = device_err_word(&errw);
    if (st) return st;
    uint32_t h = 0;
    HOPH_HIP(hipMemcpy(&h, errw, sizeof(h), hipMemcpyDeviceToHost), "hipMemcpy(error word)");
    if (h) {
        HOPH_HIP(hipMemset(errw, 0, sizeof(uint32_t)), "hipMemset(error word)");
        if (h & kErrRange) return fail(HOPH_E_RANGE, "an id >= universe (or a table value >= universe) was skipped");
        if (h & kErrBadRange) return fail(HOPH_E_INVAL, "a set's end offset is below its start (nothing was read)");
        return fail(HOPH_E_INVAL, "an empty set was sketched (its signature is all EMPTY)");
    }
    return HOPH_OK;
}

hoph_status hoph_layout_starts(const hoph_sketch_params *params, uint64_t *starts) {
    g_last_error.clear();
    if (!params || !starts) return fail(HOPH_E_INVAL, "NULL argument");
    hoph_sketch_params p = *params;
    if (p.hash == HOPH_HASH_TABLE && !p.d_perm) p.d_perm = reinterpret_cast<const uint32_t *>(1);  // not read here
    LayoutInfo lay;
    std::string err;
    hoph_status st = build_layout(p, lay, err);
    if (st) return fail(st, err);
    std::vector<uint64_t> v;
    host_starts(lay, v);
    std::copy(v.begin(), v.end(), starts);
    return HOPH_OK;
}

hoph_status hoph_layout_lookups(const hoph_sketch_params *params, uint32_t *mask) {
    g_last_error.clear();
    if (!params || !mask) return fail(HOPH_E_INVAL, "NULL argument");
    hoph_sketch_params p = *params;
    if (p.hash == HOPH_HASH_TABLE && !p.d_perm) p.d_perm = reinterpret_cast<const uint32_t *>(1);  // not read here
    LayoutInfo lay;
    std::string err;
    hoph_status st = build_layout(p, lay, err);
    if (st) return fail(st, err);
    *mask = (lay.est_ok ? 1u : 0u) | (lay.log_ok ? 2u : 0u) | (lay.pow2_ok ? 4u : 0u);
    return HOPH_OK;
}

hoph_status hoph_tail_integers(uint32_t n, hoph_ratio T, hoph_ratio eps, int32_t *j_lo, int32_t *j_hi) {
    g_last_error.clear();
    if (!j_lo || !j_hi) return fail(HOPH_E_INVAL, "NULL argument");
    std::string err;
    hoph_status st = tail_integers(n, T, eps, *j_lo, *j_hi, err);
    if (st) return fail(st, err);
    return HOPH_OK;
}

hoph_status hoph_build_decision_tables(const hoph_sketch_params *params, const hoph_query_params *qp, uint32_t goph,
                                       hoph_decision_tables *out) {
    g_last_error.clear();
    if (!params || !qp || !out) return fail(HOPH_E_INVAL, "NULL argument");
    if (!valid_ratio_T(qp->T)) return fail(HOPH_E_INVAL, "T must be an exact ratio in (0, 1]");
    if (!valid_ratio_eps(qp->eps)) return fail(HOPH_E_INVAL, "eps must be in [0, 1)");
    hoph_sketch_params p = *params;
    if (p.hash == HOPH_HASH_TABLE && !p.d_perm) p.d_perm = reinterpret_cast<const uint32_t *>(1);  // not read here
    LayoutInfo lay;
    std::string err;
    hoph_status st = build_layout(p, lay, err);
    if (st) return fail(st, err);
    st = build_tables(lay, *qp, goph != 0, *out, err);
    if (st) return fail(st, err);
    return HOPH_OK;
}

hoph_status hoph_first_group_plan(const hoph_sketch_params *params, const hoph_query_params *qp, uint32_t goph,
                                  uint32_t tri, uint32_t small_batch, const double *keep_rate, uint32_t out[3]) {
    g_last_error.clear();
    if (!params || !qp || !out) return fail(HOPH_E_INVAL, "NULL argument");
    if (!valid_ratio_T(qp->T)) return fail(HOPH_E_INVAL, "T must be an exact ratio in (0, 1]");
    if (!valid_ratio_eps(qp->eps)) return fail(HOPH_E_INVAL, "eps must be in [0, 1)");
    if (qp->empty_policy == HOPH_EMPTY_EITHER) return fail(HOPH_E_INVAL, "the first-group code pass runs under JOINT or LITERAL");
    hoph_sketch_params p = *params;
    if (p.hash == HOPH_HASH_TABLE && !p.d_perm) p.d_perm = reinterpret_cast<const uint32_t *>(1);  // not read here
    LayoutInfo lay;
    std::string err;
    hoph_status st = build_layout(p, lay, err);
    if (st) return fail(st, err);
    hoph_decision_tables t;
    st = build_tables(lay, *qp, goph != 0, t, err);
    if (st) return fail(st, err);
    ScanTab tab{};
    to_scan_tab(t, tab);
    first_group_shape(tab, lay.kp, tri != 0, small_batch != 0, keep_rate, out);
    return HOPH_OK;
}

hoph_status hoph_selftest_bins(const hoph_sketch_params *params, const uint32_t *h_perm, const uint32_t *h_ids,
                               uint64_t n, uint32_t *out_bin, uint32_t *out_off) {
    g_last_error.clear();
    if (!params || (n && (!h_ids || !out_bin || !out_off))) return fail(HOPH_E_INVAL, "NULL argument");
    hoph_sketch_params p = *params;
    if (p.hash == HOPH_HASH_TABLE) {
        if (!h_perm) return fail(HOPH_E_INVAL, "h_perm is NULL");
        p.d_perm = h_perm;
    }
    LayoutInfo lay;
    std::string err;
    hoph_status st = build_layout(p, lay, err);
    if (st) return fail(st, err);
    std::vector<uint8_t> lut;
    std::vector<uint64_t> starts;
    host_lut(lay, lut);
    host_starts(lay, starts);
    std::vector<RegionEntry> reg(lay.n_regions + 1);
    for (uint32_t r = 0; r <= lay.n_regions; ++r)
        reg[r] = RegionEntry{lay.reg_start[r], r < lay.n_regions ? lay.reg_magic[r] : 0};
    // the device's 32-bit narrow view (see narrow_value): starts clamped to 2^32 - 1
    const bool narrow = p.hash != HOPH_HASH_TABLE && narrow_view_ok(lay);
    std::vector<uint32_t> s32(starts.size()), rs(lay.reg_start.size());
    for (size_t i = 0; i < starts.size(); ++i) s32[i] = narrow_start(starts[i]);
    for (size_t i = 0; i < rs.size(); ++i) rs[i] = narrow_start(lay.reg_start[i]);
    std::vector<uint32_t> cells(2 * kLogCells), regs(2 * lay.n_regions);
    if (lay.log_ok) {
        for (uint32_t c = 0; c < kLogCells; ++c)
            log_cell_entry(c, narrow_r1(lay.R) + 1u, lay.reg_start.data(), lay.n_regions, cells[2 * c],
                           cells[2 * c + 1]);
        for (uint32_t r = 0; r < lay.n_regions; ++r) {
            regs[2 * r] = (uint32_t)lay.reg_start[r];
            regs[2 * r + 1] = lay.reg_mag32[r];
        }
    }
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t x = h_ids[i];
        if (x >= p.universe) return fail(HOPH_E_RANGE, "id >= universe");
        uint64_t v;
        if (p.hash == HOPH_HASH_TABLE) v = h_perm[x];
        else if (p.hash == HOPH_HASH_MODP31) v = psi_p31(x, p.hash_a, p.hash_b);
        else v = psi_p32(x, p.hash_a, p.hash_b);
        if (v >= lay.R) return fail(HOPH_E_RANGE, "table value >= universe");
        // the region lookup always; the uniform estimate too where the device uses it
        uint32_t b;
        uint64_t start;
        locate(v, lut.data(), lay.lut_shift, reg.data(), lay.n_regions, lay.nb, starts.data(), b, start);
        if (lay.est_ok) {
            uint32_t be;
            uint64_t se;
            locate_est(v, lay.est_mul, lay.est_shift, starts.data(), be, se);
            if (be != b || se != start) return fail(HOPH_E_UNSUPPORTED, "bin estimate and region lookup disagree");
        }
        if (narrow) {
            // the narrow lookups the device uses: the bin of the value's 32-bit view
            // and the offset of the value itself in 32-bit arithmetic
            uint32_t v32 = narrow_value(v);
            if (p.hash == HOPH_HASH_MODP32P15 && (p.hash_a >> 32) == 0 && (p.hash_b >> 32) == 0) {
                // the 32-bit form of the hash the device takes for such coefficients
                uint32_t view, low;
                psi_p32_narrow((uint32_t)x, (uint32_t)p.hash_a, (uint32_t)p.hash_b, view, low);
                const bool view_ok = v <= 0xFFFFFFFFull ? view == v32 : (view >= kNarrowLow && view <= kNarrowTop);
                if (low != (uint32_t)v || !view_ok)
                    return fail(HOPH_E_UNSUPPORTED, "32-bit and 64-bit forms of the hash disagree");
                v32 = view;
            }
            uint32_t bn, sn;
            locate_narrow(v32, lut.data(), lay.lut_shift, rs.data(), lay.reg_mag32.data(), lay.n_regions,
                          lay.nb, s32.data(), bn, sn);
            if (bn != b || (uint32_t)v - sn != (uint32_t)(v - start))
                return fail(HOPH_E_UNSUPPORTED, "narrow and wide bin lookups disagree");
            if (lay.est_ok) {
                const uint32_t e = bin_estimate(v32, lay.est_mul, lay.est_shift);
                const uint32_t be = e + (v32 >= s32[e + 1] ? 1u : 0u);
                if (be != b) return fail(HOPH_E_UNSUPPORTED, "narrow bin estimate and region lookup disagree");
            }
            if (lay.log_ok) {
                locate_log(v32, narrow_r1(lay.R), reinterpret_cast<const uint32_t(*)[2]>(cells.data()),
                           reinterpret_cast<const uint32_t(*)[2]>(regs.data()), lay.nb, s32.data(), bn, sn);
                if (bn != b || (uint32_t)v - sn != (uint32_t)(v - start))
                    return fail(HOPH_E_UNSUPPORTED, "log-cell and region lookups disagree");
            }
            if (lay.pow2_ok) {
                uint32_t bp, op;
                locate_pow2((uint32_t)v, (uint32_t)(lay.R - 1), reinterpret_cast<const uint32_t(*)[4]>(lay.pow2.data()),
                            bp, op);
                if (bp != b || op != (uint32_t)(v - start))
                    return fail(HOPH_E_UNSUPPORTED, "power-of-two and region lookups disagree");
            }
        }
        out_bin[i] = b;
        out_off[i] = (uint32_t)(v - start);
    }
    return HOPH_OK;
}

hoph_status hoph_pair_counts(const hoph_index *idx, const uint32_t *d_qsigs, uint32_t n_q, const uint32_t *d_pairs,
                             uint64_t n_pairs, uint32_t policy, uint32_t *d_m, uint32_t *d_e, void *hip_stream) {
    g_last_error.clear();
    if (!idx) return fail(HOPH_E_INVAL, "index is NULL");
    if (policy > HOPH_EMPTY_EITHER) return fail(HOPH_E_INVAL, "unknown empty policy");
    if (n_pairs == 0) return HOPH_OK;
    if (!d_qsigs || !d_pairs || !d_m || !d_e) return fail(HOPH_E_INVAL, "NULL device pointer");
    DeviceGuard dg(idx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    HOPH_HIP(launch_pair_counts(idx->slab, idx->capacity, idx->n, idx->kpad, idx->lay.kp, idx->lay.L, idx->lay.k,
                                d_qsigs, n_q, d_pairs, n_pairs, policy, d_m, d_e, s),
             "pair counts launch");
    HOPH_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    return HOPH_OK;
}

hoph_status hoph_self_join(const hoph_index *index, const hoph_query_params *qp, hoph_results *res,
                           void *hip_stream) {
    g_last_error.clear();
    if (!index) return fail(HOPH_E_INVAL, "index is NULL");
    const QueryKind kind = index->params.layout == HOPH_LAYOUT_OPH ? QueryKind::GOPH : QueryKind::HOPH;
    return run_query(index, nullptr, 0, qp, res, hip_stream, kind, true);
}

hoph_status hoph_pair_estimates(const hoph_index *idx, const uint32_t *d_qsigs, uint32_t n_q, const uint32_t *d_pairs,
                                uint64_t n_pairs, uint32_t policy, const double *d_unions, int64_t *d_est,
                                uint32_t *d_mb, uint32_t *d_eb, double *d_var, int64_t *denominator,
                                void *hip_stream) {
    g_last_error.clear();
    if (!idx) return fail(HOPH_E_INVAL, "index is NULL");
    if (policy > HOPH_EMPTY_EITHER) return fail(HOPH_E_INVAL, "unknown empty policy");
    hoph_query_params qp{};
    qp.T = hoph_ratio{1, 2};                      // the weights and rate scale do not depend on T or eps
    qp.eps = hoph_ratio{1, 2};
    qp.empty_policy = policy;
    hoph_decision_tables t;
    std::string err;
    hoph_status st = build_tables(idx->lay, qp, idx->params.layout == HOPH_LAYOUT_OPH, t, err);
    if (st) return fail(st, err);
    ScanTab tab{};
    to_scan_tab(t, tab);
    if (denominator) *denominator = (int64_t)t.wsum * tab.lambda;
    if (n_pairs == 0) return HOPH_OK;
    if (!d_qsigs || !d_pairs || !d_est || !d_mb || !d_eb || !d_var) return fail(HOPH_E_INVAL, "NULL device pointer");
    DeviceGuard dg(idx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    HOPH_HIP(launch_pair_estimates(idx->slab, idx->n, idx->lay.k, idx->lay.kp, idx->lay.L, d_qsigs, n_q, d_pairs,
                                   n_pairs, policy, d_unions, d_est, d_mb, d_eb, d_var, tab, s),
             "pair estimates launch");
    return HOPH_OK;
}

}  // extern "C"
