// Serving loop (hoph_server_*): continuous batching of single query sets over
// a resident index.  Each slot is a worker thread that owns a plan, a stream
// and pinned staging; a free worker takes the waiting requests in arrival
// order while they fit its batch, runs them as one batch, and answers each
// request with its own ascending result list.  Slots run concurrently, so the
// next batch is copied and sketched while the previous one is scanned.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace hoph;

namespace {

using Clock = std::chrono::steady_clock;
constexpr uint64_t kResultsPrefetch = 4096;   // result ids read back with the counters (16 KB)
// Under load (at least kGatherBusy other slots running a batch) a free worker
// waits up to kGatherUs for kGatherQueries requests before it starts: every
// batch re-reads the whole index's first-group codes, so a few larger batches
// serve more queries per second than many small ones.  With the device idle a
// request starts at once.
constexpr uint32_t kGatherBusy = 2;
constexpr size_t kGatherQueries = 64;
constexpr int kGatherUs = 200;

struct Request {
    uint64_t ticket = 0;
    std::vector<uint32_t> ids;
    Clock::time_point t_submit;
    std::vector<uint32_t> result;
    hoph_status status = HOPH_OK;
    bool done = false;
};

}  // namespace

struct hoph_server;

namespace {

struct Slot {
    hoph_plan *plan = nullptr;
    hipStream_t stream = nullptr;
    uint32_t *h_ids = nullptr, *d_ids = nullptr, *h_res_ids = nullptr;
    uint64_t *h_offs = nullptr, *d_offs = nullptr, *h_res_offs = nullptr;
    std::thread worker;
};

}  // namespace

struct hoph_server {
    hoph_index *idx = nullptr;
    hoph_sketch_params params{};
    hoph_query_params qp{};
    hoph_server_config cfg{};
    std::vector<std::unique_ptr<Slot>> slots;
    uint64_t slot_bytes = 0;
    // request queue and table
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> table;
    uint64_t next_ticket = 1;
    bool stop = false;
    uint32_t running = 0;            // slots running a batch
    // statistics
    std::vector<double> lat_ms;
    uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, batch_queries = 0, inserted = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;
    // inserts: grow-only device staging, so that an insert does not free
    // memory (which would wait for every batch in flight)
    std::mutex insert_mu;
    hipStream_t insert_stream = nullptr;
    // insert staging, allocated at creation (device and pinned host): inserts
    // larger than it go through in pieces, so no insert allocates
    uint32_t *ins_ids = nullptr, *h_ins_ids = nullptr;
    uint64_t *ins_offs = nullptr, *h_ins_offs = nullptr;
    uint64_t ins_ids_cap = 0, ins_sets_cap = 0;
};

namespace {

hoph_status run_batch(hoph_server *srv, Slot &sl, std::vector<std::shared_ptr<Request>> &batch) {
    // pack the request sets into pinned staging
    uint64_t n_ids = 0;
    sl.h_offs[0] = 0;
    for (size_t i = 0; i < batch.size(); ++i) {
        const auto &ids = batch[i]->ids;
        std::memcpy(sl.h_ids + n_ids, ids.data(), ids.size() * sizeof(uint32_t));
        n_ids += ids.size();
        sl.h_offs[i + 1] = n_ids;
    }
    const uint32_t n_q = (uint32_t)batch.size();
    HOPH_HIP(hipMemcpyAsync(sl.d_ids, sl.h_ids, std::max<uint64_t>(n_ids, 1) * 4, hipMemcpyHostToDevice, sl.stream),
             "stage request ids");
    HOPH_HIP(hipMemcpyAsync(sl.d_offs, sl.h_offs, ((uint64_t)n_q + 1) * 8, hipMemcpyHostToDevice, sl.stream),
             "stage request offsets");
    hoph_status st = hoph_plan_run(sl.plan, sl.d_ids, sl.d_offs, n_q, n_ids, sl.stream);
    if (st) return st;
    // counters, offsets and the first ids in one read-back (a second only for
    // a batch with more results, or one that fell back)
    uint64_t n_res = 0;
    st = plan_results_to_host(sl.plan, sl.h_res_offs, sl.h_res_ids, kResultsPrefetch, &n_res, sl.stream);
    if (st) return st;
    for (size_t i = 0; i < batch.size(); ++i)
        batch[i]->result.assign(sl.h_res_ids + sl.h_res_offs[i], sl.h_res_ids + sl.h_res_offs[i + 1]);
    return HOPH_OK;
}

void worker_loop(hoph_server *srv, Slot *sl) {
    DeviceGuard dg(srv->idx->device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv_work.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
            if (srv->stop && srv->queue.empty()) return;
            if (!srv->stop && srv->running >= kGatherBusy && srv->queue.size() < kGatherQueries) {
                srv->cv_work.wait_for(lk, std::chrono::microseconds(kGatherUs),
                                      [&] { return srv->stop || srv->queue.size() >= kGatherQueries; });
                if (srv->queue.empty()) continue;     // another worker took them
            }
            uint64_t ids = 0;
            while (!srv->queue.empty() && batch.size() < srv->cfg.max_batch_queries) {
                const auto &r = srv->queue.front();
                if (!batch.empty() && ids + r->ids.size() > srv->cfg.max_batch_ids) break;
                ids += r->ids.size();
                batch.push_back(r);
                srv->queue.pop_front();
            }
            ++srv->running;
        }
        const hoph_status st = run_batch(srv, *sl, batch);
        const auto now = Clock::now();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            --srv->running;
            for (auto &r : batch) {
                r->status = st;
                r->done = true;
                srv->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
            }
            srv->completed += batch.size();
            srv->batches += 1;
            srv->batch_queries += batch.size();
            srv->t_last = now;
        }
        srv->cv_done.notify_all();
    }
}

uint64_t plan_bytes(const hoph_index *idx, const hoph_server_config &c) {
    const uint64_t Q = c.max_batch_queries, k = idx->lay.k, L = idx->lay.L;
    const uint64_t surv = plan_survivor_capacity(idx->capacity, c.max_batch_queries);
    const uint64_t keys = sort_capacity(std::max<uint64_t>(c.max_batch_results, 1));
    return 4 * c.max_batch_ids + 8 * 4 * (Q + 1) + 4 * Q * k + 8 * Q * L + 4 * (Q + 1) * idx->cg * code_rec_words(idx->lay.kp) +
           16 * surv + 8 * keys + 4 * c.max_batch_results + 4 * (Q + 1) + 4 * c.max_batch_ids + 8 * (Q + 1);
}

void free_slot(Slot &s) {
    if (s.plan) hoph_plan_free(s.plan);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.d_ids) (void)hipFree(s.d_ids);
    if (s.d_offs) (void)hipFree(s.d_offs);
    if (s.h_ids) (void)hipHostFree(s.h_ids);
    if (s.h_offs) (void)hipHostFree(s.h_offs);
    if (s.h_res_ids) (void)hipHostFree(s.h_res_ids);
    if (s.h_res_offs) (void)hipHostFree(s.h_res_offs);
}

hoph_status fetch(hoph_server *srv, const std::shared_ptr<Request> &r, uint32_t *h_out, uint64_t cap,
                  uint64_t *n_out) {
    if (n_out) *n_out = r->result.size();
    if (r->status) return fail(r->status, "request failed");
    if (r->result.size() > cap) return fail(HOPH_E_CAPACITY, "output capacity too small");
    if (h_out && !r->result.empty()) std::memcpy(h_out, r->result.data(), r->result.size() * sizeof(uint32_t));
    srv->table.erase(r->ticket);
    return HOPH_OK;
}

hoph_status prime_slots(hoph_server *srv) {
    Slot &s0 = *srv->slots[0];
    if (srv->cfg.tune) {
        const uint32_t n_q = (uint32_t)std::min<uint64_t>(64, srv->cfg.max_batch_queries);
        const uint64_t per = std::max<uint64_t>(1, std::min<uint64_t>(800, srv->cfg.max_batch_ids / n_q));
        const uint64_t universe = std::max<uint64_t>(1, srv->params.universe);
        uint64_t x = 0x9E3779B97F4A7C15ull;
        for (uint32_t q = 0; q <= n_q; ++q) s0.h_offs[q] = (uint64_t)q * per;
        for (uint64_t i = 0; i < (uint64_t)n_q * per; ++i) {
            x = x * 6364136223846793005ull + 1442695040888963407ull;      // 64-bit LCG (Knuth's MMIX constants)
            s0.h_ids[i] = (uint32_t)((x >> 32) % universe);
        }
        HOPH_HIP(hipMemcpyAsync(s0.d_ids, s0.h_ids, (uint64_t)n_q * per * 4, hipMemcpyHostToDevice, s0.stream),
                 "prime ids");
        HOPH_HIP(hipMemcpyAsync(s0.d_offs, s0.h_offs, ((uint64_t)n_q + 1) * 8, hipMemcpyHostToDevice, s0.stream),
                 "prime offsets");
        hoph_status st = hoph_plan_run(s0.plan, s0.d_ids, s0.d_offs, n_q, (uint64_t)n_q * per, s0.stream);
        if (st) return st;
        uint64_t n_res = 0;
        st = plan_results_to_host(s0.plan, s0.h_res_offs, s0.h_res_ids, 0, &n_res, s0.stream);
        if (st && st != HOPH_E_CAPACITY) return st;          // the synthetic answers themselves are not needed
    } else {
        hoph_status st = plan_adopt_and_capture(s0.plan, nullptr);
        if (st) return st;
    }
    for (size_t i = 1; i < srv->slots.size(); ++i) {
        hoph_status st = plan_adopt_and_capture(srv->slots[i]->plan, srv->cfg.tune ? s0.plan : nullptr);
        if (st) return st;
    }
    clear_error();
    return HOPH_OK;
}

}  // namespace

extern "C" {

hoph_status hoph_server_create(hoph_index *idx, const hoph_sketch_params *params, const hoph_query_params *qp,
                               const hoph_server_config *cfg, hoph_server **out) {
    clear_error();
    if (!idx || !params || !qp || !cfg || !out) return fail(HOPH_E_INVAL, "NULL argument");
    *out = nullptr;
    if (cfg->slots == 0 || cfg->max_batch_queries == 0 || cfg->max_batch_ids == 0)
        return fail(HOPH_E_INVAL, "slots, max_batch_queries and max_batch_ids must be positive");
    std::unique_ptr<hoph_server> srv(new (std::nothrow) hoph_server());
    if (!srv) return fail(HOPH_E_NOMEM, "host allocation");
    srv->idx = idx;
    srv->params = *params;
    srv->qp = *qp;
    srv->cfg = *cfg;
    DeviceGuard dg(idx->device);
    srv->slot_bytes = plan_bytes(idx, *cfg);
    uint32_t n_slots = cfg->slots;
    if (cfg->device_mem_budget) {
        n_slots = (uint32_t)std::min<uint64_t>(n_slots, cfg->device_mem_budget / srv->slot_bytes);
        if (n_slots == 0) n_slots = 1;
    }
    hoph_plan_config pc{};
    pc.kind = cfg->kind;
    pc.max_queries = cfg->max_batch_queries;
    pc.max_query_ids = cfg->max_batch_ids;
    pc.max_results = cfg->max_batch_results;
    pc.use_graph = cfg->use_graph;
    pc.tune = cfg->tune;
    const uint64_t Q = cfg->max_batch_queries;
    for (uint32_t i = 0; i < n_slots; ++i) {
        auto sl = std::make_unique<Slot>();
        hoph_status st = hoph_plan_create(idx, params, qp, &pc, &sl->plan);
        bool ok = st == HOPH_OK && hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess &&
                  hipMalloc(&sl->d_ids, cfg->max_batch_ids * 4) == hipSuccess &&
                  hipMalloc(&sl->d_offs, (Q + 1) * 8) == hipSuccess &&
                  hipHostMalloc(&sl->h_ids, cfg->max_batch_ids * 4, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&sl->h_offs, (Q + 1) * 8, hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&sl->h_res_ids, std::max<uint64_t>(cfg->max_batch_results, 1) * 4,
                                hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc(&sl->h_res_offs, (Q + 1) * 8, hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            free_slot(*sl);
            for (auto &s : srv->slots) free_slot(*s);
            return st ? st : fail(HOPH_E_NOMEM, "server slot allocation");
        }
        srv->slots.push_back(std::move(sl));
    }
    if (hipStreamCreateWithFlags(&srv->insert_stream, hipStreamNonBlocking) != hipSuccess) {
        for (auto &s : srv->slots) free_slot(*s);
        return fail(HOPH_E_DEVICE, "hipStreamCreate");
    }
    // insert staging: one slot's ids (at least 2^20) and 65,536 sets per piece
    srv->ins_ids_cap = std::max<uint64_t>(cfg->max_batch_ids, 1u << 20);
    srv->ins_sets_cap = 65536;
    if (hipMalloc(&srv->ins_ids, srv->ins_ids_cap * 4) != hipSuccess ||
        hipMalloc(&srv->ins_offs, (srv->ins_sets_cap + 1) * 8) != hipSuccess ||
        hipHostMalloc(&srv->h_ins_ids, srv->ins_ids_cap * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&srv->h_ins_offs, (srv->ins_sets_cap + 1) * 8, hipHostMallocDefault) != hipSuccess) {
        for (auto &s : srv->slots) free_slot(*s);
        (void)hipStreamDestroy(srv->insert_stream);
        if (srv->ins_ids) (void)hipFree(srv->ins_ids);
        if (srv->ins_offs) (void)hipFree(srv->ins_offs);
        if (srv->h_ins_ids) (void)hipHostFree(srv->h_ins_ids);
        if (srv->h_ins_offs) (void)hipHostFree(srv->h_ins_offs);
        return fail(HOPH_E_NOMEM, "insert staging");
    }
    // Every slot ready before the first request: with tuning, one synthetic batch
    // (up to 64 query sets of up to 800 pseudo-random ids) through the first slot
    // times the tile shapes; every other slot takes them and captures its graph
    // now, so no request waits for a slot's tuning or graph capture.
    hoph_status pst = prime_slots(srv.get());
    if (pst) {
        for (auto &s : srv->slots) free_slot(*s);
        (void)hipStreamDestroy(srv->insert_stream);
        (void)hipFree(srv->ins_ids);
        (void)hipFree(srv->ins_offs);
        (void)hipHostFree(srv->h_ins_ids);
        (void)hipHostFree(srv->h_ins_offs);
        return pst;
    }
    hoph_server *raw = srv.get();
    for (auto &s : srv->slots) s->worker = std::thread(worker_loop, raw, s.get());
    *out = srv.release();
    return HOPH_OK;
}

hoph_status hoph_server_submit(hoph_server *srv, const uint32_t *h_ids, uint64_t n_ids, uint64_t *ticket) {
    clear_error();
    if (!srv || !ticket || (n_ids && !h_ids)) return fail(HOPH_E_INVAL, "NULL argument");
    auto r = std::make_shared<Request>();
    r->ids.assign(h_ids, h_ids + n_ids);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (!srv->have_first) {
            srv->have_first = true;
            srv->t_first = r->t_submit;
        }
        ++srv->submitted;
        if (n_ids > srv->cfg.max_batch_ids || n_ids == 0) {
            ++srv->rejected;
            *ticket = 0;
            return fail(n_ids ? HOPH_E_CAPACITY : HOPH_E_INVAL,
                        n_ids ? "query set larger than a batch" : "empty query set");
        }
        r->ticket = srv->next_ticket++;
        *ticket = r->ticket;
        srv->table[r->ticket] = r;
        srv->queue.push_back(r);
    }
    srv->cv_work.notify_one();
    return HOPH_OK;
}

hoph_status hoph_server_wait(hoph_server *srv, uint64_t ticket, uint32_t *h_out, uint64_t cap, uint64_t *n_out) {
    clear_error();
    if (!srv) return fail(HOPH_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->table.find(ticket);
    if (it == srv->table.end()) return fail(HOPH_E_INVAL, "unknown ticket");
    auto r = it->second;
    srv->cv_done.wait(lk, [&] { return r->done; });
    return fetch(srv, r, h_out, cap, n_out);
}

hoph_status hoph_server_poll(hoph_server *srv, uint64_t ticket, int32_t *done, uint32_t *h_out, uint64_t cap,
                             uint64_t *n_out) {
    clear_error();
    if (!srv || !done) return fail(HOPH_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->table.find(ticket);
    if (it == srv->table.end()) return fail(HOPH_E_INVAL, "unknown ticket");
    *done = it->second->done ? 1 : 0;
    if (!*done) return HOPH_OK;
    return fetch(srv, it->second, h_out, cap, n_out);
}

hoph_status hoph_server_insert(hoph_server *srv, const uint32_t *h_ids, const uint64_t *h_offsets, uint64_t n_sets) {
    clear_error();
    if (!srv || (n_sets && (!h_ids || !h_offsets))) return fail(HOPH_E_INVAL, "NULL argument");
    if (n_sets == 0) return HOPH_OK;
    std::lock_guard<std::mutex> ilk(srv->insert_mu);
    hoph_index *idx = srv->idx;
    DeviceGuard dg(idx->device);
    {
        std::lock_guard<std::mutex> lk(idx->mu);
        if (idx->n + n_sets > idx->max_sets) return fail(HOPH_E_CAPACITY, "index capacity exceeded");
    }
    // the offsets are on the host: a decreasing pair would make the device read
    // a range that wraps past the staged ids; a set larger than the staging
    // cannot be sketched in one piece
    for (uint64_t i = 0; i < n_sets; ++i) {
        if (h_offsets[i + 1] < h_offsets[i]) return fail(HOPH_E_INVAL, "insert offsets decrease");
        if (h_offsets[i + 1] - h_offsets[i] > srv->ins_ids_cap)
            return fail(HOPH_E_CAPACITY, "an inserted set has more ids than the insert staging holds (" +
                                             std::to_string(srv->ins_ids_cap) + ")");
    }
    uint32_t *errw = nullptr;
    hoph_status es = device_err_word(&errw);
    if (es) return es;
    hipStream_t st = srv->insert_stream;
    // pieces of at most ins_sets_cap sets and ins_ids_cap ids, each sketched into
    // rows [first, first + m) and then made visible
    for (uint64_t a = 0; a < n_sets;) {
        uint64_t b = a;
        while (b < n_sets && b - a < srv->ins_sets_cap && h_offsets[b + 1] - h_offsets[a] <= srv->ins_ids_cap) ++b;
        const uint64_t m = b - a, nnz = h_offsets[b] - h_offsets[a];
        std::memcpy(srv->h_ins_ids, h_ids + h_offsets[a], nnz * 4);
        for (uint64_t i = 0; i <= m; ++i) srv->h_ins_offs[i] = h_offsets[a + i] - h_offsets[a];
        hoph_status s = HOPH_OK;
        if (hipMemcpyAsync(srv->ins_ids, srv->h_ins_ids, nnz * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(srv->ins_offs, srv->h_ins_offs, (m + 1) * 8, hipMemcpyHostToDevice, st) != hipSuccess)
            s = fail(HOPH_E_DEVICE, "insert copy");
        uint64_t first = 0;
        if (!s) {
            std::lock_guard<std::mutex> lk(idx->mu);
            first = idx->n;
        }
        // batches dispatched meanwhile read only rows below idx->n
        if (!s && append_sets_async(idx, srv->ins_ids, srv->ins_offs, m, first, errw, st, false) != hipSuccess)
            s = fail(HOPH_E_DEVICE, "sketch-into-index launch");
        if (!s && hipStreamSynchronize(st) != hipSuccess) s = fail(HOPH_E_DEVICE, "hipStreamSynchronize");
        if (s) return s;
        {
            // visible to batches dispatched from now on; batches in flight keep their snapshot
            std::lock_guard<std::mutex> lk(idx->mu);
            idx->n = first + m;
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->inserted += m;
        }
        a = b;
    }
    return HOPH_OK;
}

hoph_status hoph_server_replay(hoph_server *srv, const uint32_t *h_ids, const uint64_t *h_offsets, uint64_t n,
                               const double *arrival_s, uint64_t *result_offsets, uint32_t *result_ids,
                               uint64_t result_cap) {
    clear_error();
    if (!srv || (n && (!h_ids || !h_offsets || !arrival_s))) return fail(HOPH_E_INVAL, "NULL argument");
    std::vector<uint64_t> tickets(n, 0);
    const auto t0 = Clock::now();
    for (uint64_t i = 0; i < n; ++i) {
        const auto due = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
        while (Clock::now() < due) {
            const auto left = due - Clock::now();
            if (left > std::chrono::microseconds(200)) std::this_thread::sleep_for(left - std::chrono::microseconds(100));
        }
        uint64_t t = 0;
        hoph_status st = hoph_server_submit(srv, h_ids + h_offsets[i], h_offsets[i + 1] - h_offsets[i], &t);
        if (st && st != HOPH_E_CAPACITY) return st;
        tickets[i] = t;
    }
    hoph_status result = HOPH_OK;
    uint64_t pos = 0;
    if (result_offsets) result_offsets[0] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (!tickets[i]) {
            if (result_offsets) result_offsets[i + 1] = pos;
            continue;
        }
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->table.find(tickets[i]);
        if (it == srv->table.end()) continue;
        auto r = it->second;
        srv->cv_done.wait(lk, [&] { return r->done; });
        if (r->status && !result) result = r->status;
        if (result_offsets) {
            if (pos + r->result.size() > result_cap) {
                result = HOPH_E_CAPACITY;
            } else if (result_ids && !r->result.empty()) {
                std::memcpy(result_ids + pos, r->result.data(), r->result.size() * 4);
            }
            pos += r->result.size();
            result_offsets[i + 1] = pos;
        }
        srv->table.erase(tickets[i]);
    }
    if (result) return fail(result, result == HOPH_E_CAPACITY ? "result capacity too small" : "a request failed");
    return HOPH_OK;
}

hoph_status hoph_server_stats_get(hoph_server *srv, hoph_server_stats *out) {
    clear_error();
    if (!srv || !out) return fail(HOPH_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->batches = srv->batches;
    out->inserted_sets = srv->inserted;
    out->slots = (uint32_t)srv->slots.size();
    out->slot_bytes = srv->slot_bytes;
    for (auto &s : srv->slots) {
        hoph_plan_info info;
        if (hoph_plan_get_info(s->plan, &info) == HOPH_OK) out->fallbacks += info.fallbacks;
    }
    if (!srv->lat_ms.empty()) {
        std::vector<double> v = srv->lat_ms;
        std::sort(v.begin(), v.end());
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / v.size();
        out->p50_ms = v[(v.size() - 1) / 2];
        out->p99_ms = v[std::min<size_t>(v.size() - 1, (size_t)(0.99 * (v.size() - 1) + 0.5))];
        out->max_ms = v.back();
    }
    if (srv->batches) out->mean_batch_queries = (double)srv->batch_queries / srv->batches;
    if (srv->have_first && srv->completed)
        out->busy_s = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
    return HOPH_OK;
}

hoph_status hoph_server_reset_stats(hoph_server *srv) {
    clear_error();
    if (!srv) return fail(HOPH_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->lat_ms.clear();
    srv->submitted = srv->completed = srv->rejected = srv->batches = srv->batch_queries = 0;
    srv->have_first = false;
    return HOPH_OK;
}

void hoph_server_destroy(hoph_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &s : srv->slots)
        if (s->worker.joinable()) s->worker.join();
    {
        DeviceGuard dg(srv->idx->device);
        for (auto &s : srv->slots) free_slot(*s);
        if (srv->insert_stream) (void)hipStreamDestroy(srv->insert_stream);
        if (srv->ins_ids) (void)hipFree(srv->ins_ids);
        if (srv->ins_offs) (void)hipFree(srv->ins_offs);
        if (srv->h_ins_ids) (void)hipHostFree(srv->h_ins_ids);
        if (srv->h_ins_offs) (void)hipHostFree(srv->h_ins_offs);
    }
    delete srv;
}

}  // extern "C"
