// Serving loop: solve requests (level, tolerance, grid and right-hand-side
// seeds) arrive at any time; a scheduler thread admits them in arrival order
// into free slots of a BatchEngine while the device-memory budget allows,
// builds each request's problem on the device (jittered geometry, assembly,
// uniform right-hand side) in a resident hierarchy of its level, and
// advances all live requests together one graph-replayed iteration at a
// time.  Requests that arrive while others run join at the next iteration
// (continuous batching); finished ones leave their slot at once.  The
// device always has the next iteration queued while the scheduler handles
// the report of the previous one, so host work does not idle the GPU.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"

namespace mg {
double mixed_solve_bytes(int L, int Lc, int nu_pre, int nu_post, const BState& S);
void fill_stats(const BState& S, int L, int Lc, int nu_pre, int nu_post, mg_stats* st);
}  // namespace mg

using namespace mg;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    uint64_t ticket;
    int L;
    double tol;
    double jitter;
    uint64_t geom_seed, rhs_seed;
    int keep_x;
    Clock::time_point t_submit, t_admit;
};

struct Result {
    mg_stats stats;
    std::vector<double> x;
};

double secs(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
}

}  // namespace

struct mg_server {
    mg_context* ctx = nullptr;
    int Lmax = 11, Lc = 1;
    size_t budget = 0;
    size_t bytes = 0;        // hierarchies owned (pool + live)
    size_t high_water = 0;
    mg_solve_opts opts{};
    BatchEngine eng;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    mg_status fatal = MG_OK;
    std::string fatal_msg;
    uint64_t next_ticket = 1;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Result> done;   // finished, not yet collected
    std::deque<uint64_t> done_order;
    std::unordered_map<uint64_t, int> pending;   // submitted, not finished
    // worker-owned
    std::vector<Request> slot_req;
    std::vector<mg_hierarchy*> slot_h;
    std::multimap<int, mg_hierarchy*> pool;      // idle hierarchies by level
    std::deque<mg_hierarchy*> pool_lru;
    std::vector<int64_t> slot_first;             // first iteration that sees the slot's problem
    int live = 0;
    bool dirty = false;                          // slots changed since the last upload
    uint64_t completed = 0;
    size_t queue_high = 0;
    double busy_seconds = 0.0;

    void run();
    bool complete(int s);
    mg_hierarchy* take_hierarchy(int L);
    void release_hierarchy(mg_hierarchy* h);
    bool admit_one(int slot, const Request& r);
    void set_fatal(mg_status s, const std::string& m) {
        std::lock_guard<std::mutex> g(mu);
        fatal = s;
        fatal_msg = m;
        stop = true;
        cv_done.notify_all();
    }
};

// A resident hierarchy of level L: from the idle pool, or newly allocated
// within the server budget (evicting idle hierarchies of other levels, least
// recently used first, when that makes room).  nullptr when it does not fit.
mg_hierarchy* mg_server::take_hierarchy(int L) {
    auto it = pool.find(L);
    if (it != pool.end()) {
        mg_hierarchy* h = it->second;
        pool.erase(it);
        for (auto q = pool_lru.begin(); q != pool_lru.end(); ++q)
            if (*q == h) {
                pool_lru.erase(q);
                break;
            }
        return h;
    }
    const size_t need = mg_hierarchy_bytes(L, Lc);
    while (bytes + need > budget && !pool_lru.empty()) {
        mg_hierarchy* v = pool_lru.front();
        pool_lru.pop_front();
        for (auto q = pool.begin(); q != pool.end(); ++q)
            if (q->second == v) {
                pool.erase(q);
                break;
            }
        bytes -= v->charged;
        mg_hierarchy_destroy(v);
    }
    if (bytes + need > budget) return nullptr;
    mg_hierarchy* h = nullptr;
    if (mg_hierarchy_create(ctx, L, Lc, 0.0, 0, nullptr, &h) != MG_OK) return nullptr;
    bytes += h->charged;
    high_water = std::max(high_water, bytes);
    return h;
}

void mg_server::release_hierarchy(mg_hierarchy* h) {
    pool.emplace(h->L, h);
    pool_lru.push_back(h);
}

// Build the request's problem in a resident hierarchy and start it in slot.
bool mg_server::admit_one(int slot, const Request& r) {
    mg_hierarchy* h = take_hierarchy(r.L);
    if (!h) return false;
    hipStream_t st = eng.setup_stream();
    const Level& F = h->lv[r.L];
    hipError_t e = launch_coords_rhs(h->coords, r.L, r.jitter, r.geom_seed, r.rhs_seed, h->dmask,
                                     F.b64, F.x64, st);
    if (e == hipSuccess) e = launch_assemble(h->coords, h->lv, Lc, r.L, h->dmask, st);
    if (e == hipSuccess) e = launch_chol_factor(h->lv[Lc], h->dmask, h->chol, h->flag, st);
    if (e != hipSuccess) {
        release_hierarchy(h);
        set_fatal(MG_ERR_DEVICE, std::string("admission: ") + hipGetErrorString(e));
        return false;
    }
    h->assembled = true;
    mg_solve_opts o = opts;
    o.rel_tol = r.tol;
    eng.set_slot(slot, h, o);
    eng.start_slot(slot);
    slot_req[slot] = r;
    slot_req[slot].t_admit = Clock::now();
    slot_h[slot] = h;
    slot_first[slot] = eng.launched();  // the upload precedes the next launch
    ++live;
    dirty = true;
    return true;
}

// Deliver the finished problem of slot s and free the slot.
bool mg_server::complete(int s) {
    mg_hierarchy* h = slot_h[s];
    const Request& r = slot_req[s];
    Result res;
    BState S;
    if (eng.fetch_state(s, &S) != MG_OK) return false;
    fill_stats(S, h->L, Lc, opts.nu_pre, opts.nu_post, &res.stats);
    if (r.keep_x) {
        res.x.resize(h->lv[h->L].n);
        if (eng.fetch(h->lv[h->L].x64, res.x.data(), res.x.size() * sizeof(double)) != MG_OK)
            return false;
    }
    const auto now = Clock::now();
    res.stats.seconds = secs(r.t_submit, now);
    res.stats.queue_seconds = secs(r.t_submit, r.t_admit);
    eng.clear_slot(s);
    release_hierarchy(h);
    slot_h[s] = nullptr;
    --live;
    dirty = true;
    std::lock_guard<std::mutex> g(mu);
    pending.erase(r.ticket);
    done.emplace(r.ticket, std::move(res));
    done_order.push_back(r.ticket);
    ++completed;
    cv_done.notify_all();
    return true;
}

void mg_server::run() {
    (void)hipSetDevice(ctx->device);
    int64_t next = eng.launched();  // oldest iteration not yet reported
    Clock::time_point t_busy{};
    for (;;) {
        {
            std::unique_lock<std::mutex> g(mu);
            const bool idle = live == 0 && next == eng.launched();
            if (idle) cv_work.wait(g, [&] { return stop || !queue.empty(); });
            if (stop && queue.empty() && live == 0 && next == eng.launched()) return;
            // admit in arrival order while a slot and memory are available
            while (!queue.empty()) {
                int slot = -1;
                for (int s = 0; s < eng.capacity(); ++s)
                    if (!slot_h[s]) {
                        slot = s;
                        break;
                    }
                if (slot < 0) break;
                Request r = queue.front();
                g.unlock();
                const bool ok = admit_one(slot, r);
                g.lock();
                if (!ok) {
                    if (fatal != MG_OK) return;
                    if (live == 0 && next == eng.launched()) {
                        // cannot fit even alone: fail the request cleanly
                        queue.pop_front();
                        pending.erase(r.ticket);
                        Result res{};
                        res.stats.status = MG_ERR_NOMEM;
                        res.stats.seconds = secs(r.t_submit, Clock::now());
                        done.emplace(r.ticket, std::move(res));
                        done_order.push_back(r.ticket);
                        cv_done.notify_all();
                        continue;
                    }
                    break;  // wait for running requests to free memory
                }
                queue.pop_front();
            }
        }
        if (dirty) {
            if (eng.upload_async() != MG_OK) {
                set_fatal(MG_ERR_DEVICE, mg_last_error());
                return;
            }
            dirty = false;
        }
        // keep two iterations in flight while problems are live
        if (live > 0 && eng.launched() - next < 2) {
            if (next == eng.launched()) t_busy = Clock::now();
            if (eng.launch_iteration() != MG_OK) {
                set_fatal(MG_ERR_DEVICE, mg_last_error());
                return;
            }
            if (eng.launched() - next < 2) continue;  // queue the second one first
        }
        if (next == eng.launched()) continue;
        int nlive = 0, sure = 0;
        const int* flags = nullptr;
        if (eng.wait_iteration(next, &nlive, &sure, &flags) != MG_OK) {
            set_fatal(MG_ERR_DEVICE, mg_last_error());
            return;
        }
        const int64_t k = next++;
        if (next == eng.launched()) busy_seconds += secs(t_busy, Clock::now());
        for (int s = 0; s < eng.capacity(); ++s) {
            if (!slot_h[s] || slot_first[s] > k || !(flags[s] & BF_DONE)) continue;
            if (!complete(s)) {
                set_fatal(MG_ERR_DEVICE, "result copy failed");
                return;
            }
        }
    }
}

extern "C" {

mg_status mg_server_create(mg_context* ctx, int slots, size_t budget, int max_level,
                           int coarse_level, const mg_solve_opts* opts, mg_server** out) {
    if (!out) return fail(MG_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!ctx) return fail(MG_ERR_INVALID, "null context");
    if (slots < 1 || slots > 4096) return fail(MG_ERR_INVALID, "slots must be in [1, 4096]");
    if (max_level < 1 || max_level > MG_MAX_LEVEL || coarse_level < 1 ||
        coarse_level > std::min(max_level, MG_MAX_COARSE_LEVEL))
        return fail(MG_ERR_INVALID, "invalid level range");
    if (budget == 0) return fail(MG_ERR_INVALID, "the server needs a memory budget");
    mg_server* s = new (std::nothrow) mg_server();
    if (!s) return fail(MG_ERR_NOMEM, "host allocation failed");
    s->ctx = ctx;
    s->Lmax = max_level;
    s->Lc = coarse_level;
    s->budget = budget;
    if (opts)
        s->opts = *opts;
    else
        mg_default_opts(&s->opts);
    s->opts.precision = MG_PREC_MIXED;
    s->opts.krylov = 0;
    if (mg_status st = s->eng.init(ctx->device, slots, max_level, coarse_level, s->opts.nu_pre,
                                   s->opts.nu_post)) {
        delete s;
        return st;
    }
    s->slot_req.resize(slots);
    s->slot_h.assign(slots, nullptr);
    s->slot_first.assign(slots, 0);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return MG_OK;
}

mg_status mg_server_submit(mg_server* s, int L, double rel_tol, double jitter, uint64_t geom_seed,
                           uint64_t rhs_seed, int keep_x, uint64_t* ticket) {
    if (!s || !ticket) return fail(MG_ERR_INVALID, "null server or ticket");
    if (L < s->Lc || L > s->Lmax) return fail(MG_ERR_INVALID, "level outside the server's range");
    if (!(rel_tol >= 0.0) || !(jitter >= 0.0 && jitter < 0.5))
        return fail(MG_ERR_INVALID, "invalid tolerance or jitter");
    if (mg_hierarchy_bytes(L, s->Lc) > s->budget)
        return fail(MG_ERR_NOMEM, "request larger than the server budget");
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal != MG_OK) return fail(s->fatal, s->fatal_msg);
    if (s->stop) return fail(MG_ERR_INVALID, "server is shutting down");
    Request r{};
    r.ticket = s->next_ticket++;
    r.L = L;
    r.tol = rel_tol;
    r.jitter = jitter;
    r.geom_seed = geom_seed;
    r.rhs_seed = rhs_seed;
    r.keep_x = keep_x;
    r.t_submit = Clock::now();
    s->queue.push_back(r);
    s->queue_high = std::max(s->queue_high, s->queue.size());
    s->pending.emplace(r.ticket, L);
    *ticket = r.ticket;
    s->cv_work.notify_one();
    return MG_OK;
}

static mg_status collect(mg_server* s, uint64_t t, double* host_x, mg_stats* st) {
    auto it = s->done.find(t);
    Result& r = it->second;
    if (host_x && !r.x.empty()) std::memcpy(host_x, r.x.data(), r.x.size() * sizeof(double));
    if (st) *st = r.stats;
    const mg_status status = r.stats.status;
    s->done.erase(it);
    for (auto q = s->done_order.begin(); q != s->done_order.end(); ++q)
        if (*q == t) {
            s->done_order.erase(q);
            break;
        }
    return status;
}

mg_status mg_server_poll(mg_server* s, uint64_t ticket, double* host_x, mg_stats* st) {
    if (!s) return fail(MG_ERR_INVALID, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    if (s->done.count(ticket)) return collect(s, ticket, host_x, st);
    if (s->pending.count(ticket)) {
        if (s->fatal != MG_OK) return fail(s->fatal, s->fatal_msg);
        return MG_ERR_BUSY;
    }
    return fail(MG_ERR_INVALID, "unknown or already collected ticket");
}

mg_status mg_server_next(mg_server* s, double timeout_s, uint64_t* ticket, double* host_x,
                         mg_stats* st) {
    if (!s || !ticket) return fail(MG_ERR_INVALID, "null server or ticket");
    std::unique_lock<std::mutex> g(s->mu);
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                          std::chrono::duration<double>(timeout_s));
    s->cv_done.wait_until(g, until, [&] { return !s->done_order.empty() || s->fatal != MG_OK; });
    if (s->done_order.empty()) {
        if (s->fatal != MG_OK) return fail(s->fatal, s->fatal_msg);
        return MG_ERR_BUSY;
    }
    const uint64_t t = s->done_order.front();
    *ticket = t;
    return collect(s, t, host_x, st);
}

mg_status mg_server_info(mg_server* s, mg_server_info_t* info) {
    if (!s || !info) return fail(MG_ERR_INVALID, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    info->completed = s->completed;
    info->queued = s->queue.size();
    info->live = s->live;
    info->queue_high_water = s->queue_high;
    info->bytes = s->bytes;
    info->bytes_high_water = s->high_water;
    info->busy_seconds = s->busy_seconds;
    return MG_OK;
}

mg_status mg_server_destroy(mg_server* s) {
    if (!s) return fail(MG_ERR_INVALID, "null server");
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->pool) mg_hierarchy_destroy(kv.second);
    for (mg_hierarchy* h : s->slot_h)
        if (h) mg_hierarchy_destroy(h);
    delete s;
    return MG_OK;
}

}  // extern "C"
