// Continuous-batching scheduler of the solve server, independent of the
// device: requests are admitted in arrival order into free slots while
// their hierarchy fits a memory budget (device memory is a hard limit,
// Sec. 4.2), idle hierarchies are kept in a pool per level and evicted
// least recently used, two iterations are kept in flight while problems are
// live, and finished problems leave their slot at once.  The device side is
// an Executor: the HIP server supplies one backed by the batch engine, the
// CPU tests a fake one with a simulated clock.  Header only, plain C++17
// (no HIP), so the same code runs under the host sanitizers.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mgfem.h"

namespace mg {

struct SchedRequest {
    uint64_t ticket = 0;
    int L = 0;
    double tol = 0.0;
    double jitter = 0.0;
    uint64_t geom_seed = 0, rhs_seed = 0;
    int keep_x = 0;
    double t_submit = 0.0, t_admit = 0.0;  // executor clock, seconds
};

struct SchedResult {
    mg_stats stats{};
    std::vector<double> x;
};

// What the scheduler needs from the device side.  Every call except now()
// comes from the scheduler's worker thread; now() also from submitters.
class Executor {
public:
    virtual ~Executor() = default;
    virtual double now() = 0;  // seconds, monotone
    virtual int capacity() const = 0;  // slots
    // Memory a hierarchy of level L takes (charged against the budget).
    virtual size_t hierarchy_bytes(int L) const = 0;
    // A new hierarchy of level L, or nullptr when the device cannot provide
    // it (the scheduler has already checked the budget).
    virtual void* create_hierarchy(int L) = 0;
    virtual void destroy_hierarchy(void* h) = 0;
    // Build r's problem in hierarchy h and start it in the (free) slot; it
    // joins the iterations launched after the next upload().
    virtual mg_status admit(int slot, void* h, const SchedRequest& r) = 0;
    virtual mg_status upload() = 0;
    virtual mg_status launch_iteration() = 0;
    virtual int64_t launched() const = 0;  // iterations launched so far
    // Wait for iteration k (k < launched()); done[s] != 0 for every slot
    // whose problem had finished by its end (valid until the next call).
    virtual mg_status wait_iteration(int64_t k, const int** done) = 0;
    // Collect the finished problem of slot s (stats and, with keep_x, the
    // solution) and free the slot.
    virtual mg_status finish(int slot, void* h, int keep_x, SchedResult* out) = 0;
    // Text of the last failure of a call above (from the worker thread).
    virtual std::string error_message() { return std::string(); }
};

class Scheduler {
public:
    // budget: bytes of hierarchies held at once (live and idle).
    Scheduler(Executor* ex, size_t budget) : ex_(ex), budget_(budget) {
        const int cap = ex_->capacity();
        slot_req_.resize(cap);
        slot_h_.assign(cap, nullptr);
        slot_first_.assign(cap, 0);
    }
    ~Scheduler() { shutdown(); }
    Scheduler(const Scheduler&) = delete;
    Scheduler& operator=(const Scheduler&) = delete;

    void start() { worker_ = std::thread([this] { run(); }); }

    // Queue a request (never waits for the device).  The caller has
    // validated its arguments against the server's limits.
    mg_status submit(int L, double tol, double jitter, uint64_t geom_seed, uint64_t rhs_seed,
                     int keep_x, uint64_t* ticket, std::string* err) {
        if (ex_->hierarchy_bytes(L) > budget_) {
            if (err) *err = "request larger than the server budget";
            return MG_ERR_NOMEM;
        }
        std::lock_guard<std::mutex> g(mu_);
        if (fatal_ != MG_OK) {
            if (err) *err = fatal_msg_;
            return fatal_;
        }
        if (stop_) {
            if (err) *err = "server is shutting down";
            return MG_ERR_INVALID;
        }
        SchedRequest r;
        r.ticket = next_ticket_++;
        r.L = L;
        r.tol = tol;
        r.jitter = jitter;
        r.geom_seed = geom_seed;
        r.rhs_seed = rhs_seed;
        r.keep_x = keep_x;
        r.t_submit = ex_->now();
        queue_.push_back(r);
        queue_high_ = std::max(queue_high_, queue_.size());
        pending_.emplace(r.ticket, L);
        *ticket = r.ticket;
        cv_work_.notify_one();
        return MG_OK;
    }

    // MG_ERR_BUSY while pending; else the request's status and results.
    mg_status poll(uint64_t ticket, double* host_x, mg_stats* st, std::string* err) {
        std::lock_guard<std::mutex> g(mu_);
        if (done_.count(ticket)) return collect(ticket, host_x, st);
        if (pending_.count(ticket)) {
            if (fatal_ != MG_OK) {
                if (err) *err = fatal_msg_;
                return fatal_;
            }
            return MG_ERR_BUSY;
        }
        if (err) *err = "unknown or already collected ticket";
        return MG_ERR_INVALID;
    }

    // The oldest finished request, waiting up to timeout_s.
    mg_status next(double timeout_s, uint64_t* ticket, double* host_x, mg_stats* st,
                   std::string* err) {
        std::unique_lock<std::mutex> g(mu_);
        const auto until = std::chrono::steady_clock::now() +
                           std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                               std::chrono::duration<double>(timeout_s));
        cv_done_.wait_until(g, until, [&] { return !done_order_.empty() || fatal_ != MG_OK; });
        if (done_order_.empty()) {
            if (fatal_ != MG_OK) {
                if (err) *err = fatal_msg_;
                return fatal_;
            }
            return MG_ERR_BUSY;
        }
        const uint64_t t = done_order_.front();
        *ticket = t;
        return collect(t, host_x, st);
    }

    void info(mg_server_info_t* info) {
        std::lock_guard<std::mutex> g(mu_);
        info->completed = completed_;
        info->queued = queue_.size();
        info->live = live_.load();
        info->queue_high_water = queue_high_;
        info->bytes = bytes_.load();
        info->bytes_high_water = high_water_.load();
        info->busy_seconds = busy_seconds_.load();
    }

    // Finish every queued and running request, stop the worker and destroy
    // the idle hierarchies.  Idempotent.
    void shutdown() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
            cv_work_.notify_all();
        }
        if (worker_.joinable()) worker_.join();
        for (PoolEntry& e : pool_) ex_->destroy_hierarchy(e.h);
        pool_.clear();
        for (size_t s = 0; s < slot_h_.size(); ++s)
            if (slot_h_[s]) {
                ex_->destroy_hierarchy(slot_h_[s]);
                slot_h_[s] = nullptr;
            }
    }

private:
    struct PoolEntry {
        void* h;
        int L;
        size_t bytes;
    };

    // A hierarchy of level L: an idle one of that level, or a new one within
    // the budget, evicting idle hierarchies of other levels (least recently
    // used first) only when that makes room.  nullptr when it does not fit.
    void* take_hierarchy(int L) {
        for (auto it = pool_.begin(); it != pool_.end(); ++it)
            if (it->L == L) {
                void* h = it->h;
                pool_.erase(it);
                return h;
            }
        const size_t need = ex_->hierarchy_bytes(L);
        size_t idle = 0;
        for (const PoolEntry& e : pool_) idle += e.bytes;
        if (bytes_.load() - idle + need > budget_) return nullptr;
        while (bytes_.load() + need > budget_ && !pool_.empty()) {
            PoolEntry v = pool_.front();
            pool_.pop_front();
            bytes_ -= v.bytes;
            ex_->destroy_hierarchy(v.h);
        }
        void* h = ex_->create_hierarchy(L);
        if (!h) return nullptr;
        bytes_ += need;
        if (bytes_.load() > high_water_.load()) high_water_.store(bytes_.load());  // one writer
        return h;
    }

    void release_hierarchy(void* h, int L) {
        pool_.push_back({h, L, ex_->hierarchy_bytes(L)});
    }

    void set_fatal(mg_status s, const std::string& m) {
        std::lock_guard<std::mutex> g(mu_);
        fatal_ = s;
        fatal_msg_ = m;
        stop_ = true;
        cv_done_.notify_all();
    }

    // 1: admitted; 0: no memory now; -1: executor failure (fatal set).
    int admit_one(int slot, const SchedRequest& r) {
        void* h = take_hierarchy(r.L);
        if (!h) return 0;
        if (mg_status s = ex_->admit(slot, h, r)) {
            release_hierarchy(h, r.L);
            set_fatal(s, "admission failed: " + ex_->error_message());
            return -1;
        }
        slot_req_[slot] = r;
        slot_req_[slot].t_admit = ex_->now();
        slot_h_[slot] = h;
        slot_first_[slot] = ex_->launched();  // the upload precedes the next launch
        ++live_;
        dirty_ = true;
        return 1;
    }

    // Deliver the finished problem of slot s and free the slot.
    bool complete(int s) {
        const SchedRequest r = slot_req_[s];
        SchedResult res;
        if (ex_->finish(s, slot_h_[s], r.keep_x, &res) != MG_OK) return false;
        const double now = ex_->now();
        res.stats.seconds = now - r.t_submit;
        res.stats.queue_seconds = r.t_admit - r.t_submit;
        release_hierarchy(slot_h_[s], r.L);
        slot_h_[s] = nullptr;
        --live_;
        dirty_ = true;
        std::lock_guard<std::mutex> g(mu_);
        pending_.erase(r.ticket);
        done_.emplace(r.ticket, std::move(res));
        done_order_.push_back(r.ticket);
        ++completed_;
        cv_done_.notify_all();
        return true;
    }

    // Caller holds mu_.
    mg_status collect(uint64_t t, double* host_x, mg_stats* st) {
        auto it = done_.find(t);
        SchedResult& r = it->second;
        if (host_x && !r.x.empty()) std::memcpy(host_x, r.x.data(), r.x.size() * sizeof(double));
        if (st) *st = r.stats;
        const mg_status status = r.stats.status;
        done_.erase(it);
        for (auto q = done_order_.begin(); q != done_order_.end(); ++q)
            if (*q == t) {
                done_order_.erase(q);
                break;
            }
        return status;
    }

    void run() {
        int64_t next = ex_->launched();  // oldest iteration not yet reported
        double t_busy = 0.0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(mu_);
                const bool idle = live_.load() == 0 && next == ex_->launched();
                if (idle) cv_work_.wait(g, [&] { return stop_ || !queue_.empty(); });
                if (fatal_ != MG_OK) return;
                if (stop_ && queue_.empty() && live_.load() == 0 && next == ex_->launched())
                    return;
                // admit in arrival order while a slot and memory are available
                while (!queue_.empty()) {
                    int slot = -1;
                    for (int s = 0; s < (int)slot_h_.size(); ++s)
                        if (!slot_h_[s]) {
                            slot = s;
                            break;
                        }
                    if (slot < 0) break;
                    const SchedRequest r = queue_.front();
                    g.unlock();
                    const int ok = admit_one(slot, r);
                    g.lock();
                    if (ok < 0) return;
                    if (ok == 0) {
                        if (live_.load() == 0 && next == ex_->launched()) {
                            // cannot fit even alone: fail the request cleanly
                            queue_.pop_front();
                            pending_.erase(r.ticket);
                            SchedResult res;
                            res.stats.status = MG_ERR_NOMEM;
                            res.stats.seconds = ex_->now() - r.t_submit;
                            done_.emplace(r.ticket, std::move(res));
                            done_order_.push_back(r.ticket);
                            ++completed_;
                            cv_done_.notify_all();
                            continue;
                        }
                        break;  // wait for running requests to free memory
                    }
                    queue_.pop_front();
                }
            }
            if (dirty_) {
                if (mg_status s = ex_->upload()) {
                    set_fatal(s, "upload failed: " + ex_->error_message());
                    return;
                }
                dirty_ = false;
            }
            // keep two iterations in flight while problems are live
            if (live_.load() > 0 && ex_->launched() - next < 2) {
                if (next == ex_->launched()) t_busy = ex_->now();
                if (mg_status s = ex_->launch_iteration()) {
                    set_fatal(s, "iteration launch failed: " + ex_->error_message());
                    return;
                }
                if (ex_->launched() - next < 2) continue;  // queue the second one first
            }
            if (next == ex_->launched()) continue;
            const int* done = nullptr;
            if (mg_status s = ex_->wait_iteration(next, &done)) {
                set_fatal(s, "iteration failed: " + ex_->error_message());
                return;
            }
            const int64_t k = next++;
            if (next == ex_->launched()) busy_seconds_.store(busy_seconds_.load() + ex_->now() - t_busy);
            for (int s = 0; s < (int)slot_h_.size(); ++s) {
                if (!slot_h_[s] || slot_first_[s] > k || !done[s]) continue;
                if (!complete(s)) {
                    set_fatal(MG_ERR_DEVICE, "result copy failed: " + ex_->error_message());
                    return;
                }
            }
        }
    }

    Executor* ex_;
    const size_t budget_;
    std::thread worker_;
    // shared with the submitting and collecting threads (under mu_)
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    bool stop_ = false;
    mg_status fatal_ = MG_OK;
    std::string fatal_msg_;
    uint64_t next_ticket_ = 1;
    std::deque<SchedRequest> queue_;
    std::unordered_map<uint64_t, SchedResult> done_;  // finished, not yet collected
    std::deque<uint64_t> done_order_;
    std::unordered_map<uint64_t, int> pending_;  // submitted, not finished
    uint64_t completed_ = 0;
    size_t queue_high_ = 0;
    // written by the worker, read by info()
    std::atomic<int> live_{0};
    std::atomic<size_t> bytes_{0};  // hierarchies held (live + idle pool)
    std::atomic<size_t> high_water_{0};
    std::atomic<double> busy_seconds_{0.0};  // time with an iteration on the device
    // worker-owned
    std::vector<SchedRequest> slot_req_;
    std::vector<void*> slot_h_;
    std::vector<int64_t> slot_first_;  // first iteration that sees the slot's problem
    std::list<PoolEntry> pool_;        // idle hierarchies, least recently used first
    bool dirty_ = false;               // slots changed since the last upload
};

}  // namespace mg
