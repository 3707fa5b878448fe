// CPU tests of the server's scheduler (paper_0904_4152_amd/csrc/scheduler.h)
// against a fake executor with a simulated clock: one tick per launched
// iteration, problems that finish after a known number of iterations, and
// failures injected through the request seeds.  Built plain (g++), with
// -fsanitize=thread (clang++) and with -fsanitize=address,undefined (g++),
// and run by tests/test_native_sanitizers.py; prints "PASS <scenario>" per
// scenario and exits non-zero on the first failed check.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "scheduler.h"

using namespace mg;

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);     \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

constexpr uint64_t SEED_NAN = 777;         // the problem ends with a NaN residual
constexpr uint64_t SEED_ADMIT_FAIL = 666;  // building the problem fails on the device
constexpr double TICK = 1e-3;              // simulated seconds per iteration

struct FakeH {
    int L;
    int id;
};

class FakeExecutor final : public Executor {
public:
    FakeExecutor(int slots, size_t budget) : budget_(budget), slots_(slots), done_(slots, 0) {}

    double now() override { return ticks_.load() * TICK; }
    int capacity() const override { return slots_; }
    size_t hierarchy_bytes(int L) const override { return size_t(1) << (2 * L); }
    void* create_hierarchy(int L) override {
        if (L == create_fail_level) return nullptr;
        in_use_ += hierarchy_bytes(L);
        CHECK(in_use_ <= budget_);  // the scheduler never exceeds its budget
        ++creates;
        return new FakeH{L, next_id_++};
    }
    void destroy_hierarchy(void* hv) override {
        FakeH* h = (FakeH*)hv;
        in_use_ -= hierarchy_bytes(h->L);
        destroyed_levels.push_back(h->L);
        delete h;
    }
    mg_status admit(int slot, void* hv, const SchedRequest& r) override {
        if (r.geom_seed == SEED_ADMIT_FAIL) return MG_ERR_DEVICE;
        Slot& s = slot_state(slot);
        CHECK(!s.used);  // a slot holds one problem at a time
        CHECK(((FakeH*)hv)->L == r.L);
        s = Slot{};
        s.used = true;
        s.ticket = r.ticket;
        s.L = r.L;
        s.need = 1 + int(r.rhs_seed % 5);  // iterations until the problem is done
        s.nan = r.geom_seed == SEED_NAN;
        s.start = -1;  // visible from the first iteration after the next upload
        admitted.push_back(r.ticket);
        return MG_OK;
    }
    mg_status upload() override {
        for (auto& kv : slots_state_)
            if (kv.second.used && kv.second.start < 0) kv.second.start = launched_;
        ++uploads;
        return MG_OK;
    }
    mg_status launch_iteration() override {
        const int64_t k = launched_++;
        ++ticks_;
        max_in_flight = std::max<int64_t>(max_in_flight, launched_ - reported_);
        for (auto& kv : slots_state_) {
            Slot& s = kv.second;
            if (!s.used || s.start < 0 || k < s.start || s.done_at >= 0) continue;
            if (--s.need == 0) s.done_at = k;
        }
        return MG_OK;
    }
    int64_t launched() const override { return launched_; }
    mg_status wait_iteration(int64_t k, const int** done) override {
        CHECK(k == reported_ && k < launched_);  // reports in order, of launched iterations
        reported_ = k + 1;
        for (int s = 0; s < slots_; ++s) {
            auto it = slots_state_.find(s);
            done_[s] = it != slots_state_.end() && it->second.used && it->second.done_at >= 0 &&
                       it->second.done_at <= k;
        }
        *done = done_.data();
        return MG_OK;
    }
    mg_status finish(int slot, void* hv, int keep_x, SchedResult* out) override {
        Slot& s = slot_state(slot);
        CHECK(s.used && s.done_at >= 0);
        out->stats.status = s.nan ? MG_ERR_NUMERIC : MG_OK;
        out->stats.rel_res = s.nan ? NAN : 1e-9;
        if (keep_x) out->x = {double(s.ticket), double(((FakeH*)hv)->L)};
        s.used = false;
        return MG_OK;
    }

    int create_fail_level = -1;
    int creates = 0;
    int uploads = 0;
    int64_t max_in_flight = 0;
    std::vector<uint64_t> admitted;
    std::vector<int> destroyed_levels;

private:
    struct Slot {
        bool used = false;
        uint64_t ticket = 0;
        int L = 0;
        int need = 0;
        bool nan = false;
        int64_t start = -1, done_at = -1;
    };
    Slot& slot_state(int s) { return slots_state_[s]; }

    const size_t budget_;
    const int slots_;
    std::atomic<int64_t> ticks_{0};
    size_t in_use_ = 0;
    int next_id_ = 0;
    int64_t launched_ = 0, reported_ = 0;
    std::map<int, Slot> slots_state_;
    std::vector<int> done_;
};

static mg_status wait_result(Scheduler& s, uint64_t t, mg_stats* st, double* x = nullptr) {
    for (int i = 0; i < 200000; ++i) {
        std::string err;
        const mg_status r = s.poll(t, x, st, &err);
        if (r != MG_ERR_BUSY) return r;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    CHECK(!"result never arrived");
    return MG_ERR_BUSY;
}

// Many requests from two submitting threads while a third collects: every
// request completes once with its own result, admission follows arrival
// order, at most two iterations are in flight.
static void scenario_concurrent() {
    const size_t budget = size_t(1) << 40;
    FakeExecutor ex(4, budget);
    Scheduler sched(&ex, budget);
    sched.start();
    const int per_thread = 200;
    std::mutex mu;
    std::set<uint64_t> submitted;
    auto submitter = [&](int id) {
        for (int i = 0; i < per_thread; ++i) {
            uint64_t t = 0;
            std::string err;
            const int L = 3 + (i + id) % 4;
            CHECK(sched.submit(L, 1e-8, 0.1, 1000 + i, 2000 + 7 * i + id, 1, &t, &err) == MG_OK);
            std::lock_guard<std::mutex> g(mu);
            CHECK(submitted.insert(t).second);
        }
    };
    std::atomic<int> got{0};
    std::thread collector([&] {
        while (got.load() < 2 * per_thread) {
            uint64_t t = 0;
            double x[2] = {-1, -1};
            mg_stats st{};
            std::string err;
            const mg_status r = sched.next(5.0, &t, x, &st, &err);
            CHECK(r == MG_OK);
            CHECK(x[0] == double(t));  // each result belongs to its ticket
            CHECK(st.status == MG_OK && st.seconds >= st.queue_seconds && st.queue_seconds >= 0);
            ++got;
        }
    });
    std::thread a(submitter, 0), b(submitter, 1);
    a.join();
    b.join();
    collector.join();
    sched.shutdown();
    CHECK(ex.admitted.size() == size_t(2 * per_thread));
    for (size_t i = 1; i < ex.admitted.size(); ++i) CHECK(ex.admitted[i - 1] < ex.admitted[i]);
    CHECK(ex.max_in_flight <= 2);
    mg_server_info_t info{};
    sched.info(&info);
    CHECK(info.completed == uint64_t(2 * per_thread) && info.live == 0 && info.queued == 0);
    std::printf("PASS concurrent\n");
}

// The budget holds two level-6 hierarchies: never more is held at once, and
// every request still completes.
static void scenario_budget() {
    const size_t budget = 2 * (size_t(1) << 12);
    FakeExecutor ex(8, budget);
    Scheduler sched(&ex, budget);
    std::vector<uint64_t> ts;
    for (int i = 0; i < 40; ++i) {
        uint64_t t = 0;
        std::string err;
        CHECK(sched.submit(5 + i % 2, 1e-8, 0.0, 1, 3 + i, 0, &t, &err) == MG_OK);
        ts.push_back(t);
    }
    sched.start();
    for (uint64_t t : ts) {
        mg_stats st{};
        CHECK(wait_result(sched, t, &st) == MG_OK);
    }
    mg_server_info_t info{};
    sched.info(&info);
    CHECK(info.bytes_high_water <= budget);
    sched.shutdown();
    std::printf("PASS budget\n");
}

// Idle hierarchies are evicted least recently used first, and only as many
// as the new one needs; an idle hierarchy of the requested level is reused.
static void scenario_lru_eviction() {
    const size_t budget = (size_t(1) << 12) + (size_t(1) << 8);  // L6 + L4
    FakeExecutor ex(1, budget);
    Scheduler sched(&ex, budget);
    sched.start();
    auto run1 = [&](int L) {
        uint64_t t = 0;
        std::string err;
        CHECK(sched.submit(L, 1e-8, 0.0, 1, 0, 0, &t, &err) == MG_OK);
        mg_stats st{};
        CHECK(wait_result(sched, t, &st) == MG_OK);
    };
    run1(5);  // pool: 5
    run1(4);  // pool: 5, 4
    run1(3);  // pool: 5, 4, 3 (1344 of 4352 bytes)
    CHECK(ex.creates == 3 && ex.destroyed_levels.empty());
    run1(6);  // needs 4096: evicts 5 (least recent), then 4; 3 stays
    CHECK(ex.destroyed_levels == std::vector<int>({5, 4}));
    const int creates = ex.creates;
    run1(3);  // reused from the pool
    CHECK(ex.creates == creates);
    sched.shutdown();
    std::printf("PASS lru_eviction\n");
}

// A large request at the head of the queue waits for memory; later small
// requests do not overtake it (arrival order), and it completes.
static void scenario_no_overtaking() {
    const size_t budget = size_t(1) << 14;  // one level-7 hierarchy
    FakeExecutor ex(4, budget);
    Scheduler sched(&ex, budget);
    std::vector<uint64_t> ts;
    std::string err;
    uint64_t t = 0;
    for (int i = 0; i < 3; ++i) {  // three level-6 problems, 4 iterations each
        CHECK(sched.submit(6, 1e-8, 0.0, 1, 3, 0, &t, &err) == MG_OK);
        ts.push_back(t);
    }
    CHECK(sched.submit(7, 1e-8, 0.0, 1, 0, 0, &t, &err) == MG_OK);  // needs the whole budget
    const uint64_t big = t;
    ts.push_back(t);
    for (int i = 0; i < 4; ++i) {
        CHECK(sched.submit(5, 1e-8, 0.0, 1, 0, 0, &t, &err) == MG_OK);
        ts.push_back(t);
    }
    sched.start();
    for (uint64_t x : ts) {
        mg_stats st{};
        CHECK(wait_result(sched, x, &st) == MG_OK);
    }
    sched.shutdown();
    for (size_t i = 1; i < ex.admitted.size(); ++i) CHECK(ex.admitted[i - 1] < ex.admitted[i]);
    CHECK(ex.admitted.size() == ts.size() && ex.admitted[3] == big);
    std::printf("PASS no_overtaking\n");
}

// Simulated latency: a lone request that needs k iterations is collected
// after k + 1 launched iterations (one iteration is always queued ahead).
static void scenario_latency() {
    const size_t budget = size_t(1) << 20;
    FakeExecutor ex(2, budget);
    Scheduler sched(&ex, budget);
    uint64_t t = 0;
    std::string err;
    CHECK(sched.submit(5, 1e-8, 0.0, 1, 2, 0, &t, &err) == MG_OK);  // 3 iterations
    sched.start();
    mg_stats st{};
    CHECK(wait_result(sched, t, &st) == MG_OK);
    CHECK(st.queue_seconds == 0.0);
    CHECK(std::fabs(st.seconds - 4 * TICK) < 1e-12);
    sched.shutdown();
    CHECK(ex.max_in_flight == 2);
    std::printf("PASS latency\n");
}

// Requests larger than the budget are refused at submission; a request the
// device cannot hold even when idle finishes with MG_ERR_NOMEM; a NaN result
// finishes with MG_ERR_NUMERIC; the server keeps serving.
static void scenario_statuses() {
    const size_t budget = size_t(1) << 12;
    FakeExecutor ex(2, budget);
    ex.create_fail_level = 4;
    Scheduler sched(&ex, budget);
    sched.start();
    uint64_t t = 0;
    std::string err;
    CHECK(sched.submit(7, 1e-8, 0.0, 1, 0, 0, &t, &err) == MG_ERR_NOMEM);
    CHECK(sched.submit(4, 1e-8, 0.0, 1, 0, 0, &t, &err) == MG_OK);
    mg_stats st{};
    CHECK(wait_result(sched, t, &st) == MG_ERR_NOMEM && st.status == MG_ERR_NOMEM);
    CHECK(sched.submit(5, 1e-8, 0.0, SEED_NAN, 1, 0, &t, &err) == MG_OK);
    CHECK(wait_result(sched, t, &st) == MG_ERR_NUMERIC && std::isnan(st.rel_res));
    CHECK(sched.submit(5, 1e-8, 0.0, 1, 1, 1, &t, &err) == MG_OK);
    double x[2] = {0, 0};
    CHECK(wait_result(sched, t, &st, x) == MG_OK && x[0] == double(t) && x[1] == 5.0);
    CHECK(sched.poll(t, nullptr, &st, &err) == MG_ERR_INVALID);  // collected once
    sched.shutdown();
    std::printf("PASS statuses\n");
}

// A device failure while building a problem stops the server: pending
// tickets and new submissions report it, and shutdown still returns.
static void scenario_executor_failure() {
    const size_t budget = size_t(1) << 20;
    FakeExecutor ex(2, budget);
    Scheduler sched(&ex, budget);
    uint64_t ok = 0, bad = 0, later = 0;
    std::string err;
    CHECK(sched.submit(5, 1e-8, 0.0, SEED_ADMIT_FAIL, 0, 0, &bad, &err) == MG_OK);
    CHECK(sched.submit(5, 1e-8, 0.0, 1, 0, 0, &later, &err) == MG_OK);
    sched.start();
    mg_stats st{};
    CHECK(wait_result(sched, bad, &st) == MG_ERR_DEVICE);
    CHECK(sched.poll(later, nullptr, &st, &err) == MG_ERR_DEVICE);
    CHECK(sched.submit(5, 1e-8, 0.0, 1, 0, 0, &ok, &err) == MG_ERR_DEVICE);
    uint64_t t = 0;
    CHECK(sched.next(0.01, &t, nullptr, &st, &err) == MG_ERR_DEVICE);
    sched.shutdown();
    std::printf("PASS executor_failure\n");
}

int main() {
    scenario_concurrent();
    scenario_budget();
    scenario_lru_eviction();
    scenario_no_overtaking();
    scenario_latency();
    scenario_statuses();
    scenario_executor_failure();
    std::printf("ALL PASS\n");
    return 0;
}
