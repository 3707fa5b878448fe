// Serving loop: solve requests (level, tolerance, grid and right-hand-side
// seeds) arrive at any time; the scheduler (scheduler.h) admits them in
// arrival order into free slots of a BatchEngine while the device-memory
// budget allows, and this file's executor builds each request's problem on
// the device (jittered geometry, assembly, uniform right-hand side) in a
// resident hierarchy of its level and advances all live requests together
// one graph-replayed iteration at a time.  Requests that arrive while others
// run join at the next iteration (continuous batching); finished ones leave
// their slot at once.  The device always has the next iteration queued while
// the scheduler handles the report of the previous one, so host work does
// not idle the GPU.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <vector>

#include "batch.h"
#include "scheduler.h"

namespace mg {
double mixed_solve_bytes(int L, int Lc, int nu_pre, int nu_post, const BState& S);
void fill_stats(const BState& S, int L, int Lc, int nu_pre, int nu_post, mg_stats* st);
}  // namespace mg

using namespace mg;

namespace {

// The device side of the server: resident hierarchies and the batch engine.
class HipExecutor final : public Executor {
public:
    mg_status init(mg_context* ctx, int slots, int Lmax, int Lc, const mg_solve_opts& o) {
        ctx_ = ctx;
        Lc_ = Lc;
        opts_ = o;
        done_.assign(slots, 0);
        eng_.use_tuned_widths(false);  // the live mix changes every iteration
        return eng_.init(ctx->device, slots, Lmax, Lc, o.nu_pre, o.nu_post);
    }
    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }
    int capacity() const override { return eng_.capacity(); }
    size_t hierarchy_bytes(int L) const override { return mg_hierarchy_bytes(L, Lc_); }
    void* create_hierarchy(int L) override {
        (void)hipSetDevice(ctx_->device);
        mg_hierarchy* h = nullptr;
        if (mg_hierarchy_create(ctx_, L, Lc_, 0.0, 0, nullptr, &h) != MG_OK) return nullptr;
        return h;
    }
    void destroy_hierarchy(void* h) override { mg_hierarchy_destroy((mg_hierarchy*)h); }
    // Coordinates, right-hand side and x0 = 0, assembly of every level and
    // the coarse factor on the setup stream; upload() orders the next
    // iteration after them.
    mg_status admit(int slot, void* hv, const SchedRequest& r) override {
        (void)hipSetDevice(ctx_->device);
        mg_hierarchy* h = (mg_hierarchy*)hv;
        hipStream_t st = eng_.setup_stream();
        const Level& F = h->lv[r.L];
        MG_HIP(launch_coords_rhs(h->coords, r.L, r.jitter, r.geom_seed, r.rhs_seed, h->dmask,
                                 F.b64, F.x64, st));
        MG_HIP(launch_assemble(h->coords, h->lv, Lc_, r.L, h->dmask, st));
        MG_HIP(launch_chol_factor(h->lv[Lc_], h->dmask, h->chol, h->flag, st));
        h->assembled = true;
        mg_solve_opts o = opts_;
        o.rel_tol = r.tol;
        eng_.set_slot(slot, h, o);
        eng_.start_slot(slot);
        return MG_OK;
    }
    mg_status upload() override { return eng_.upload_async(); }
    mg_status launch_iteration() override {
        const TraceRange trace("serve iteration launch");
        return eng_.launch_iteration();
    }
    int64_t launched() const override { return eng_.launched(); }
    mg_status wait_iteration(int64_t k, const int** done) override {
        int nlive = 0, sure = 0;
        const int* flags = nullptr;
        if (mg_status s = eng_.wait_iteration(k, &nlive, &sure, &flags)) return s;
        for (size_t s = 0; s < done_.size(); ++s) done_[s] = (flags[s] & BF_DONE) != 0;
        *done = done_.data();
        return MG_OK;
    }
    // A finished problem's state and iterate are no longer written by the
    // queued iterations: read on the engine's read stream.
    mg_status finish(int slot, void* hv, int keep_x, SchedResult* out) override {
        mg_hierarchy* h = (mg_hierarchy*)hv;
        BState S;
        if (mg_status s = eng_.fetch_state(slot, &S)) return s;
        fill_stats(S, h->L, Lc_, opts_.nu_pre, opts_.nu_post, &out->stats);
        if (keep_x) {
            const Level& F = h->lv[h->L];
            out->x.resize(F.n);
            if (mg_status s = eng_.fetch(F.x64, out->x.data(), out->x.size() * sizeof(double)))
                return s;
        }
        eng_.clear_slot(slot);
        return MG_OK;
    }
    std::string error_message() override { return mg_last_error(); }

private:
    mg_context* ctx_ = nullptr;
    int Lc_ = 1;
    mg_solve_opts opts_{};
    BatchEngine eng_;
    std::vector<int> done_;
};

}  // namespace

struct mg_server {
    mg_context* ctx = nullptr;
    int Lmax = 11, Lc = 1;
    size_t budget = 0;
    HipExecutor ex;
    Scheduler* sched = nullptr;  // after ex (uses it), destroyed before it
    ~mg_server() { delete sched; }
};

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
    mg_solve_opts o;
    if (opts)
        o = *opts;
    else
        mg_default_opts(&o);
    o.precision = MG_PREC_MIXED;
    o.krylov = 0;
    if (mg_status st = s->ex.init(ctx, slots, max_level, coarse_level, o)) {
        delete s;
        return st;
    }
    s->sched = new (std::nothrow) Scheduler(&s->ex, budget);
    if (!s->sched) {
        delete s;
        return fail(MG_ERR_NOMEM, "host allocation failed");
    }
    s->sched->start();
    *out = s;
    return MG_OK;
}

mg_status mg_server_submit(mg_server* s, int L, double rel_tol, double jitter, uint64_t geom_seed,
                           uint64_t rhs_seed, int keep_x, uint64_t* ticket) {
    if (!s || !ticket) return fail(MG_ERR_INVALID, "null server or ticket");
    if (L < s->Lc || L > s->Lmax) return fail(MG_ERR_INVALID, "level outside the server's range");
    if (!(rel_tol >= 0.0) || !(jitter >= 0.0 && jitter < 0.5))
        return fail(MG_ERR_INVALID, "invalid tolerance or jitter");
    std::string err;
    const mg_status st =
        s->sched->submit(L, rel_tol, jitter, geom_seed, rhs_seed, keep_x, ticket, &err);
    return st == MG_OK ? MG_OK : fail(st, err);
}

mg_status mg_server_poll(mg_server* s, uint64_t ticket, double* host_x, mg_stats* st) {
    if (!s) return fail(MG_ERR_INVALID, "null server");
    std::string err;
    const mg_status r = s->sched->poll(ticket, host_x, st, &err);
    if (!err.empty()) return fail(r, err);
    return r;
}

mg_status mg_server_next(mg_server* s, double timeout_s, uint64_t* ticket, double* host_x,
                         mg_stats* st) {
    if (!s || !ticket) return fail(MG_ERR_INVALID, "null server or ticket");
    std::string err;
    const mg_status r = s->sched->next(timeout_s, ticket, host_x, st, &err);
    if (!err.empty()) return fail(r, err);
    return r;
}

mg_status mg_server_info(mg_server* s, mg_server_info_t* info) {
    if (!s || !info) return fail(MG_ERR_INVALID, "null argument");
    s->sched->info(info);
    return MG_OK;
}

mg_status mg_server_destroy(mg_server* s) {
    if (!s) return fail(MG_ERR_INVALID, "null server");
    s->sched->shutdown();
    delete s;
    return MG_OK;
}

}  // extern "C"
