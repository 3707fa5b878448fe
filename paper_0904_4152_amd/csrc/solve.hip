// Multigrid drivers (Sec. 6.2): the V(nu_pre, nu_post) cycle with damped
// Jacobi smoothing, the FP64 solver and the mixed-precision defect
// correction with single-precision inner cycles.  Cycles are captured once
// per hierarchy into HIP graphs and replayed, which removes the launch cost
// of the coarse levels (tens of tiny kernels per cycle).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "fused_ops.h"
#include "solve.h"

struct GraphEntry {
    int kind;  // 0: FP64 cycle + residual norm; 1: FP32 inner cycle + residual norm;
               // 2, 3: preconditioned CG step with an FP64 / FP32 cycle;
               // 4: `reps` guarded FP32 inner cycles, each with its norm and control
    int reps;
    int nu_pre, nu_post;
    double omega;
    bool x_zero;
    hipGraphExec_t exec;
    double bytes;
    uint64_t epoch;  // tile table epoch the fused passes were captured with
};

struct GraphCache {
    hipStream_t st = nullptr;  // internal non-blocking stream (capture needs one)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;  // order st after / before the caller's stream
    bool capture_ok = true;
    std::vector<GraphEntry> entries;
};

namespace mg {

namespace {

template <typename T>
struct LV;
template <>
struct LV<double> {
    static double* x(Level& l) { return l.x64; }
    static double* b(Level& l) { return l.b64; }
    static double* t(Level& l) { return l.t64; }
    static const double* bands(const Level& l) { return l.bands64; }
};
template <>
struct LV<float> {
    static float* x(Level& l) { return l.x32; }
    static float* b(Level& l) { return l.b32; }
    static float* t(Level& l) { return l.t32; }
    static const float* bands(const Level& l) { return l.bands32; }
};

#define MG_TRY(call)                         \
    do {                                     \
        hipError_t e_ = (call);              \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

}  // namespace

// Byte model (algorithmic HBM traffic, s = sizeof(T)): band product family
// 9 bands + x (+ b) (+ output); Jacobi from zero: diagonal + b + output;
// restriction: fine defect + coarse rhs; prolongation: coarse x + fine x
// read and written.
template <typename T>
hipError_t enqueue_vcycle(mg_hierarchy* h, int l, T* x, const T* b, bool x_zero, int nu_pre,
                          int nu_post, double omega, Enq& q) {
    Level& lv = h->lv[l];
    const double s = sizeof(T), n = (double)lv.n;
    const T om = (T)omega;
    if (l == h->Lc) {
        MG_TRY(launch_coarse<T>(coarse_solver(h), lv.N, b, x, q.st));
        q.bytes += 2 * s * n;
        return hipSuccess;
    }
    const T* bands = LV<T>::bands(lv);
    T* cur = x;
    T* oth = LV<T>::t(lv);
    bool zero = x_zero;
    if (zero && nu_pre == 0) {
        MG_TRY(launch_fill<T>(cur, lv.n, T(0), q.st));
        q.bytes += s * n;
        zero = false;
    }
    for (int k = 0; k < nu_pre; ++k) {
        if (zero) {
            MG_TRY(launch_jacobi_zero<T>(lv, bands, b, oth, om, q.st));
            q.bytes += 3 * s * n;
            zero = false;
        } else {
            MG_TRY(launch_jacobi<T>(lv, bands, b, cur, oth, om, q.st));
            q.bytes += 12 * s * n;
        }
        std::swap(cur, oth);
    }
    MG_TRY(launch_defect<T>(lv, bands, b, cur, oth, nullptr, nullptr, 0, nullptr, q.st));
    q.bytes += 12 * s * n;
    Level& lc = h->lv[l - 1];
    MG_TRY(launch_restrict<T>(lv.N, oth, LV<T>::b(lc), h->dmask, q.st));
    q.bytes += s * (n + (double)lc.n);
    MG_TRY(enqueue_vcycle<T>(h, l - 1, LV<T>::x(lc), LV<T>::b(lc), true, nu_pre, nu_post, omega,
                             q));
    MG_TRY(launch_prolong<T>(lv.N, LV<T>::x(lc), cur, q.st));
    q.bytes += s * ((double)lc.n + 2 * n);
    for (int k = 0; k < nu_post; ++k) {
        MG_TRY(launch_jacobi<T>(lv, bands, b, cur, oth, om, q.st));
        q.bytes += 12 * s * n;
        std::swap(cur, oth);
    }
    if (cur != x) {
        MG_TRY(launch_copy<T>(cur, x, lv.n, q.st));
        q.bytes += 2 * s * n;
    }
    return hipSuccess;
}

template hipError_t enqueue_vcycle<double>(mg_hierarchy*, int, double*, const double*, bool, int,
                                           int, double, Enq&);
template hipError_t enqueue_vcycle<float>(mg_hierarchy*, int, float*, const float*, bool, int,
                                          int, double, Enq&);

// V(2,2) cycle from the fused passes: per level one pre pass (two sweeps,
// defect, restriction: x -> t, b_c) and one post pass (prolongation, two
// sweeps: t + P x_c -> x).  With partials the top-level post pass also
// reduces ||b - A x|| into scal[slot], scal[slot + 1] (and host[slot..]).  Byte model: bands
// (9 s), iterate in (s, not when from zero), b (s) and iterate out (s) per
// node and pass, plus the coarse vector (s per coarse node).
template <typename T>
hipError_t enqueue_vcycle_fused(mg_hierarchy* h, int l, T* x, const T* b, bool x_zero,
                                double omega, Enq& q, double* partials, double* scal, int slot,
                                double* host) {
    Level& lv = h->lv[l];
    const double s = sizeof(T), n = (double)lv.n;
    const T om = (T)omega;
    const T* bands = LV<T>::bands(lv);
    if (l == h->Lc) {
        if (q.guard) return hipErrorInvalidValue;  // guarded cycles need a level above the tail
        MG_TRY(launch_coarse<T>(coarse_solver(h), lv.N, b, x, q.st));
        q.bytes += 2 * s * n;
        if (partials) {
            MG_TRY(launch_defect<T>(lv, bands, b, x, nullptr, partials, scal, slot, host, q.st));
            q.bytes += 11 * s * n;
        }
        return hipSuccess;
    }
    Level& lc = h->lv[l - 1];
    T* t = LV<T>::t(lv);
    MG_TRY(launch_pre<T>(lv, bands, x, x_zero, b, om, t, LV<T>::b(lc), h->dmask, q.st, q.guard));
    q.bytes += (x_zero ? 11 : 12) * s * n + s * (double)lc.n;
    if (l - 1 <= tail_max_level()) {
        // every coarser level in one workgroup; same bytes as the unfused cycle there
        MG_TRY(launch_tail<T>(h->lv, l - 1, h->Lc, coarse_solver(h), om, q.st, q.guard));
        for (int k = h->Lc + 1; k < l; ++k) q.bytes += 84.0 * s * (double)h->lv[k].n;
    } else {
        MG_TRY(enqueue_vcycle_fused<T>(h, l - 1, LV<T>::x(lc), LV<T>::b(lc), true, omega, q,
                                       nullptr, nullptr, 0, nullptr));
    }
    MG_TRY(launch_post<T>(lv, bands, t, LV<T>::x(lc), b, om, x, partials, scal, slot, host,
                          q.st, q.guard, partials ? q.ctl : RedCtl{}));
    q.bytes += 12 * s * n + s * (double)lc.n;
    return hipSuccess;
}

template hipError_t enqueue_vcycle_fused<double>(mg_hierarchy*, int, double*, const double*, bool,
                                                 double, Enq&, double*, double*, int, double*);
template hipError_t enqueue_vcycle_fused<float>(mg_hierarchy*, int, float*, const float*, bool,
                                                double, Enq&, double*, double*, int, double*);

// One step of CG preconditioned by one V-cycle from zero (Sec. 4.1: a
// solver as another's preconditioner; the cycle of Sec. 6.2), on the finest
// level's vectors: x in x64, r in d64, p in b64 (the right-hand side copy is
// not needed once r0 is formed), and z / q sharing the FP32 pair x32|b32
// (never live together, nor with the FP32 cycle's own use of the pair):
//   z = M r (kind 2: FP64 cycle; kind 3: FP32 cycle on r / ||r||, z =
//   ||r|| c32); rz = r.z; p = z + (rz / rz_old) p; rz_old = rz; q = A p;
//   alpha = rz / p.q; x += alpha p; r -= alpha q; ||r|| to the host mirror.
// Before the first step scal[SC_RZ_OLD] is +inf, so the first p is z.
static hipError_t enqueue_pcg_step(mg_hierarchy* h, bool mixed, int nu_pre, int nu_post,
                                   double omega, Enq& q) {
    Level& F = h->lv[h->L];
    const int64_t n = F.n;
    const double dn = (double)n;
    double* r = h->d64;
    double* p = F.b64;
    double* zq = reinterpret_cast<double*>(F.x32);
    const bool fused = nu_pre == 2 && nu_post == 2;
    if (!mixed) {
        if (fused)
            MG_TRY(enqueue_vcycle_fused<double>(h, h->L, zq, r, true, omega, q, nullptr, nullptr,
                                                0, nullptr));
        else
            MG_TRY(enqueue_vcycle<double>(h, h->L, zq, r, true, nu_pre, nu_post, omega, q));
        MG_TRY(launch_dot<double>(r, zq, n, h->scal, -1, h->partials, h->scal, SC_RZ, q.st));
        MG_TRY(launch_pcg_dir<double>(p, zq, n, h->scal, -1, SC_RZ, SC_RZ_OLD, q.st));
        q.bytes += (16.0 + 24.0) * dn;
    } else {
        MG_TRY(launch_cast_scaled(r, F.b32, n, h->scal, SC_RR, q.st));
        if (fused)
            MG_TRY(enqueue_vcycle_fused<float>(h, h->L, F.x32, F.b32, true, omega, q, nullptr,
                                               nullptr, 0, nullptr));
        else
            MG_TRY(enqueue_vcycle<float>(h, h->L, F.x32, F.b32, true, nu_pre, nu_post, omega, q));
        MG_TRY(launch_dot<float>(r, F.x32, n, h->scal, SC_RR, h->partials, h->scal, SC_RZ, q.st));
        MG_TRY(launch_pcg_dir<float>(p, F.x32, n, h->scal, SC_RR, SC_RZ, SC_RZ_OLD, q.st));
        q.bytes += (12.0 + 12.0 + 20.0) * dn;
    }
    MG_TRY(launch_scalar_copy(h->scal, SC_RZ, SC_RZ_OLD, q.st));
    MG_TRY(launch_spmv<double>(F, F.bands64, p, zq, q.st, true));
    MG_TRY(launch_dot<double>(p, zq, n, h->scal, -1, h->partials, h->scal, SC_PQ, q.st));
    MG_TRY(launch_pcg_step(F.x64, r, p, zq, n, h->scal, SC_RZ, SC_PQ, h->partials, SC_RR,
                           h->host_scal, q.st));
    q.bytes += (88.0 + 16.0 + 48.0) * dn;
    return hipSuccess;
}

// The unit replayed per iteration: FP64 cycle + FP64 residual norm (kind 0)
// or FP32 inner cycle + FP32 residual norm (kind 1), on the finest level's
// own vectors, or a preconditioned CG step (kinds 2, 3), or `reps` fused
// FP32 inner cycles under device control (kind 4: each cycle's kernels
// return at once when scal[SC_STOP] is set, and the reduction of its
// residual norm decides whether the loop goes on: RED_STEP).
static hipError_t enqueue_unit(mg_hierarchy* h, int kind, int reps, int nu_pre, int nu_post,
                               double omega, bool x_zero, Enq& q) {
    Level& F = h->lv[h->L];
    const double n = (double)F.n;
    if (kind == 4) {
        Enq g{q.st, 0.0, h->scal + SC_STOP};
        g.ctl.mode = RED_STEP;
        for (int i = 0; i < reps; ++i)
            MG_TRY(enqueue_vcycle_fused<float>(h, h->L, F.x32, F.b32, x_zero && i == 0, omega, g,
                                               h->partials, h->scal, SC_R32, h->host_scal));
        q.bytes += g.bytes;
        return hipSuccess;
    }
    if (kind >= 2) return enqueue_pcg_step(h, kind == 3, nu_pre, nu_post, omega, q);
    if (nu_pre == 2 && nu_post == 2) {
        if (kind == 0)
            return enqueue_vcycle_fused<double>(h, h->L, F.x64, F.b64, false, omega, q,
                                                h->partials, h->scal, SC_R64, h->host_scal);
        return enqueue_vcycle_fused<float>(h, h->L, F.x32, F.b32, x_zero, omega, q, h->partials,
                                           h->scal, SC_R32, h->host_scal);
    }
    if (kind == 0) {
        MG_TRY(enqueue_vcycle<double>(h, h->L, F.x64, F.b64, false, nu_pre, nu_post, omega, q));
        MG_TRY(launch_defect<double>(F, F.bands64, F.b64, F.x64, nullptr, h->partials, h->scal,
                                     SC_R64, h->host_scal, q.st));
        q.bytes += 11 * 8 * n;
    } else {
        MG_TRY(enqueue_vcycle<float>(h, h->L, F.x32, F.b32, x_zero, nu_pre, nu_post, omega, q));
        MG_TRY(launch_defect<float>(F, F.bands32, F.b32, F.x32, nullptr, h->partials, h->scal,
                                    SC_R32, h->host_scal, q.st));
        q.bytes += 11 * 4 * n;
    }
    return hipSuccess;
}

static GraphCache* cache(mg_hierarchy* h) {
    if (!h->graphs) h->graphs = new GraphCache();
    return h->graphs;
}

void destroy_graphs(mg_hierarchy* h) {
    if (!h->graphs) return;
    for (auto& e : h->graphs->entries) (void)hipGraphExecDestroy(e.exec);
    if (h->graphs->ev_in) (void)hipEventDestroy(h->graphs->ev_in);
    if (h->graphs->ev_out) (void)hipEventDestroy(h->graphs->ev_out);
    if (h->graphs->st) (void)hipStreamDestroy(h->graphs->st);
    delete h->graphs;
    h->graphs = nullptr;
}

// Run one unit, from a captured graph when allowed.
static hipError_t run_unit(mg_hierarchy* h, int kind, const mg_solve_opts& o, bool x_zero,
                           bool use_graph, Enq& q, int reps = 1) {
    GraphCache* gc = cache(h);
    if (use_graph && gc->capture_ok) {
        const uint64_t epoch = tile_table_epoch();
        for (size_t i = 0; i < gc->entries.size(); ++i) {
            GraphEntry& e = gc->entries[i];
            if (e.kind == kind && e.reps == reps && e.nu_pre == o.nu_pre &&
                e.nu_post == o.nu_post && e.omega == o.omega && e.x_zero == x_zero) {
                if (e.epoch == epoch) {
                    q.bytes += e.bytes;
                    return hipGraphLaunch(e.exec, q.st);
                }
                // tiles changed since the capture: wait for earlier replays,
                // then capture again below
                MG_TRY(hipStreamSynchronize(q.st));
                (void)hipGraphExecDestroy(e.exec);
                gc->entries.erase(gc->entries.begin() + i);
                break;
            }
        }
        Enq cq{q.st, 0.0};
        hipError_t e = hipStreamBeginCapture(q.st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t ee = enqueue_unit(h, kind, reps, o.nu_pre, o.nu_post, o.omega, x_zero, cq);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(q.st, &g);
            if (ee != hipSuccess) e = ee;
            hipGraphExec_t ex = nullptr;
            if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e == hipSuccess) {
                gc->entries.push_back(
                    {kind, reps, o.nu_pre, o.nu_post, o.omega, x_zero, ex, cq.bytes, epoch});
                q.bytes += cq.bytes;
                return hipGraphLaunch(ex, q.st);
            }
        }
        (void)hipGetLastError();
        gc->capture_ok = false;  // fall back to direct launches for this hierarchy
    }
    return enqueue_unit(h, kind, reps, o.nu_pre, o.nu_post, o.omega, x_zero, q);
}

// Host read-back of reduced norms.  Every reduction the drivers read writes
// its result straight into the hierarchy's pinned mirror (no copy).  Before
// the producing work is enqueued the host arms the slot with a value no
// norm takes; it then spins on the mirror, which returns as soon as the
// final reduction kernel has stored the norm, without the wake-up latency
// of a blocking stream synchronisation.  After 50 ms of spinning it falls
// back to synchronising the stream (which also reports device errors).
constexpr double kArmed = -1.0;

static void arm_scalar(mg_hierarchy* h, int slot) {
    ((volatile double*)h->host_scal)[slot + 1] = kArmed;
}

static hipError_t read_scalar(mg_hierarchy* h, int slot, hipStream_t st, double* out) {
    const TraceRange trace("host waits for a norm");
    const volatile double* v = (const volatile double*)h->host_scal + slot + 1;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned i = 1;; ++i) {
        const double x = *v;
        if (!(x == kArmed)) {
            *out = x;
            return hipSuccess;
        }
        if ((i & 4095u) == 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50))
            break;
    }
    MG_TRY(hipStreamSynchronize(st));
    *out = *v;
    return hipSuccess;
}

// The inner-loop state k_inner_ctrl mirrors (cycles run, plus ITER_DONE once
// the loop is over): wait until the loop is over or has run `want` cycles.
static void arm_iter(mg_hierarchy* h) { ((volatile double*)h->host_scal)[SC_ITER] = kArmed; }

static hipError_t read_iter(mg_hierarchy* h, int want, hipStream_t st, int* cycles, bool* done) {
    const TraceRange trace("host waits for the inner loop");
    const volatile double* v = (const volatile double*)h->host_scal + SC_ITER;
    const auto t0 = std::chrono::steady_clock::now();
    double x = kArmed;
    for (unsigned i = 1;; ++i) {
        x = *v;
        if (!(x == kArmed) && (x >= ITER_DONE || x == (double)want)) break;
        if ((i & 4095u) == 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
            MG_TRY(hipStreamSynchronize(st));
            x = *v;
            break;
        }
    }
    *done = x >= ITER_DONE;
    *cycles = (int)(*done ? x - ITER_DONE : x);
    return hipSuccess;
}

}  // namespace mg

using namespace mg;

#define MG_HIPS(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            st.status = MG_ERR_DEVICE;                                                        \
            if (stats) *stats = st;                                                           \
            return fail(MG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
        }                                                                                     \
    } while (0)

static mg_status validate_opts(const mg_solve_opts& o) {
    if (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post == 0 || o.nu_pre > 16 ||
        o.nu_post > 16)
        return fail(MG_ERR_INVALID, "smoothing steps must be in [0,16] and not both 0");
    if (!(o.omega > 0.0 && o.omega < 2.0)) return fail(MG_ERR_INVALID, "omega must lie in (0,2)");
    if (!(o.rel_tol >= 0.0) || o.max_cycles < 1)
        return fail(MG_ERR_INVALID, "rel_tol must be >= 0 and max_cycles >= 1");
    if (o.precision != MG_PREC_FP64 && o.precision != MG_PREC_MIXED)
        return fail(MG_ERR_INVALID, "unknown precision");
    if (o.precision == MG_PREC_MIXED &&
        (!(o.inner_reduction >= 0.0 && o.inner_reduction < 1.0) || o.inner_max_cycles < 1))
        return fail(MG_ERR_INVALID, "inner_reduction in [0,1) and inner_max_cycles >= 1 required");
    if (o.fixed_cycles < 0) return fail(MG_ERR_INVALID, "fixed_cycles must be >= 0");
    if (o.krylov != 0 && o.krylov != 1) return fail(MG_ERR_INVALID, "krylov must be 0 or 1");
    if (o.zero_guess != 0 && o.zero_guess != 1)
        return fail(MG_ERR_INVALID, "zero_guess must be 0 or 1");
    return MG_OK;
}

extern "C" mg_status mg_vcycle(mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                               void* x, int nu_pre, int nu_post, double omega, int fused,
                               void* stream) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (level < h->Lc || level > h->L) return fail(MG_ERR_INVALID, "level out of range");
    if (!h->assembled) return fail(MG_ERR_INVALID, "hierarchy not assembled");
    if (!b || !x || ((uintptr_t)b & 15) || ((uintptr_t)x & 15) || b == x)
        return fail(MG_ERR_INVALID, "b, x must be distinct 16-byte aligned device pointers");
    if (nu_pre < 0 || nu_post < 0 || nu_pre > 16 || nu_post > 16)
        return fail(MG_ERR_INVALID, "smoothing steps out of range");
    MG_HIP(hipSetDevice(h->ctx->device));
    Enq q{(hipStream_t)stream, 0.0};
    if (fused && (nu_pre != 2 || nu_post != 2))
        return fail(MG_ERR_INVALID, "the fused cycle is V(2,2)");
    if (fused && dtype == MG_F64)
        MG_HIP(enqueue_vcycle_fused<double>(h, level, (double*)x, (const double*)b, false, omega, q,
                                            nullptr, nullptr, 0, nullptr));
    else if (fused)
        MG_HIP(enqueue_vcycle_fused<float>(h, level, (float*)x, (const float*)b, false, omega, q,
                                           nullptr, nullptr, 0, nullptr));
    else if (dtype == MG_F64)
        MG_HIP(enqueue_vcycle<double>(h, level, (double*)x, (const double*)b, false, nu_pre,
                                      nu_post, omega, q));
    else
        MG_HIP(enqueue_vcycle<float>(h, level, (float*)x, (const float*)b, false, nu_pre, nu_post,
                                     omega, q));
    return MG_OK;
}

extern "C" mg_status mg_solve(mg_hierarchy* h, const double* dev_b, double* dev_x,
                              const mg_solve_opts* opts, void* stream, mg_stats* stats) {
    const TraceRange trace("mg_solve");
    const auto t0 = std::chrono::steady_clock::now();
    mg_stats st{};
    if (stats) *stats = st;
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (!h->assembled) return fail(MG_ERR_INVALID, "hierarchy not assembled");
    if (!dev_b || !dev_x || dev_b == dev_x || ((uintptr_t)dev_b & 15) || ((uintptr_t)dev_x & 15))
        return fail(MG_ERR_INVALID, "b, x must be distinct 16-byte aligned device pointers");
    mg_solve_opts o;
    if (opts)
        o = *opts;
    else
        mg_default_opts(&o);
    if (mg_status s = validate_opts(o)) return s;
    MG_HIP(hipSetDevice(h->ctx->device));
    GraphCache* gc = cache(h);
    if (!gc->st) MG_HIP(hipStreamCreateWithFlags(&gc->st, hipStreamNonBlocking));
    if (!gc->ev_in) MG_HIP(hipEventCreateWithFlags(&gc->ev_in, hipEventDisableTiming));
    if (!gc->ev_out) MG_HIP(hipEventCreateWithFlags(&gc->ev_out, hipEventDisableTiming));
    // The internal stream waits (on the device) for the caller's producers
    // of b and x.
    MG_HIPS(hipEventRecord(gc->ev_in, (hipStream_t)stream));
    MG_HIPS(hipStreamWaitEvent(gc->st, gc->ev_in, 0));
    Enq q{gc->st, 0.0};
    Level& F = h->lv[h->L];
    const int64_t n = F.n;
    const bool graphs = o.use_graph != 0;
    // The mixed-precision loop touches the FP64 vectors only in directly
    // launched kernels (defect, update), so it reads the caller's b and
    // updates the caller's x in place; the other solvers' captured graphs
    // work on the hierarchy's own copies.
    const bool direct = !o.krylov && o.precision == MG_PREC_MIXED;
    const double* B64 = direct ? dev_b : F.b64;
    double* X64 = direct ? dev_x : F.x64;
    // zero_guess: x0 = 0 whatever dev_x holds (not read; the mixed solve's
    // first update writes x without reading it)
    const bool zg = o.zero_guess != 0;
    if (!direct) {
        MG_HIPS(launch_copy<double>(dev_b, F.b64, n, q.st));
        if (zg)
            MG_HIPS(launch_fill<double>(F.x64, n, 0.0, q.st));
        else
            MG_HIPS(launch_copy<double>(dev_x, F.x64, n, q.st));
        q.bytes += zg ? 8.0 * 3 * n : 8.0 * 4 * n;
    }
    // the mixed solve under device control (see the last branch below)
    const bool devctl = !o.krylov && o.precision == MG_PREC_MIXED && o.nu_pre == 2 &&
                        o.nu_post == 2 && h->L > tail_max_level() &&
                        o.inner_max_cycles < (int)ITER_DONE;
    auto nslot = [](int k) { return (k & 1) ? SC_R64 : SC_R64B; };
    auto outer_ctl = [&](int k) {
        RedCtl c;
        c.mode = RED_OUTER;
        c.thr = o.fixed_cycles > 0 ? -1.0 : o.rel_tol;
        c.div = 1e3;
        c.cap = (o.fixed_cycles > 0 ? k > o.fixed_cycles : k > o.max_cycles) ? 1 : 0;
        c.reset = 1;  // a step that goes on starts its inner loop
        c.ithr = o.inner_reduction;
        c.icap = o.inner_max_cycles;
        return c;
    };
    const double* wait = h->scal + SC_WAIT;
    // the update of step k and the defect of step k + 1
    auto queue_update_defect = [&](int k) -> hipError_t {
        MG_TRY(launch_update(X64, F.x32, n, h->scal, q.st, wait, zg && k == 1));
        arm_scalar(h, nslot(k + 1));
        return launch_defect_cast(F, F.bands64, B64, X64, F.b32, h->partials, h->scal,
                                  nslot(k + 1), h->host_scal, q.st, wait, outer_ctl(k + 1));
    };
    int last = 0;      // cycles of the previous inner loop of this solve
    int pred = 0;      // cycles queued at once for the latest queued step
    double cycle_bytes = 0.0;
    // the predicted cycles, the update and the next defect of step k (the
    // defect of step k wrote the FP32 right-hand side and started the loop)
    auto queue_step = [&](int k) -> hipError_t {
        const int slot = std::min(k, 8) - 1;
        pred = h->inner_pred[slot] > 0 ? h->inner_pred[slot] : (last > 0 ? last : 2);
        pred = std::min(pred, o.inner_max_cycles);
        arm_iter(h);
        Enq cq{q.st, 0.0};
        MG_TRY(run_unit(h, 4, o, true, graphs, cq, pred));
        cycle_bytes = cq.bytes / pred;
        MG_TRY(queue_update_defect(k));
        return hipSuccess;
    };
    auto ahead = [&](int k) { return h->outer_prev <= 0 || k <= h->outer_prev; };
    bool queued = false;  // outer step k already queued
    arm_scalar(h, SC_B);
    MG_HIPS(launch_norm<double>(B64, n, h->partials, h->scal, SC_B, h->host_scal, q.st));
    q.bytes += 8.0 * n;
    // A zero initial iterate (the usual start) makes the first defect b
    // itself: its kernel then reads b alone (same bits, see
    // launch_defect_zero_x).
    if (!zg) {
        arm_scalar(h, SC_XNZ);
        RedCtl zflag;
        zflag.mode = devctl ? RED_ZFLAG : RED_NONE;
        MG_HIPS(launch_count_nonzero(X64, n, h->partials, h->scal, SC_XNZ, h->host_scal, q.st,
                                     zflag));
        q.bytes += 8.0 * n;
    }
    if (devctl) {
        // the first defect (of the zero or the given iterate: the other
        // kernel returns at once) and step 1, before ||b|| reaches the host;
        // the device's tests read ||b|| from its own copy
        arm_scalar(h, nslot(1));
        MG_HIPS(launch_defect_zero_x_cast(F, B64, F.b32, h->partials, h->scal, nslot(1),
                                          h->host_scal, q.st,
                                          zg ? nullptr : h->scal + SC_XNZ, outer_ctl(1)));
        if (!zg)
            MG_HIPS(launch_defect_cast(F, F.bands64, B64, X64, F.b32, h->partials, h->scal,
                                       nslot(1), h->host_scal, q.st, h->scal + SC_XZ,
                                       outer_ctl(1)));
        queued = ahead(1);
        if (queued) MG_HIPS(queue_step(1));
    }
    double bn = 0.0, xnz = 0.0;
    MG_HIPS(read_scalar(h, SC_B, q.st, &bn));
    if (!zg) MG_HIPS(read_scalar(h, SC_XNZ, q.st, &xnz));
    const bool x_zero = xnz == 0.0;
    st.bnorm = bn;
    mg_status result = MG_OK;
    if (!std::isfinite(bn)) {
        result = fail(MG_ERR_NUMERIC, "right-hand side contains NaN or Inf");
    } else if (bn == 0.0) {
        MG_HIPS(launch_fill<double>(X64, n, 0.0, q.st));
    } else if (o.krylov) {
        // r0 = b - A x0 and its norm; the first direction is z (beta = 0)
        double r = 0.0;
        arm_scalar(h, SC_RR);
        if (x_zero) {
            MG_HIPS(launch_defect_zero_x(F, F.b64, h->d64, h->partials, h->scal, SC_RR,
                                         h->host_scal, q.st));
            q.bytes += 16.0 * n;
        } else {
            MG_HIPS(launch_defect<double>(F, F.bands64, F.b64, F.x64, h->d64, h->partials,
                                          h->scal, SC_RR, h->host_scal, q.st));
            q.bytes += 12.0 * 8 * n;
        }
        MG_HIPS(launch_fill<double>(h->scal + SC_RZ_OLD, 1, INFINITY, q.st));
        MG_HIPS(read_scalar(h, SC_RR, q.st, &r));
        st.rel_res = r / bn;
        const int kind = o.precision == MG_PREC_FP64 ? 2 : 3;
        for (int k = 1;; ++k) {
            if (o.fixed_cycles > 0) {
                if (k > o.fixed_cycles) break;
            } else {
                if (r <= o.rel_tol * bn) break;
                if (k > o.max_cycles) {
                    result = fail(MG_ERR_NOCONV, "no convergence within max_cycles");
                    break;
                }
            }
            arm_scalar(h, SC_RR);
            MG_HIPS(run_unit(h, kind, o, false, graphs, q));
            MG_HIPS(read_scalar(h, SC_RR, q.st, &r));
            st.cycles = k;
            if (st.n_hist < MG_HIST) st.res_hist[st.n_hist++] = r / bn;
            if (!std::isfinite(r) || r > 1e3 * bn) {
                result = fail(MG_ERR_NUMERIC, "residual diverged or became NaN");
                break;
            }
        }
        // the true residual at exit, from the caller's b (the copy holds p)
        double rt = 0.0;
        arm_scalar(h, SC_R64);
        MG_HIPS(launch_defect<double>(F, F.bands64, dev_b, F.x64, nullptr, h->partials, h->scal,
                                      SC_R64, h->host_scal, q.st));
        q.bytes += 11.0 * 8 * n;
        MG_HIPS(read_scalar(h, SC_R64, q.st, &rt));
        st.rel_res = rt / bn;
    } else if (o.precision == MG_PREC_FP64) {
        double r = 0.0;
        arm_scalar(h, SC_R64);
        if (x_zero) {
            MG_HIPS(launch_defect_zero_x(F, F.b64, nullptr, h->partials, h->scal, SC_R64,
                                         h->host_scal, q.st));
            q.bytes += 8.0 * n;
        } else {
            MG_HIPS(launch_defect<double>(F, F.bands64, F.b64, F.x64, nullptr, h->partials,
                                          h->scal, SC_R64, h->host_scal, q.st));
            q.bytes += 11.0 * 8 * n;
        }
        MG_HIPS(read_scalar(h, SC_R64, q.st, &r));
        st.rel_res = r / bn;
        for (int k = 1;; ++k) {
            if (o.fixed_cycles > 0) {
                if (k > o.fixed_cycles) break;
            } else {
                if (r <= o.rel_tol * bn) break;
                if (k > o.max_cycles) {
                    result = fail(MG_ERR_NOCONV, "no convergence within max_cycles");
                    break;
                }
            }
            arm_scalar(h, SC_R64);
            MG_HIPS(run_unit(h, 0, o, false, graphs, q));
            MG_HIPS(read_scalar(h, SC_R64, q.st, &r));
            st.cycles = k;
            st.rel_res = r / bn;
            if (st.n_hist < MG_HIST) st.res_hist[st.n_hist++] = r / bn;
            if (!std::isfinite(r) || r > 1e3 * bn) {
                result = fail(MG_ERR_NUMERIC, "residual diverged or became NaN");
                break;
            }
        }
    } else if (!devctl) {
        // host-driven loop: one host read per FP64 defect and per FP32 cycle
        for (int k = 1;; ++k) {
            const TraceRange step("mixed outer step");
            double s = 0.0;
            arm_scalar(h, SC_R64);
            if (k == 1 && x_zero) {
                MG_HIPS(launch_defect_zero_x_cast(F, B64, F.b32, h->partials, h->scal, SC_R64,
                                                  h->host_scal, q.st));
                q.bytes += 12.0 * n;
            } else {
                MG_HIPS(launch_defect_cast(F, F.bands64, B64, X64, F.b32, h->partials, h->scal,
                                           SC_R64, h->host_scal, q.st));
                q.bytes += 92.0 * n;
            }
            MG_HIPS(read_scalar(h, SC_R64, q.st, &s));
            st.rel_res = s / bn;
            if (k > 1 && st.n_hist < MG_HIST) st.res_hist[st.n_hist++] = s / bn;
            if (!std::isfinite(s) || s > 1e3 * bn) {
                result = fail(MG_ERR_NUMERIC, "residual diverged or became NaN");
                break;
            }
            if (o.fixed_cycles > 0) {
                if (k > o.fixed_cycles) break;
            } else {
                if (s <= o.rel_tol * bn) break;
                if (k > o.max_cycles) {
                    result = fail(MG_ERR_NOCONV, "no convergence within max_cycles");
                    break;
                }
            }
            if (s == 0.0) break;
            // the FP32 right-hand side is the defect scaled by a power of
            // two: its loop stops relative to the scaled defect's norm
            const double dn = dev::pow2_scale(bn) * s;
            for (int it = 1; it <= o.inner_max_cycles; ++it) {
                double r32 = 0.0;
                arm_scalar(h, SC_R32);
                MG_HIPS(run_unit(h, 1, o, it == 1, graphs, q));
                MG_HIPS(read_scalar(h, SC_R32, q.st, &r32));
                st.cycles++;
                if (!std::isfinite(r32)) break;
                if (r32 <= o.inner_reduction * dn) break;
            }
            MG_HIPS(launch_update(X64, F.x32, n, h->scal, q.st, nullptr, zg && k == 1));
            q.bytes += 20.0 * n;
            st.outer_steps = k;
        }
    } else {
        // Device control (fused V(2,2) cycle): the decisions of the loop
        // above, taken on the device by the reductions that produce the
        // norms they test (RedCtl), with everything that follows a decision
        // queued behind it under a guard.  The FP64 defect of outer step k
        // writes the FP32 right-hand side, and its norm's reduction starts
        // the inner loop unless the solve is over.  After it the host
        // queues the FP32 cycles step k took in
        // the previous solve (each returning at once after the loop is
        // over), the update and the defect of step k + 1, which wait on the
        // device for the loop's end -- before reading the defect's norm when
        // the previous solve also took step k (then the device does not wait
        // for the host between outer steps), after it otherwise (a converged
        // solve leaves no skipped cycles behind).  The host reads the
        // defect's norm (its tests are the device's), then the loop's state;
        // if the loop needs more cycles than were queued, it queues single
        // cycles and then the update and the next defect.  Same kernels,
        // same decisions, same bits as the loop above.  Outer steps
        // alternate between two norm slots, so queueing step k + 1 never
        // overwrites a norm the host has yet to read.
        q.bytes += x_zero ? 12.0 * n : 92.0 * n;  // the first defect
        for (int k = 1;; ++k) {
            const TraceRange step("mixed outer step");
            double s = 0.0;
            MG_HIPS(read_scalar(h, nslot(k), q.st, &s));
            st.rel_res = s / bn;
            if (k > 1 && st.n_hist < MG_HIST) st.res_hist[st.n_hist++] = s / bn;
            if (!std::isfinite(s) || s > 1e3 * bn) {
                result = fail(MG_ERR_NUMERIC, "residual diverged or became NaN");
                break;
            }
            if (o.fixed_cycles > 0) {
                if (k > o.fixed_cycles) break;
            } else {
                if (s <= o.rel_tol * bn) break;
                if (k > o.max_cycles) {
                    result = fail(MG_ERR_NOCONV, "no convergence within max_cycles");
                    break;
                }
            }
            if (s == 0.0) break;
            if (!queued) MG_HIPS(queue_step(k));
            const int slot = std::min(k, 8) - 1;
            int cycles = 0;
            bool done = false;
            MG_HIPS(read_iter(h, pred, q.st, &cycles, &done));
            if (!done) {
                // the queued update and defect were skipped: more cycles, then those
                while (!done) {
                    arm_iter(h);
                    Enq c1{q.st, 0.0};
                    MG_HIPS(run_unit(h, 4, o, false, graphs, c1, 1));
                    MG_HIPS(read_iter(h, cycles + 1, q.st, &cycles, &done));
                }
                MG_HIPS(queue_update_defect(k));
            }
            q.bytes += cycle_bytes * cycles + 20.0 * n + 92.0 * n;
            st.cycles += cycles;
            h->inner_pred[slot] = cycles;
            last = cycles;
            st.outer_steps = k;
            queued = ahead(k + 1);
            if (queued) MG_HIPS(queue_step(k + 1));
        }
        if (result == MG_OK) h->outer_prev = st.outer_steps;
    }
    if (!direct) {
        MG_HIPS(launch_copy<double>(F.x64, dev_x, n, q.st));
        q.bytes += 16.0 * n;
    } else if (zg && st.outer_steps == 0 && bn != 0.0) {
        // no update wrote the caller's x: the result is the zero guess
        MG_HIPS(launch_fill<double>(X64, n, 0.0, q.st));
        q.bytes += 8.0 * n;
    }
    // Later work on the caller's stream runs after the solve's.  The mixed
    // solve's last write of x came before the defect whose norm the host
    // has read, so only the others wait here for their final copy.
    MG_HIPS(hipEventRecord(gc->ev_out, q.st));
    MG_HIPS(hipStreamWaitEvent((hipStream_t)stream, gc->ev_out, 0));
    if (!direct || result != MG_OK || bn == 0.0) MG_HIPS(hipStreamSynchronize(q.st));
    st.status = result;
    st.alg_bytes = q.bytes;
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return result;
}

// ---------------------------------------------------------------- tiles
// Sec. 3: the thread-block partition of the GPU kernels is a runtime
// parameter.  For every level on which the hierarchy's V(2,2) cycle runs
// fused passes, time the FP32 pre- and post-smoothing passes (as the mixed
// solve runs them: the finest level's pre pass from a given iterate and its
// post pass with the residual norm, the others from zero and without) for
// each candidate tile and keep the fastest in the tile table under one
// problem.
extern "C" mg_status mg_hierarchy_autotune(mg_hierarchy* h, int reps, mg_tile_choice* out,
                                           int out_cap, int* n_out) {
    if (n_out) *n_out = 0;
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (!h->assembled) return fail(MG_ERR_INVALID, "hierarchy not assembled");
    if (reps < 1 || reps > 1000) return fail(MG_ERR_INVALID, "reps must lie in [1, 1000]");
    if (out_cap < 0 || (out_cap > 0 && !out)) return fail(MG_ERR_INVALID, "bad output array");
    const TraceRange trace("mg_hierarchy_autotune");
    static const int kRows[] = {4, 8, 12, 16, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256};
    static const int kWidths[] = {64, 128, 192, 256};
    MG_HIP(hipSetDevice(h->ctx->device));
    GraphCache* gc = cache(h);
    if (!gc->st) MG_HIP(hipStreamCreateWithFlags(&gc->st, hipStreamNonBlocking));
    hipStream_t st = gc->st;
    struct Guard {
        hipEvent_t a = nullptr, b = nullptr;
        ~Guard() {
            set_single_trial(0, 0, 0);
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } g;
    MG_HIP(hipEventCreate(&g.a));
    MG_HIP(hipEventCreate(&g.b));
    const float om = 0.7f;
    std::vector<mg_tile_choice> rows;
    for (int l = h->L; l > h->Lc; --l) {
        if (!(l > tail_max_level() || l == h->L)) continue;
        Level& v = h->lv[l];
        Level& c = h->lv[l - 1];
        const bool finest = l == h->L;
        auto pair = [&]() -> hipError_t {
            MG_TRY(launch_pre<float>(v, v.bands32, v.x32, !finest, v.b32, om, v.t32, c.b32,
                                     h->dmask, st));
            return launch_post<float>(v, v.bands32, v.t32, c.x32, v.b32, om, v.x32,
                                      finest ? h->partials : nullptr, h->scal, SC_USER, nullptr,
                                      st);
        };
        int best_rows = 0, best_bt = 0, best_cols = 0;
        float best_ms = 0.0f;
        // marching tiles (width x rows), then block tiles on small levels
        std::vector<std::array<int, 3>> cand;
        for (int bt : kWidths)
            for (int rh : kRows) cand.push_back({bt, rh, 0});
        if (v.N <= dev::BLK_MAX_N)
            for (int s = 1; s <= dev::BLK_SHAPES; ++s)
                cand.push_back({dev::BLK_THREADS, dev::block_rows(s), dev::BLK_COLS});
        for (const auto& c : cand) {
            {
                const int bt = c[0], rh = c[1];
                set_single_trial(v.N, rh, bt, c[2]);
                for (int w = 0; w < 2; ++w) MG_HIP(pair());
                MG_HIP(hipEventRecord(g.a, st));
                for (int r = 0; r < reps; ++r) MG_HIP(pair());
                MG_HIP(hipEventRecord(g.b, st));
                MG_HIP(hipEventSynchronize(g.b));
                float ms = 0.0f;
                MG_HIP(hipEventElapsedTime(&ms, g.a, g.b));
                if (!best_rows || ms < best_ms) {
                    best_rows = rh;
                    best_bt = bt;
                    best_cols = c[2];
                    best_ms = ms;
                }
            }
        }
        set_single_trial(0, 0, 0);
        tile_table_set(l, 1, best_rows, best_bt, best_cols);
        rows.push_back({l, 1, best_rows, best_bt / 64, best_cols, 1e3 * best_ms / reps});
    }
    const int n = std::min<int>(out_cap, (int)rows.size());
    for (int i = 0; i < n; ++i) out[i] = rows[i];
    if (n_out) *n_out = (int)rows.size();
    return MG_OK;
}
