// C ABI: error reporting, contexts with a device-memory budget, device
// hierarchies (geometry, assembly) and the single-operator entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "device_ops.h"
#include "mg_internal.h"
#include "solve.h"

namespace mg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

mg_status fail(mg_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

int64_t vec_len(int64_t n) { return (n + 63) / 64 * 64; }

int64_t band_stride(int64_t n) { return (n + 1023) / 1024 * 1024 + 64; }

// Partial sums a reduction on the finest level of a level-L hierarchy can
// produce: FP64 band-product tiles, or the fused post pass's per-row ones.
static int64_t max_partials(int L) {
    const int64_t N = (int64_t(1) << L) + 1;
    const int64_t fused = fused_max_norm_parts(N);
    return std::max(stencil_blocks(N * N, 8), fused);
}

// The partials buffer: partials, padding to 64, then the segment sums of a
// two-stage reduction.
static int64_t partials_len(int L) {
    return (max_partials(L) + 63) / 64 * 64 + dev::RED_MAX_SEGS + 64;
}

// Bytes of every device array of a hierarchy, in allocation order.
static void hierarchy_arrays(int L, int Lc, std::vector<size_t>& sizes) {
    const int64_t nL = ((int64_t(1) << L) + 1) * ((int64_t(1) << L) + 1);
    sizes.push_back(2 * nL * sizeof(double));  // coords
    for (int l = Lc; l <= L; ++l) {
        const int64_t n = ((int64_t(1) << l) + 1) * ((int64_t(1) << l) + 1);
        const int64_t bs = band_stride(n), vl = vec_len(n);
        sizes.push_back(9 * bs * sizeof(double));
        sizes.push_back(9 * bs * sizeof(float));
        for (int v = 0; v < 3; ++v) sizes.push_back(vl * sizeof(double));
        // x32 and b32 back to back: together one FP64 vector (the Krylov
        // solver's z / q, which is never live with them)
        sizes.push_back(2 * vl * sizeof(float));
        sizes.push_back(vl * sizeof(float));
    }
    sizes.push_back(vec_len(nL) * sizeof(double));                    // d64
    sizes.push_back((PARTIALS_FRONT + partials_len(L)) * sizeof(double));  // ticket + partials
    sizes.push_back(64 * sizeof(double));                             // scal
    const size_t nc = ((size_t(1) << Lc) + 1) * ((size_t(1) << Lc) + 1);
    sizes.push_back(nc * nc * sizeof(double));                         // chol (m <= nc)
    sizes.push_back(64);                                              // flag
}

static size_t round_alloc(size_t b) { return (b + 4095) / 4096 * 4096; }

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static mg_status check_level(const mg_hierarchy* h, int level) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (level < h->Lc || level > h->L)
        return fail(MG_ERR_INVALID, "level " + std::to_string(level) + " outside [" +
                                        std::to_string(h->Lc) + ", " + std::to_string(h->L) + "]");
    if (!h->assembled) return fail(MG_ERR_INVALID, "hierarchy not assembled");
    return MG_OK;
}

static mg_status set_device(const mg_hierarchy* h) {
    MG_HIP(hipSetDevice(h->ctx->device));
    return MG_OK;
}

static_assert(MG_MAX_COARSE_LEVEL == dev::COARSE_MAX_LEVEL, "coarse level bound");

dev::CoarseSolver coarse_solver(const mg_hierarchy* h) {
    dev::CoarseSolver cs{};
    cs.chol = h->chol;
    cs.bands = h->lv[h->Lc].bands64;
    cs.bs = h->lv[h->Lc].bs;
    cs.m = h->m;
    cs.dmask = h->dmask;
    cs.cg = h->coarse_cg;
    cs.max_iter = h->coarse_max_iter;
    cs.tol = h->coarse_tol;
    return cs;
}

}  // namespace mg

using namespace mg;

bool mg_context::reserve(size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    if (budget != 0 && in_use + bytes > budget) return false;
    in_use += bytes;
    high_water = std::max(high_water, in_use);
    return true;
}

void mg_context::release(size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    in_use -= std::min(in_use, bytes);
}

extern "C" {

void mg_default_opts(mg_solve_opts* o) {
    if (!o) return;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->omega = 0.7;
    o->rel_tol = 1e-8;
    o->max_cycles = 100;
    o->precision = MG_PREC_FP64;
    o->inner_reduction = 1e-2;
    o->inner_max_cycles = 8;
    o->fixed_cycles = 0;
    o->use_graph = 1;
    o->krylov = 0;
    o->zero_guess = 0;
}

const char* mg_last_error(void) { return g_last_error.c_str(); }

const char* mg_status_string(mg_status s) {
    switch (s) {
        case MG_OK: return "MG_OK";
        case MG_ERR_INVALID: return "MG_ERR_INVALID";
        case MG_ERR_NOMEM: return "MG_ERR_NOMEM";
        case MG_ERR_NOCONV: return "MG_ERR_NOCONV";
        case MG_ERR_NUMERIC: return "MG_ERR_NUMERIC";
        case MG_ERR_DEVICE: return "MG_ERR_DEVICE";
        case MG_ERR_BUSY: return "MG_ERR_BUSY";
    }
    return "MG_ERR_UNKNOWN";
}

mg_status mg_context_create(int device, size_t budget, mg_context** out) {
    if (!out) return fail(MG_ERR_INVALID, "null output pointer");
    *out = nullptr;
    int count = 0;
    MG_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(MG_ERR_INVALID, "device " + std::to_string(device) + " not present");
    MG_HIP(hipSetDevice(device));
    mg_context* c = new (std::nothrow) mg_context();
    if (!c) return fail(MG_ERR_NOMEM, "host allocation failed");
    c->device = device;
    c->budget = budget;
    *out = c;
    return MG_OK;
}

mg_status mg_context_destroy(mg_context* ctx) {
    if (!ctx) return fail(MG_ERR_INVALID, "null context");
    if (ctx->blas_scratch || ctx->blas_host) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        if (ctx->blas_scratch) (void)hipFree(ctx->blas_scratch);
        if (ctx->blas_host) (void)hipHostFree(ctx->blas_host);
    }
    delete ctx;
    return MG_OK;
}

mg_status mg_context_memory(const mg_context* ctx, size_t* in_use, size_t* high_water) {
    if (!ctx) return fail(MG_ERR_INVALID, "null context");
    mg_context* c = const_cast<mg_context*>(ctx);
    std::lock_guard<std::mutex> g(c->mu);
    if (in_use) *in_use = c->in_use;
    if (high_water) *high_water = c->high_water;
    return MG_OK;
}

size_t mg_hierarchy_bytes(int L, int Lc) {
    if (L < 1 || L > MG_MAX_LEVEL || Lc < 1 || Lc > std::min(L, MG_MAX_COARSE_LEVEL)) return 0;
    std::vector<size_t> sizes;
    hierarchy_arrays(L, Lc, sizes);
    size_t total = 0;
    for (size_t s : sizes) total += round_alloc(s);
    return total;
}

static void free_arrays(mg_hierarchy* h) {
    for (void* p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    if (h->host_scal) (void)hipHostFree(h->host_scal);
    h->host_scal = nullptr;
}

mg_status mg_hierarchy_create(mg_context* ctx, int L, int Lc, double jitter, uint64_t seed,
                              const double* host_xy, mg_hierarchy** out) {
    return mg_hierarchy_create_bc(ctx, L, Lc, jitter, seed, host_xy, MG_ALL_DIRICHLET, out);
}

mg_status mg_hierarchy_create_bc(mg_context* ctx, int L, int Lc, double jitter, uint64_t seed,
                                 const double* host_xy, int dirichlet_sides, mg_hierarchy** out) {
    if (!out) return fail(MG_ERR_INVALID, "null output pointer");
    *out = nullptr;
    if (!ctx) return fail(MG_ERR_INVALID, "null context");
    if (dirichlet_sides < 1 || dirichlet_sides > MG_ALL_DIRICHLET)
        return fail(MG_ERR_INVALID, "dirichlet_sides=" + std::to_string(dirichlet_sides) +
                                        " outside [1, 15]: at least one side must be Dirichlet");
    if (L < 1 || L > MG_MAX_LEVEL)
        return fail(MG_ERR_INVALID, "level L=" + std::to_string(L) + " outside [1, 14]");
    if (Lc < 1 || Lc > std::min(L, MG_MAX_COARSE_LEVEL))
        return fail(MG_ERR_INVALID, "coarse level " + std::to_string(Lc) + " outside [1, min(L, 4)]");
    if (!(jitter >= 0.0 && jitter < 0.5))
        return fail(MG_ERR_INVALID, "jitter must lie in [0, 0.5)");
    MG_HIP(hipSetDevice(ctx->device));
    std::vector<size_t> sizes;
    hierarchy_arrays(L, Lc, sizes);
    size_t total = 0;
    for (size_t s : sizes) total += round_alloc(s);
    if (!ctx->reserve(total))
        return fail(MG_ERR_NOMEM, "hierarchy L=" + std::to_string(L) + " needs " +
                                      std::to_string(total) + " bytes, over the context budget");
    mg_hierarchy* h = new (std::nothrow) mg_hierarchy();
    if (!h) {
        ctx->release(total);
        return fail(MG_ERR_NOMEM, "host allocation failed");
    }
    h->ctx = ctx;
    h->L = L;
    h->Lc = Lc;
    h->dmask = dirichlet_sides;
    h->charged = total;
    std::vector<void*> ptrs;
    for (size_t s : sizes) {
        void* p = nullptr;
        if (hipMalloc(&p, round_alloc(s)) != hipSuccess) {
            (void)hipGetLastError();
            for (void* q : ptrs) (void)hipFree(q);
            ctx->release(total);
            delete h;
            return fail(MG_ERR_NOMEM, "hipMalloc failed for hierarchy L=" + std::to_string(L));
        }
        ptrs.push_back(p);
    }
    h->allocs = ptrs;
    for (size_t a = 0; a < ptrs.size(); ++a) {
        if (hipMemset(ptrs[a], 0, round_alloc(sizes[a])) != hipSuccess) {
            free_arrays(h);
            ctx->release(total);
            delete h;
            return fail(MG_ERR_DEVICE, "hipMemset failed");
        }
    }
    size_t a = 0;
    h->coords = (double*)ptrs[a++];
    for (int l = Lc; l <= L; ++l) {
        Level& lv = h->lv[l];
        lv.l = l;
        lv.N = (1 << l) + 1;
        lv.n = (int64_t)lv.N * lv.N;
        lv.bs = band_stride(lv.n);
        lv.bands64 = (double*)ptrs[a++];
        lv.bands32 = (float*)ptrs[a++];
        lv.x64 = (double*)ptrs[a++];
        lv.b64 = (double*)ptrs[a++];
        lv.t64 = (double*)ptrs[a++];
        lv.x32 = (float*)ptrs[a++];
        lv.b32 = lv.x32 + vec_len(lv.n);
        lv.t32 = (float*)ptrs[a++];
    }
    h->d64 = (double*)ptrs[a++];
    h->partials = (double*)ptrs[a++] + PARTIALS_FRONT;
    h->n_partials = partials_len(L);
    h->scal = (double*)ptrs[a++];
    h->chol = (double*)ptrs[a++];
    h->flag = (int*)ptrs[a++];
    {
        const int Nc = (1 << Lc) + 1;
        h->m = 0;
        for (int j = 0; j < Nc; ++j)
            for (int i = 0; i < Nc; ++i) h->m += dev::is_dirichlet(Nc, i, j, h->dmask) ? 0 : 1;
    }
    if (hipHostMalloc((void**)&h->host_scal, 64 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        h->host_scal = nullptr;
        free_arrays(h);
        ctx->release(total);
        delete h;
        return fail(MG_ERR_NOMEM, "pinned host allocation failed");
    }
    const int64_t nL = h->lv[L].n;
    hipError_t e;
    if (host_xy)
        e = hipMemcpy(h->coords, host_xy, 2 * nL * sizeof(double), hipMemcpyHostToDevice);
    else
        e = launch_coords(h->coords, L, jitter, seed, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);  // null stream only: others keep running
    if (e != hipSuccess) {
        free_arrays(h);
        ctx->release(total);
        delete h;
        return fail(MG_ERR_DEVICE, std::string("geometry: ") + hipGetErrorString(e));
    }
    *out = h;
    return MG_OK;
}

mg_status mg_hierarchy_assemble(mg_hierarchy* h, void* stream) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (mg_status s = set_device(h)) return s;
    hipStream_t st = (hipStream_t)stream;
    MG_HIP(launch_assemble(h->coords, h->lv, h->Lc, h->L, h->dmask, st));
    MG_HIP(launch_chol_factor(h->lv[h->Lc], h->dmask, h->chol, h->flag, st));
    int flag = 0;
    MG_HIP(hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    if (flag) return fail(MG_ERR_NUMERIC, "coarse-grid block is not positive definite");
    h->assembled = true;
    return MG_OK;
}

mg_status mg_hierarchy_set_coarse_solver(mg_hierarchy* h, int solver, double tol, int max_iter) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (solver != MG_COARSE_CHOLESKY && solver != MG_COARSE_CG)
        return fail(MG_ERR_INVALID, "unknown coarse solver " + std::to_string(solver));
    if (solver == MG_COARSE_CG) {
        if (!(tol >= 0.0 && tol < 1.0))
            return fail(MG_ERR_INVALID, "coarse CG tolerance must lie in [0, 1)");
        if (max_iter < 1 || max_iter > MG_COARSE_CG_MAX_ITER)
            return fail(MG_ERR_INVALID, "coarse CG step limit outside [1, " +
                                            std::to_string(MG_COARSE_CG_MAX_ITER) + "]");
    }
    if (mg_status s = set_device(h)) return s;
    // captured cycles hold the old solver in their kernel arguments
    MG_HIP(hipDeviceSynchronize());
    destroy_graphs(h);
    h->coarse_cg = solver == MG_COARSE_CG;
    if (h->coarse_cg) {
        h->coarse_tol = tol;
        h->coarse_max_iter = max_iter;
    }
    return MG_OK;
}

mg_status mg_hierarchy_destroy(mg_hierarchy* h) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    (void)hipSetDevice(h->ctx->device);
    (void)hipDeviceSynchronize();
    destroy_graphs(h);
    free_arrays(h);
    h->ctx->release(h->charged);
    delete h;
    return MG_OK;
}

mg_status mg_hierarchy_info(const mg_hierarchy* h, int* L, int* Lc, int64_t* n) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (L) *L = h->L;
    if (Lc) *Lc = h->Lc;
    if (n) *n = h->lv[h->L].n;
    return MG_OK;
}

mg_status mg_get_bands(const mg_hierarchy* h, int level, mg_dtype dtype, void* host_out) {
    if (mg_status s = check_level(h, level)) return s;
    if (!host_out) return fail(MG_ERR_INVALID, "null output");
    if (mg_status s = set_device(h)) return s;
    const Level& lv = h->lv[level];
    const size_t es = dtype == MG_F64 ? 8 : 4;
    const char* base = dtype == MG_F64 ? (const char*)lv.bands64 : (const char*)lv.bands32;
    for (int k = 0; k < 9; ++k)
        MG_HIP(hipMemcpy((char*)host_out + k * lv.n * es, base + k * lv.bs * es, lv.n * es,
                         hipMemcpyDeviceToHost));
    return MG_OK;
}

mg_status mg_get_coords(const mg_hierarchy* h, int level, double* host_out) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (level < h->Lc || level > h->L) return fail(MG_ERR_INVALID, "level out of range");
    if (!host_out) return fail(MG_ERR_INVALID, "null output");
    if (mg_status s = set_device(h)) return s;
    const int N = (1 << level) + 1, Nf = (1 << h->L) + 1, sd = 1 << (h->L - level);
    std::vector<double> all((size_t)2 * Nf * Nf);
    MG_HIP(hipMemcpy(all.data(), h->coords, all.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            const size_t pf = (size_t)(j * sd) * Nf + (size_t)(i * sd);
            host_out[2 * ((size_t)j * N + i)] = all[2 * pf];
            host_out[2 * ((size_t)j * N + i) + 1] = all[2 * pf + 1];
        }
    return MG_OK;
}

mg_status mg_rhs_sinsin(const mg_hierarchy* h, double* dev_b, void* stream) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (!dev_b) return fail(MG_ERR_INVALID, "null b");
    if (h->dmask != MG_ALL_DIRICHLET)
        return fail(MG_ERR_INVALID, "the sin-sin load vector needs Dirichlet conditions on every side");
    if (mg_status s = set_device(h)) return s;
    MG_HIP(launch_rhs_sinsin(h->coords, h->lv[h->L].N, dev_b, (hipStream_t)stream));
    return MG_OK;
}

mg_status mg_rhs_uniform(const mg_hierarchy* h, uint64_t seed, double* dev_b, void* stream) {
    if (!h) return fail(MG_ERR_INVALID, "null hierarchy");
    if (!dev_b) return fail(MG_ERR_INVALID, "null b");
    if (mg_status s = set_device(h)) return s;
    MG_HIP(launch_rhs_uniform(h->lv[h->L].N, seed, h->dmask, dev_b, nullptr, (hipStream_t)stream));
    return MG_OK;
}

mg_status mg_spmv(const mg_hierarchy* h, int level, mg_dtype dtype, const void* x, void* y,
                  void* stream) {
    if (mg_status s = check_level(h, level)) return s;
    if (!x || !y || !aligned16(x) || !aligned16(y))
        return fail(MG_ERR_INVALID, "x and y must be non-null and 16-byte aligned");
    if (x == y) return fail(MG_ERR_INVALID, "x and y must not alias");
    if (mg_status s = set_device(h)) return s;
    const Level& lv = h->lv[level];
    hipStream_t st = (hipStream_t)stream;
    if (dtype == MG_F64)
        MG_HIP(launch_spmv<double>(lv, lv.bands64, (const double*)x, (double*)y, st));
    else
        MG_HIP(launch_spmv<float>(lv, lv.bands32, (const float*)x, (float*)y, st));
    return MG_OK;
}

mg_status mg_defect(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                    const void* x, void* d, double* host_norm, void* stream) {
    if (mg_status s = check_level(h, level)) return s;
    if (!b || !x || !aligned16(b) || !aligned16(x) || (d && !aligned16(d)))
        return fail(MG_ERR_INVALID, "b, x, d must be 16-byte aligned device pointers");
    if (!d && !host_norm) return fail(MG_ERR_INVALID, "nothing to compute (d and norm null)");
    if (d && (d == x || d == b)) return fail(MG_ERR_INVALID, "d must not alias b or x");
    if (mg_status s = set_device(h)) return s;
    const Level& lv = h->lv[level];
    hipStream_t st = (hipStream_t)stream;
    mg_hierarchy* hm = const_cast<mg_hierarchy*>(h);
    double* part = host_norm ? hm->partials : nullptr;
    if (dtype == MG_F64)
        MG_HIP(launch_defect<double>(lv, lv.bands64, (const double*)b, (const double*)x,
                                     (double*)d, part, hm->scal, SC_USER, hm->host_scal, st));
    else
        MG_HIP(launch_defect<float>(lv, lv.bands32, (const float*)b, (const float*)x, (float*)d,
                                    part, hm->scal, SC_USER, hm->host_scal, st));
    if (host_norm) {
        MG_HIP(hipStreamSynchronize(st));
        *host_norm = ((const volatile double*)hm->host_scal)[SC_USER + 1];
    }
    return MG_OK;
}

mg_status mg_smooth(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b, void* x,
                    int sweeps, double omega, void* stream) {
    if (mg_status s = check_level(h, level)) return s;
    if (!b || !x || !aligned16(b) || !aligned16(x) || b == x)
        return fail(MG_ERR_INVALID, "b, x must be distinct 16-byte aligned device pointers");
    if (sweeps < 0) return fail(MG_ERR_INVALID, "negative sweep count");
    if (mg_status s = set_device(h)) return s;
    const Level& lv = h->lv[level];
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < sweeps; ++s) {
        if (dtype == MG_F64) {
            MG_HIP(launch_jacobi<double>(lv, lv.bands64, (const double*)b, (const double*)x,
                                         lv.t64, omega, st));
            MG_HIP(launch_copy<double>(lv.t64, (double*)x, lv.n, st));
        } else {
            MG_HIP(launch_jacobi<float>(lv, lv.bands32, (const float*)b, (const float*)x,
                                        lv.t32, (float)omega, st));
            MG_HIP(launch_copy<float>(lv.t32, (float*)x, lv.n, st));
        }
    }
    return MG_OK;
}

mg_status mg_jacobi(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                    const void* x, void* x_out, double omega, void* stream) {
    if (mg_status s = check_level(h, level)) return s;
    if (!b || !x || !x_out || !aligned16(b) || !aligned16(x) || !aligned16(x_out))
        return fail(MG_ERR_INVALID, "b, x, x_out must be 16-byte aligned device pointers");
    if (x_out == x || x_out == b) return fail(MG_ERR_INVALID, "x_out must not alias x or b");
    if (mg_status s = set_device(h)) return s;
    const Level& lv = h->lv[level];
    hipStream_t st = (hipStream_t)stream;
    if (dtype == MG_F64)
        MG_HIP(launch_jacobi<double>(lv, lv.bands64, (const double*)b, (const double*)x,
                                     (double*)x_out, omega, st));
    else
        MG_HIP(launch_jacobi<float>(lv, lv.bands32, (const float*)b, (const float*)x,
                                    (float*)x_out, (float)omega, st));
    return MG_OK;
}

mg_status mg_pre_smooth(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                        const void* x, int x_zero, double omega, void* x2, void* b_c,
                        void* stream) {
    if (mg_status s = check_level(h, level)) return s;
    if (level <= h->Lc) return fail(MG_ERR_INVALID, "no coarser level below level");
    if (!b || !x2 || !b_c || (!x_zero && !x))
        return fail(MG_ERR_INVALID, "null vector");
    if (x2 == b || (!x_zero && x2 == x) || b_c == x2)
        return fail(MG_ERR_INVALID, "x2 must not alias x, b or b_c");
    if (mg_status s = set_device(h)) return s;
    const Level& lv = h->lv[level];
    hipStream_t st = (hipStream_t)stream;
    if (dtype == MG_F64)
        MG_HIP(launch_pre<double>(lv, lv.bands64, (const double*)x, x_zero != 0, (const double*)b,
                                  omega, (double*)x2, (double*)b_c, h->dmask, st));
    else
        MG_HIP(launch_pre<float>(lv, lv.bands32, (const float*)x, x_zero != 0, (const float*)b,
                                 (float)omega, (float*)x2, (float*)b_c, h->dmask, st));
    return MG_OK;
}

mg_status mg_post_smooth(const mg_hierarchy* h, int level, mg_dtype dtype, const void* b,
                         const void* x, const void* x_c, double omega, void* x_out,
                         double* host_norm, void* stream) {
    if (mg_status s = check_level(h, level)) return s;
    if (level <= h->Lc) return fail(MG_ERR_INVALID, "no coarser level below level");
    if (!b || !x || !x_c || !x_out) return fail(MG_ERR_INVALID, "null vector");
    if (x_out == x || x_out == x_c || x_out == b)
        return fail(MG_ERR_INVALID, "x_out must not alias x, x_c or b");
    if (mg_status s = set_device(h)) return s;
    const Level& lv = h->lv[level];
    hipStream_t st = (hipStream_t)stream;
    mg_hierarchy* hm = const_cast<mg_hierarchy*>(h);
    double* part = host_norm ? hm->partials : nullptr;
    if (dtype == MG_F64)
        MG_HIP(launch_post<double>(lv, lv.bands64, (const double*)x, (const double*)x_c,
                                   (const double*)b, omega, (double*)x_out, part, hm->scal, SC_USER,
                                   hm->host_scal, st));
    else
        MG_HIP(launch_post<float>(lv, lv.bands32, (const float*)x, (const float*)x_c,
                                  (const float*)b, (float)omega, (float*)x_out, part, hm->scal,
                                  SC_USER, hm->host_scal, st));
    if (host_norm) {
        MG_HIP(hipStreamSynchronize(st));
        *host_norm = ((const volatile double*)hm->host_scal)[SC_USER + 1];
    }
    return MG_OK;
}

mg_status mg_restrict(const mg_hierarchy* h, int fine_level, mg_dtype dtype, const void* d_f,
                      void* b_c, void* stream) {
    if (mg_status s = check_level(h, fine_level)) return s;
    if (fine_level <= h->Lc) return fail(MG_ERR_INVALID, "no coarser level below fine_level");
    if (!d_f || !b_c) return fail(MG_ERR_INVALID, "null vector");
    if (mg_status s = set_device(h)) return s;
    const int Nf = h->lv[fine_level].N;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == MG_F64)
        MG_HIP(launch_restrict<double>(Nf, (const double*)d_f, (double*)b_c, h->dmask, st));
    else
        MG_HIP(launch_restrict<float>(Nf, (const float*)d_f, (float*)b_c, h->dmask, st));
    return MG_OK;
}

mg_status mg_prolong(const mg_hierarchy* h, int fine_level, mg_dtype dtype, const void* x_c,
                     void* x_f, void* stream) {
    if (mg_status s = check_level(h, fine_level)) return s;
    if (fine_level <= h->Lc) return fail(MG_ERR_INVALID, "no coarser level below fine_level");
    if (!x_c || !x_f) return fail(MG_ERR_INVALID, "null vector");
    if (mg_status s = set_device(h)) return s;
    const int Nf = h->lv[fine_level].N;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == MG_F64)
        MG_HIP(launch_prolong<double>(Nf, (const double*)x_c, (double*)x_f, st));
    else
        MG_HIP(launch_prolong<float>(Nf, (const float*)x_c, (float*)x_f, st));
    return MG_OK;
}

mg_status mg_coarse_solve(const mg_hierarchy* h, mg_dtype dtype, const void* b, void* x,
                          void* stream) {
    if (mg_status s = check_level(h, h ? h->Lc : 1)) return s;
    if (!b || !x) return fail(MG_ERR_INVALID, "null vector");
    if (mg_status s = set_device(h)) return s;
    hipStream_t st = (hipStream_t)stream;
    const int Nc = h->lv[h->Lc].N;
    if (dtype == MG_F64)
        MG_HIP(launch_coarse<double>(coarse_solver(h), Nc, (const double*)b, (double*)x, st));
    else
        MG_HIP(launch_coarse<float>(coarse_solver(h), Nc, (const float*)b, (float*)x, st));
    return MG_OK;
}

}  // extern "C"
