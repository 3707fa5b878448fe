// Solver drivers shared by the C ABI entry points.
#pragma once

#include "mg_internal.h"

namespace mg {

// Algorithmic HBM bytes of the kernels enqueued (see the byte model of each
// launcher in solve.hip); accumulated while enqueueing.
struct Enq {
    hipStream_t st;
    double bytes = 0.0;
    const double* guard = nullptr;  // device flag: the fused cycle's kernels skip while != 0
    RedCtl ctl{};                   // what the top-level residual norm's reduction decides
};

// One V(nu_pre, nu_post) cycle on level l with iterate x and right-hand side
// b of the level; x_zero states that x is logically zero on entry (its
// memory may hold stale values).  Levels below l use the hierarchy's own
// vectors.
template <typename T>
hipError_t enqueue_vcycle(mg_hierarchy* h, int l, T* x, const T* b, bool x_zero, int nu_pre,
                          int nu_post, double omega, Enq& q);

// The same cycle for V(2,2) from the fused smoothing passes; with partials
// the top-level pass also reduces the residual norm into scal[slot] (and
// into host[slot] when host is not null).
template <typename T>
hipError_t enqueue_vcycle_fused(mg_hierarchy* h, int l, T* x, const T* b, bool x_zero,
                                double omega, Enq& q, double* partials, double* scal, int slot,
                                double* host);

void destroy_graphs(mg_hierarchy* h);

}  // namespace mg
