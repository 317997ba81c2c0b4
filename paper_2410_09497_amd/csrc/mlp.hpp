// Smoother sweep with the selectable local solver, and the V-cycle driver
// shared by vcycle(), solve() and pair capture.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "handle.hpp"

namespace smg {

// training-pair sink of one capture call (rows *n .. cap-1 of X and T are free)
struct Capture {
    float* X;
    float* T;
    int64_t cap;
    int64_t* n;
};

// one sweep of the colourized smoother on `level`: per colour the residual,
// then the local solves (exact; learned on interior patches with the MLP
// solver; exact with pair capture when `cap` is given)
// One sweep of Alg. 2.  The residual vector and the CG counters come from the
// workspace unless `r` / `counters` are given (the no-allocation entry point
// passes its static scratch; counters may then be null).
int smooth_sweep(stokesmg* h, int level, bool f64, void* x, const void* b, hipStream_t st, const Capture* cap,
                 void* r = nullptr, unsigned long long* counters = nullptr, bool own_counters = false);

// the learned correction of every interior patch of one colour
int mlp_interior_solve(stokesmg* h, int level, bool f64, void* x, const void* r, int colour, hipStream_t st);

// x = P^{-1} b on the finest level (b, x in the cycle's precision); pairs are
// captured on the finest level when `cap` is given
int vcycle_run(stokesmg* h, bool f64, const void* b, void* x, hipStream_t st, const Capture* cap);

}  // namespace smg
