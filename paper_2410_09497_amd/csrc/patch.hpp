#pragma once

#include <hip/hip_runtime.h>

namespace smg {

// Local solves of every patch of colour `colour` on a level with n cells per
// direction: x += R_j^T A_j^{-1} R_j r.  counters[0] += CG iterations,
// counters[1] += solves.  Degrees 1..5.  boundary_only: skip the patches
// whose cells touch no boundary face (those the learned solver handles).
hipError_t launch_patch_solve(int k, bool f64, void* x, const void* r, const void* ptab, int n, int colour,
                              double cg_rtol, int cg_max_it, unsigned long long* counters, bool boundary_only, hipStream_t st);

// launch_patch_solve for an FP32 level (degrees 1..3) with the in-plane eigenbasis products of the fast
// diagonalization on the matrix cores (BF16 operands, FP32 accumulation); every patch of the colour.
hipError_t launch_patch_solve_mf(int k, void* x, const void* r, const void* ptab, int n, int colour, double cg_rtol,
                                 int cg_max_it, unsigned long long* counters, hipStream_t st);

// The interior patches p0 .. p0 + count - 1 of colour `colour` (the order of the network's batches), each
// Schur CG started from the pressure the network predicted: y rows hold (U, h P) / s, s the input scales
// (float, from the MLP workspace).  Same tolerance test as the cold start (relative to the cold-start
// residual), so the result is the same exact local solve up to that tolerance.
hipError_t launch_patch_solve_warm(int k, bool f64, void* x, const void* r, const void* ptab, int n, int colour,
                                   double cg_rtol, int cg_max_it, unsigned long long* counters, int p0, int count, const float* y,
                                   int ldy, const float* s, hipStream_t st);

}  // namespace smg
