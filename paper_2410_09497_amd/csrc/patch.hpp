#pragma once

#include <hip/hip_runtime.h>

namespace smg {

// Local solves of every patch of colour `colour` on a level with n cells per
// direction: x += R_j^T A_j^{-1} R_j r.  counters[0] += CG iterations,
// counters[1] += solves.  Degrees 1..5.  boundary_only: skip the patches
// whose cells touch no boundary face (those the learned solver handles).
hipError_t launch_patch_solve(int k, bool f64, void* x, const void* r, const void* ptab, int n, int colour,
                              double cg_rtol, int cg_max_it, int* counters, bool boundary_only, hipStream_t st);

}  // namespace smg
