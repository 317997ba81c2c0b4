// Multigrid / Krylov vector kernels (launchers).  All asynchronous on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

namespace smg {

// out (+)= T_3D in, with T_3D the tensor product of 1D row lists: the
// continuous list in a component's own direction, the DG list otherwise
// (prolongation: out fine, in coarse; restriction: the transposed lists).
// Applied as three 1D passes (x, y, z) through two intermediates in `tmp`,
// which needs room for 3/4 of the larger level's vector plus 256 bytes
// (device; distinct from in and out).
hipError_t launch_transfer(bool f64, bool acc, const void* in, void* out, int N1_out, int N1_in, const int* dgi,
                           const double* dgw, int wd, const int* cni, const double* cnw, int wc, void* tmp,
                           hipStream_t st);

// x = A b, A dense FP64 (n x n row-major), b and x in FP64 or FP32
hipError_t launch_coarse_gemv(bool f64, const double* A, const void* b, void* x, int n, hipStream_t st);

// b = a converted FP64 -> FP32 (from_f64) or FP32 -> FP64
hipError_t launch_convert(bool from_f64, const void* a, void* b, size_t n, hipStream_t st);

hipError_t launch_zero(bool f64, void* a, size_t n, hipStream_t st);

// out[j] = V_j . w (j < nv, V_j = V + j ld), two-stage reduction through
// `partial` (nblocks x nv)
hipError_t launch_multidot(const double* V, size_t ld, const double* w, int nv, size_t n, double* partial, int nblocks,
                           double* out, hipStream_t st);

// w = alpha w + csign sum_j c_j V_j (c on the device)
hipError_t launch_multiaxpy(const double* V, size_t ld, const double* c, int nv, double csign, double alpha, double* w,
                            size_t n, hipStream_t st);

// subtract the integral mean of the pressure block (weights h^3 w_a w_b w_c);
// scratch holds kMomentBlocks + 1 doubles
constexpr int kMomentBlocks = 1024;
hipError_t launch_normalize_pressure(bool f64, void* x, int N1, int m, const double* wg, double h, double* scratch,
                                     hipStream_t st);

}  // namespace smg
