#pragma once

#include <hip/hip_runtime.h>

namespace smg {

// y = K x (resid = false) or y = b - K x (resid = true) on one level with
// n cells per direction; `tab` is that level's device stencil table in the
// same dtype (used by the generic kernel).  Asynchronous on `st`.
hipError_t launch_apply(int k, bool f64, bool resid, const void* x, const void* b, void* y,
                        const void* tab, int n, hipStream_t st);

// one translation unit per degree (apply_k<K>.hip)
template <int K>
hipError_t launch_apply_k(bool f64, bool resid, const void* x, const void* b, void* y, const void* tab, int n,
                          hipStream_t st);

// cell layers per workgroup along z for the tile kernels (per degree and level size)
int apply_chunk_layers(int k, int n, int blocks_xy);

}  // namespace smg
