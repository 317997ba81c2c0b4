// Operator kernels of degree 5 (generic kernel: runtime stencil tables).
#include "apply_launch.hpp"

namespace smg {

template <>
hipError_t launch_apply_k<5>(bool f64, bool resid, const void* x, const void* b, void* y, const void* tab, int n,
                              hipStream_t st) {
    if (f64) return resid ? launch_generic<5, double, true>(x, b, y, tab, n, st)
                          : launch_generic<5, double, false>(x, b, y, tab, n, st);
    return resid ? launch_generic<5, float, true>(x, b, y, tab, n, st)
                 : launch_generic<5, float, false>(x, b, y, tab, n, st);
}

}  // namespace smg
