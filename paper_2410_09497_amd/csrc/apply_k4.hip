// Operator kernels of degree 4 (generic kernel: runtime stencil tables).
#include "apply_launch.hpp"

namespace smg {

template <>
hipError_t launch_apply_k<4>(bool f64, bool resid, const void* x, const void* b, void* y, const void* tab, int n,
                              hipStream_t st) {
    if (f64) return resid ? launch_generic<4, double, true>(x, b, y, tab, n, st)
                          : launch_generic<4, double, false>(x, b, y, tab, n, st);
    return resid ? launch_generic<4, float, true>(x, b, y, tab, n, st)
                 : launch_generic<4, float, false>(x, b, y, tab, n, st);
}

}  // namespace smg
