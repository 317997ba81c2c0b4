// Operator kernels of degree 1 (kernel choice in apply_launch.hpp).
#include "apply_launch.hpp"

namespace smg {

template <>
hipError_t launch_apply_k<1>(bool f64, bool resid, const void* x, const void* b, void* y, const void* tab, int n,
                              hipStream_t st) {
    return launch_degree<1>(f64, resid, x, b, y, tab, n, st);
}

}  // namespace smg
