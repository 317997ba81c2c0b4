// Dispatch of the fused operator / residual kernels by degree.
#include "apply.hpp"

namespace smg {

hipError_t launch_apply(int k, bool f64, bool resid, const void* x, const void* b, void* y, const void* tab,
                        int n, hipStream_t st) {
    switch (k) {
        case 1: return launch_apply_k<1>(f64, resid, x, b, y, tab, n, st);
        case 2: return launch_apply_k<2>(f64, resid, x, b, y, tab, n, st);
        case 3: return launch_apply_k<3>(f64, resid, x, b, y, tab, n, st);
        case 4: return launch_apply_k<4>(f64, resid, x, b, y, tab, n, st);
        case 5: return launch_apply_k<5>(f64, resid, x, b, y, tab, n, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace smg
