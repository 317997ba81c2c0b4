// Operator kernels of degree 1: one wave per in-cell position (compile-time
// coefficients); the generic kernel is kept for comparison runs.
#include <cstdlib>
#include <string>

#include "apply_launch.hpp"

namespace smg {

template <>
hipError_t launch_apply_k<1>(bool f64, bool resid, const void* x, const void* b, void* y, const void* tab, int n,
                              hipStream_t st) {
    // measured on MI355X (64^3 cells, HBM-resident): the wave-per-position kernel is faster only for
    // FP32 at degree 1; elsewhere its FP64 constant/register pressure makes it spill, and the generic
    // kernel (runtime tables) is used.  STOKESMG_APPLY_KERNEL=generic|position overrides.
    static const int choice = [] {
        const char* s = std::getenv("STOKESMG_APPLY_KERNEL");
        if (!s) return 0;
        return std::string(s) == "position" ? 2 : 1;
    }();
    const bool position = choice == 2 || (choice == 0 && !f64 && 1 == 1);
    if (!position || (1 == 3 && f64)) {
        if (f64) return resid ? launch_generic<1, double, true>(x, b, y, tab, n, st)
                              : launch_generic<1, double, false>(x, b, y, tab, n, st);
        return resid ? launch_generic<1, float, true>(x, b, y, tab, n, st)
                     : launch_generic<1, float, false>(x, b, y, tab, n, st);
    }
    if (f64) return resid ? launch_wave_position<1, double, true>(x, b, y, n, st)
                          : launch_wave_position<1, double, false>(x, b, y, n, st);
    return resid ? launch_wave_position<1, float, true>(x, b, y, n, st)
                 : launch_wave_position<1, float, false>(x, b, y, n, st);
}

}  // namespace smg
