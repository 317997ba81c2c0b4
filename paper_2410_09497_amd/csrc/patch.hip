// Launcher of the vertex-patch local solves (one workgroup per patch of a colour).
#include "patch.hpp"

#include "patch_kernel.hpp"

namespace smg {

namespace {

// vertices v in 1..n-1 with v mod 2 == parity
int count_parity(int n, int parity) {
    const int first = parity ? 1 : 2;
    return (n - 1 >= first) ? (n - 1 - first) / 2 + 1 : 0;
}

template <int K, typename T, int NTP>
hipError_t launch_nt(void* x, const void* r, const void* ptab, int n, int colour, double rtol, int maxit,
                     int* counters, bool bonly, hipStream_t st) {
    const int cx = count_parity(n, colour & 1), cy = count_parity(n, (colour >> 1) & 1),
              cz = count_parity(n, (colour >> 2) & 1);
    const int grid = cx * cy * cz;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((patch_solve_kernel<K, T, NTP>), dim3(grid), dim3(PatchShape<K, NTP>::NT), 0, st,
                       static_cast<T*>(x),
                       static_cast<const T*>(r), static_cast<const T*>(ptab), n, colour, cx, cy, T(rtol), maxit,
                       counters, int(bonly));
    return hipGetLastError();
}

// threads per patch: the degree's default (PatchShape)
template <int K, typename T>
hipError_t launch(void* x, const void* r, const void* ptab, int n, int colour, double rtol, int maxit, int* counters,
                  bool bonly, hipStream_t st) {
    return launch_nt<K, T, 0>(x, r, ptab, n, colour, rtol, maxit, counters, bonly, st);
}

}  // namespace

hipError_t launch_patch_solve(int k, bool f64, void* x, const void* r, const void* ptab, int n, int colour,
                              double cg_rtol, int cg_max_it, int* counters, bool boundary_only, hipStream_t st) {
    switch (k) {
        case 1: return f64 ? launch<1, double>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st)
                           : launch<1, float>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st);
        case 2: return f64 ? launch<2, double>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st)
                           : launch<2, float>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st);
        case 3: return f64 ? launch<3, double>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st)
                           : launch<3, float>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st);
        case 4: return f64 ? launch<4, double>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st)
                           : launch<4, float>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st);
        case 5: return f64 ? launch<5, double>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st)
                           : launch<5, float>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace smg
