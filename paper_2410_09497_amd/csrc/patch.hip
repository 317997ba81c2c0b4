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

// interior vertices (2 <= v <= n-2) with v mod 2 == parity
int count_interior(int n, int parity) {
    const int first = parity ? 3 : 2;
    return (n - 2 >= first) ? (n - 2 - first) / 2 + 1 : 0;
}

template <int K, typename T, int NTP, bool MF = false>
hipError_t launch_nt(void* x, const void* r, const void* ptab, int n, int colour, double rtol, int maxit,
                     unsigned long long* counters, bool bonly, const PatchWarm* warm, int warm_count, hipStream_t st) {
    const int cx = count_parity(n, colour & 1), cy = count_parity(n, (colour >> 1) & 1),
              cz = count_parity(n, (colour >> 2) & 1);
    const int grid = warm ? warm_count : cx * cy * cz;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((patch_solve_kernel<K, T, NTP, MF>), dim3(grid), dim3(PatchShape<K, NTP>::NT), 0, st,
                       static_cast<T*>(x),
                       static_cast<const T*>(r), static_cast<const T*>(ptab), n, colour, cx, cy, T(rtol), maxit,
                       counters, int(bonly), warm ? *warm : PatchWarm{});
    return hipGetLastError();
}

// threads per patch: the degree's default (PatchShape)
template <int K, typename T>
hipError_t launch(void* x, const void* r, const void* ptab, int n, int colour, double rtol, int maxit, unsigned long long* counters,
                  bool bonly, hipStream_t st, const PatchWarm* warm = nullptr, int warm_count = 0) {
    return launch_nt<K, T, 0>(x, r, ptab, n, colour, rtol, maxit, counters, bonly, warm, warm_count, st);
}

template <typename T>
hipError_t launch_k(int k, void* x, const void* r, const void* ptab, int n, int colour, double rtol, int maxit,
                    unsigned long long* counters, bool bonly, hipStream_t st, const PatchWarm* warm, int warm_count) {
    switch (k) {
        case 1: return launch<1, T>(x, r, ptab, n, colour, rtol, maxit, counters, bonly, st, warm, warm_count);
        case 2: return launch<2, T>(x, r, ptab, n, colour, rtol, maxit, counters, bonly, st, warm, warm_count);
        case 3: return launch<3, T>(x, r, ptab, n, colour, rtol, maxit, counters, bonly, st, warm, warm_count);
        case 4: return launch<4, T>(x, r, ptab, n, colour, rtol, maxit, counters, bonly, st, warm, warm_count);
        case 5: return launch<5, T>(x, r, ptab, n, colour, rtol, maxit, counters, bonly, st, warm, warm_count);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_patch_solve(int k, bool f64, void* x, const void* r, const void* ptab, int n, int colour,
                              double cg_rtol, int cg_max_it, unsigned long long* counters, bool boundary_only, hipStream_t st) {
    return f64 ? launch_k<double>(k, x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st, nullptr, 0)
               : launch_k<float>(k, x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, boundary_only, st, nullptr, 0);
}

hipError_t launch_patch_solve_mf(int k, void* x, const void* r, const void* ptab, int n, int colour, double cg_rtol,
                                 int cg_max_it, unsigned long long* counters, hipStream_t st) {
    switch (k) {
        case 1: return launch_nt<1, float, 0, true>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, false, nullptr, 0, st);
        case 2: return launch_nt<2, float, 0, true>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, false, nullptr, 0, st);
        case 3: return launch_nt<3, float, 0, true>(x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, false, nullptr, 0, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_patch_solve_warm(int k, bool f64, void* x, const void* r, const void* ptab, int n, int colour,
                                   double cg_rtol, int cg_max_it, unsigned long long* counters, int p0, int count, const float* y,
                                   int ldy, const float* s, hipStream_t st) {
    PatchWarm w;
    w.y = y;
    w.s = s;
    w.ldy = ldy;
    w.p0 = p0;
    for (int d = 0; d < 3; ++d) w.cnt[d] = count_interior(n, (colour >> d) & 1);
    return f64 ? launch_k<double>(k, x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, false, st, &w, count)
               : launch_k<float>(k, x, r, ptab, n, colour, cg_rtol, cg_max_it, counters, false, st, &w, count);
}

}  // namespace smg
