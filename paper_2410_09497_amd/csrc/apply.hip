// Launchers of the fused operator / residual kernel (one instantiation per
// degree, dtype and mode).
#include "apply.hpp"

#include <algorithm>
#include <cstdlib>

#include "apply_kernel.hpp"

namespace smg {

namespace {

// Tile (cells in x, cells in y) per degree: positions per tile side are
// multiples of k+1; chosen so that a workgroup is 144..288 threads.
template <int K> struct TileOf;
template <> struct TileOf<1> { static constexpr int CX = 8, CY = 8; };
template <> struct TileOf<2> { static constexpr int CX = 8, CY = 4; };
template <> struct TileOf<3> { static constexpr int CX = 4, CY = 4; };
template <> struct TileOf<4> { static constexpr int CX = 4, CY = 2; };
template <> struct TileOf<5> { static constexpr int CX = 4, CY = 2; };

int choose_cz(int n, int blocks_xy) {
    if (const char* s = std::getenv("STOKESMG_APPLY_CZ")) {
        int v = std::atoi(s);
        if (v > 0) return std::min(v, n);
    }
    // aim at >= 2048 workgroups (8 per CU) while keeping chunks >= 4 layers
    int chunks = (2048 + blocks_xy - 1) / blocks_xy;
    int cz = (n + chunks - 1) / chunks;
    cz = std::max(cz, std::min(4, n));
    return std::min(cz, n);
}

template <int K, typename T, bool RESID>
hipError_t launch(const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    constexpr int CX = TileOf<K>::CX, CY = TileOf<K>::CY;
    using S = ApplyShape<K, CX, CY>;
    const int N1 = n * S::M;
    const int tiles_x = (N1 + S::TX - 1) / S::TX;
    const int tiles_y = (N1 + S::TY - 1) / S::TY;
    const int cz = choose_cz(n, tiles_x * tiles_y);
    const int nzc = (n + cz - 1) / cz;
    const int grid = tiles_x * tiles_y * nzc;
    hipLaunchKernelGGL((stokes_apply_kernel<K, T, CX, CY, RESID>), dim3(grid), dim3(S::NT), 0, st,
                       static_cast<const T*>(x), static_cast<const T*>(b), static_cast<T*>(y),
                       static_cast<const T*>(tab), n, cz, tiles_x, tiles_y);
    return hipGetLastError();
}

template <typename T, bool RESID>
hipError_t dispatch_k(int k, const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    switch (k) {
        case 1: return launch<1, T, RESID>(x, b, y, tab, n, st);
        case 2: return launch<2, T, RESID>(x, b, y, tab, n, st);
        case 3: return launch<3, T, RESID>(x, b, y, tab, n, st);
        case 4: return launch<4, T, RESID>(x, b, y, tab, n, st);
        case 5: return launch<5, T, RESID>(x, b, y, tab, n, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_apply(int k, bool f64, bool resid, const void* x, const void* b, void* y,
                        const void* tab, int n, hipStream_t st) {
    if (f64) return resid ? dispatch_k<double, true>(k, x, b, y, tab, n, st)
                          : dispatch_k<double, false>(k, x, b, y, tab, n, st);
    return resid ? dispatch_k<float, true>(k, x, b, y, tab, n, st)
                 : dispatch_k<float, false>(k, x, b, y, tab, n, st);
}

}  // namespace smg
