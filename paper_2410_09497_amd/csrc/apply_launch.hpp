// Launch helpers shared by the per-degree translation units.
#pragma once

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "apply.hpp"
#include "apply2_kernel.hpp"
#include "apply3_kernel.hpp"
#include "apply_kernel.hpp"

namespace smg {

// Tile (cells in x, cells in y) of the generic kernel per degree.
template <int K> struct TileOf;
template <> struct TileOf<1> { static constexpr int CX = 8, CY = 8; };
template <> struct TileOf<2> { static constexpr int CX = 7, CY = 4; };   // 252 threads: no scratch in FP64
template <> struct TileOf<3> { static constexpr int CX = 4, CY = 4; };
template <> struct TileOf<4> { static constexpr int CX = 4, CY = 2; };
template <> struct TileOf<5> { static constexpr int CX = 3, CY = 2; };   // 216 threads: no scratch

template <int K, typename T, bool RESID, int CX = TileOf<K>::CX, int CY = TileOf<K>::CY, bool PF = false>
hipError_t launch_generic(const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    using S = ApplyShape<K, CX, CY>;
    const int N1 = n * S::M;
    const int tiles_x = (N1 + S::TX - 1) / S::TX;
    const int tiles_y = (N1 + S::TY - 1) / S::TY;
    const int cz = apply_chunk_layers(K, n, tiles_x * tiles_y);
    const int nzc = (n + cz - 1) / cz;
    hipLaunchKernelGGL((stokes_apply_kernel<K, T, CX, CY, RESID, PF>), dim3(tiles_x * tiles_y * nzc), dim3(S::NT), 0,
                       st, static_cast<const T*>(x), static_cast<const T*>(b), static_cast<T*>(y),
                       static_cast<const T*>(tab), n, cz, tiles_x, tiles_y);
    return hipGetLastError();
}

template <int K, typename T, bool RESID, int CX = TileOf<K>::CX, int CY = TileOf<K>::CY>
hipError_t launch_split(const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    using S = SplitShape<K, CX, CY>;
    const int N1 = n * S::M;
    const int tiles_x = (N1 + S::TX - 1) / S::TX;
    const int tiles_y = (N1 + S::TY - 1) / S::TY;
    const int cz = apply_chunk_layers(K, n, tiles_x * tiles_y);
    const int nzc = (n + cz - 1) / cz;
    hipLaunchKernelGGL((stokes_apply_split_kernel<K, T, CX, CY, RESID>), dim3(tiles_x * tiles_y * nzc), dim3(S::NT),
                       0, st, static_cast<const T*>(x), static_cast<const T*>(b), static_cast<T*>(y),
                       static_cast<const T*>(tab), n, cz, tiles_x, tiles_y);
    return hipGetLastError();
}

template <int K, typename T, bool RESID>
hipError_t launch_wave_position(const void* x, const void* b, void* y, int n, hipStream_t st) {
    using S = Ap2<K>;
    const int tiles = (n + S::C - 1) / S::C;
    const int cz = apply_chunk_layers_position(n, tiles * tiles);
    const int nzc = (n + cz - 1) / cz;
    hipLaunchKernelGGL((apply2_kernel<K, T, RESID>), dim3(tiles * tiles * nzc), dim3(S::NT), 0, st,
                       static_cast<const T*>(x), static_cast<const T*>(b), static_cast<T*>(y), n, cz, tiles,
                       T(1.0 / n));
    return hipGetLastError();
}

// Kernel choice.  Defaults are the fastest measured on MI355X at 64^3 cells
// (HBM-resident); STOKESMG_APPLY_KERNEL = generic | pipelined | position | split
// overrides them for comparison runs.
struct ApplyChoice {
    int kernel = 0;   // 0 default, 1 generic, 2 generic with pipelined loads, 3 wave per position, 4 split groups
};
inline ApplyChoice apply_choice() {
    static const ApplyChoice c = [] {
        ApplyChoice r;
        if (const char* s = std::getenv("STOKESMG_APPLY_KERNEL")) {
            if (!std::strcmp(s, "generic")) r.kernel = 1;
            else if (!std::strcmp(s, "pipelined")) r.kernel = 2;
            else if (!std::strcmp(s, "position")) r.kernel = 3;
            else if (!std::strcmp(s, "split")) r.kernel = 4;
        }
        return r;
    }();
    return c;
}

// measured defaults per degree and precision
template <int K> constexpr bool position_default(bool f64) { return K == 1 && !f64; }
// (degree 2 also compared 8x4, 6x4, 7x3 and 5x5 tiles and 16-layer chunks for the split kernel: all slower)
template <int K> constexpr bool split_default(bool f64) { return K == 2 || K == 3 || K == 5 || (K == 4 && !f64); }
template <int K> constexpr bool pipelined_default(bool f64) { return K <= 4 || !f64; }

template <int K, typename T, bool R>
hipError_t launch_degree_t(bool f64, const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    const ApplyChoice c = apply_choice();
    // the wave-per-position kernel is wrong in FP64 at degree 3: never used there
    const bool position = (c.kernel == 3 || (c.kernel == 0 && position_default<K>(f64))) && !(K == 3 && f64);
    // the wave-per-position kernel is built for degrees 1..3 only
    if constexpr (K <= 3)
        if (position) return launch_wave_position<K, T, R>(x, b, y, n, st);
    if (c.kernel == 4 || (c.kernel == 0 && split_default<K>(f64))) return launch_split<K, T, R>(x, b, y, tab, n, st);
    const bool pf = c.kernel == 2 || (c.kernel == 0 && pipelined_default<K>(f64));
    return pf ? launch_generic<K, T, R, TileOf<K>::CX, TileOf<K>::CY, true>(x, b, y, tab, n, st)
              : launch_generic<K, T, R, TileOf<K>::CX, TileOf<K>::CY, false>(x, b, y, tab, n, st);
}

template <int K>
hipError_t launch_degree(bool f64, bool resid, const void* x, const void* b, void* y, const void* tab, int n,
                         hipStream_t st) {
    if (f64) return resid ? launch_degree_t<K, double, true>(true, x, b, y, tab, n, st)
                          : launch_degree_t<K, double, false>(true, x, b, y, tab, n, st);
    return resid ? launch_degree_t<K, float, true>(false, x, b, y, tab, n, st)
                 : launch_degree_t<K, float, false>(false, x, b, y, tab, n, st);
}

}  // namespace smg
