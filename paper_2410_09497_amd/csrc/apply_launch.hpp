// Launch helpers shared by the per-degree translation units.
#pragma once

#include <algorithm>

#include "apply.hpp"
#include "apply2_kernel.hpp"
#include "apply_kernel.hpp"

namespace smg {

// Tile (cells in x, cells in y) of the generic kernel per degree.
template <int K> struct TileOf;
template <> struct TileOf<1> { static constexpr int CX = 8, CY = 8; };
template <> struct TileOf<2> { static constexpr int CX = 8, CY = 4; };
template <> struct TileOf<3> { static constexpr int CX = 4, CY = 4; };
template <> struct TileOf<4> { static constexpr int CX = 4, CY = 2; };
template <> struct TileOf<5> { static constexpr int CX = 4, CY = 2; };

template <int K, typename T, bool RESID>
hipError_t launch_generic(const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    constexpr int CX = TileOf<K>::CX, CY = TileOf<K>::CY;
    using S = ApplyShape<K, CX, CY>;
    const int N1 = n * S::M;
    const int tiles_x = (N1 + S::TX - 1) / S::TX;
    const int tiles_y = (N1 + S::TY - 1) / S::TY;
    const int cz = apply_chunk_layers(n, tiles_x * tiles_y);
    const int nzc = (n + cz - 1) / cz;
    hipLaunchKernelGGL((stokes_apply_kernel<K, T, CX, CY, RESID>), dim3(tiles_x * tiles_y * nzc), dim3(S::NT), 0,
                       st, static_cast<const T*>(x), static_cast<const T*>(b), static_cast<T*>(y),
                       static_cast<const T*>(tab), n, cz, tiles_x, tiles_y);
    return hipGetLastError();
}

template <int K, typename T, bool RESID>
hipError_t launch_wave_position(const void* x, const void* b, void* y, int n, hipStream_t st) {
    using S = Ap2<K>;
    const int tiles = (n + S::C - 1) / S::C;
    const int cz = apply_chunk_layers(n, tiles * tiles);
    const int nzc = (n + cz - 1) / cz;
    hipLaunchKernelGGL((apply2_kernel<K, T, RESID>), dim3(tiles * tiles * nzc), dim3(S::NT), 0, st,
                       static_cast<const T*>(x), static_cast<const T*>(b), static_cast<T*>(y), n, cz, tiles,
                       T(1.0 / n));
    return hipGetLastError();
}

}  // namespace smg
