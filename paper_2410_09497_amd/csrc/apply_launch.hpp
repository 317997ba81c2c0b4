// Launch helpers shared by the per-degree translation units.
#pragma once

#include <algorithm>
#include <cstdio>

#include "apply.hpp"
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

// Options of the split kernel per degree and precision: where each group
// takes its in-plane stencil rows from (HA / HB: the group holds the rows that
// stay fixed along its plane loop in registers; GA / GB: the group reads its
// rows from global memory, otherwise from LDS), whether group A forms the
// Mc_y u_y plane (AVY), the padded LDS pitch (PAD) and the forward z
// accumulation (ZP; it removes most of the register spills of FP64 at degree
// 5, and costs time where nothing spills).  The fastest of the combinations
// measured on MI355X at 64^3 cells; holding needs the registers (group A's
// rows spill in FP64 at degrees 3 and 5; in FP32 at degrees 1 and 2 the
// kernel's launch bounds hold it to 128 VGPRs, two workgroups per CU).
template <int K, typename T> struct SplitTables {
    static constexpr bool f64 = sizeof(T) == 8;
    static constexpr bool HA = f64 ? (K == 1 || K == 2) : K != 4;
    static constexpr bool GA = false;
    static constexpr bool GB = f64 ? K == 3 : K == 5;
    static constexpr bool HB = f64 ? K == 2 : K != 4;
    static constexpr bool AVY = K <= 3 || (!f64 && K == 5);
    static constexpr bool PAD = f64 && K == 2;
    static constexpr bool ZP = f64 && K == 5;
};

template <int K, typename T, bool RESID, int CX = TileOf<K>::CX, int CY = TileOf<K>::CY>
hipError_t launch_split(const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    using S = SplitShape<K, CX, CY, SplitTables<K, T>::PAD>;
    const int N1 = n * S::M;
    const int tiles_x = (N1 + S::TX - 1) / S::TX;
    const int tiles_y = (N1 + S::TY - 1) / S::TY;
    const int cz = apply_chunk_layers(K, n, tiles_x * tiles_y);
    const int nzc = (n + cz - 1) / cz;
    hipLaunchKernelGGL((stokes_apply_split_kernel<K, T, CX, CY, RESID, SplitTables<K, T>::GA, SplitTables<K, T>::GB,
                                                 SplitTables<K, T>::HA, SplitTables<K, T>::HB,
                                                 SplitTables<K, T>::AVY, SplitTables<K, T>::PAD,
                                                 SplitTables<K, T>::ZP>),
                       dim3(tiles_x * tiles_y * nzc), dim3(S::NT),
                       0, st, static_cast<const T*>(x), static_cast<const T*>(b), static_cast<T*>(y),
                       static_cast<const T*>(tab), n, cz, tiles_x, tiles_y);
    return hipGetLastError();
}

// Kernel choice per degree and precision: the fastest measured on MI355X at
// 64^3 cells (HBM-resident).  The split kernel serves every degree except
// FP64 at degree 4, which the single-group kernel with pipelined plane loads
// serves (the split kernel spills there, with windows or forward sums).
// (degree 2 also compared 8x4, 6x4, 7x3 and 5x5 tiles and 16-layer chunks for the split kernel: all slower)
template <int K> constexpr bool split_default(bool f64) { return K != 4 || !f64; }

template <int K, typename T, bool R>
hipError_t launch_degree_t(bool f64, const void* x, const void* b, void* y, const void* tab, int n, hipStream_t st) {
    if (split_default<K>(f64)) return launch_split<K, T, R>(x, b, y, tab, n, st);
    return launch_generic<K, T, R, TileOf<K>::CX, TileOf<K>::CY, true>(x, b, y, tab, n, st);
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
