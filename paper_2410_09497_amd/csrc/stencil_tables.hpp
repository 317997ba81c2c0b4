// Layout of the 1D stencil tables the operator kernel reads (host + device).
//
// The operator K = [[A, B^T], [B, 0]] on a Cartesian mesh is a sum of
// Kronecker products of 1D matrices (Sec. 2.2; for the patch matrices
// Eqs. block_A and b):
//   A_x = Lc (x) Md (x) Md + Mc (x) Ld (x) Md + Mc (x) Md (x) Ld,
//   A_y, A_z cyclically (the continuous factor sits in the component's own
//   direction), B_x = -D (x) Md (x) Md, and cyclically,
// factors written in (x, y, z) order.  Each 1D matrix is banded with a
// structure that repeats from cell to cell, so one row per position-in-cell
// describes it.  m = k + 1 positions per cell in every direction:
//
//  MC[b][o], LC[b][o]  b < m, o < 2m+1: row of Mc / Lc at the continuous
//                      position X = cell*m + b (node g = X+1), column X+o-m.
//                      No boundary variants: columns at eliminated boundary
//                      nodes multiply zero values.
//  DT[b][a]            b < m, a < 2m: row of D^T at continuous position
//                      cell*m + b, column (pressure) cell*m + a.
//  DD[a][j]            a < m, j < m+1: row of D at DG position cell*m + a,
//                      column (continuous position) cell*m + j - 1.
//  LD[v][a][o]         v < 4, a < m, o < 3m: row of Ld at DG position
//                      cell*m + a, column cell*m - m + o; v = 0 interior
//                      cell, 1 first cell, 2 last cell, 3 single cell (n = 1).
//  MDg[a]              a < m: the diagonal DG mass h w_a.
#pragma once

namespace smg {

template <int K>
struct Tab {
    static constexpr int m = K + 1;
    static constexpr int MC = 0;
    static constexpr int LC = MC + m * (2 * m + 1);
    static constexpr int DT = LC + m * (2 * m + 1);
    static constexpr int DD = DT + m * 2 * m;
    static constexpr int LD = DD + m * (m + 1);
    static constexpr int MDg = LD + 4 * m * 3 * m;
    static constexpr int size = MDg + m;
};

inline int tab_size(int k) {
    const int m = k + 1;
    return m * (2 * m + 1) * 2 + m * 2 * m + m * (m + 1) + 4 * m * 3 * m + m;
}

// variant of the DG row of cell c among n cells
__host__ __device__ inline int ld_variant(int c, int n) {
    return n == 1 ? 3 : (c == 0 ? 1 : (c == n - 1 ? 2 : 0));
}

}  // namespace smg
