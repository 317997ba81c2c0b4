// Layout of the per-level vertex-patch tables (host + device).
//
// A vertex patch (Sec. 3.1) is 2 x 2 x 2 cells.  In one direction its local
// space has NC = 2k+1 interior continuous nodes (the normal nodes on the
// patch boundary are excluded, caption of Fig. smoother) and ND = 2k+2
// discontinuous indices.  The patch matrix A_j is, per velocity component, a
// Kronecker sum of restricted 1D stiffness/mass matrices (Sec. 3.2), so its
// inverse is the fast diagonalization (Eqs. inverse2d / fast_inverse):
//   A^{-1} = (S_z (x) S_y (x) S_x) diag(1 / (l_x + l_y + l_z)) (...)^T,
//   L_d S_d = M_d S_d diag(l_d),  S_d^T M_d S_d = I.
// The continuous window has one type; a discontinuous window has four:
// 0 interior, 1 lower face on the domain boundary, 2 upper face on the
// boundary, 3 both (n = 2).  B_j = -(D (x) Md (x) Md, ...) with D the
// restriction of the 1D divergence block (ND x NC) and Md = h w.
#pragma once

namespace smg {

template <int K>
struct PatchTab {
    static constexpr int NC = 2 * K + 1, ND = 2 * K + 2;
    static constexpr int SC = 0;                   // S of the continuous window, NC x NC (row-major)
    static constexpr int LC = SC + NC * NC;        // its eigenvalues
    static constexpr int SD = LC + NC;             // 4 types: ND x ND each
    static constexpr int LDv = SD + 4 * ND * ND;   // 4 types: ND eigenvalues each
    static constexpr int DP = LDv + 4 * ND;        // ND x NC
    static constexpr int MDP = DP + ND * NC;       // ND: h w_(i mod (k+1))
    static constexpr int size = MDP + ND;
};

inline int patch_tab_size(int k) {
    const int nc = 2 * k + 1, nd = 2 * k + 2;
    return nc * nc + nc + 4 * nd * nd + 4 * nd + nd * nc + nd;
}

}  // namespace smg
