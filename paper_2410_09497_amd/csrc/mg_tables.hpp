// Host construction of the multigrid data: 1D transfer lists and the dense
// coarse-level pseudo-inverse (FP64).
#pragma once

#include <vector>

#include "fe1d.hpp"

namespace smg {

// One 1D transfer operator as padded row lists: row i has `width` entries
// (idx[i*width + t], w[i*width + t]), idx = -1 for padding.
struct Rows1D {
    int rows = 0, width = 0;
    std::vector<int> idx;
    std::vector<double> w;
};

// Prolongation between levels with nc and 2 nc cells (Sec. 3: the canonical
// embedding; with nodal bases its entries are the coarse basis functions
// evaluated at the fine support points), one list per direction kind, and
// the transposed lists (restriction = P^T).
struct Transfer1D {
    Rows1D pd, pc;   // fine DG positions -> coarse DG; fine interior nodes -> coarse interior nodes
    Rows1D rd, rc;   // transposes
};

Transfer1D build_transfer(const Ref1D& r, int n_coarse);

// Dense K_0 of the level with one cell (Kronecker form of the 1D matrices)
// and its pseudo-inverse.  The kernel of K_0 is spanned by the constant
// pressure c (normalized); [[K_0, c], [c^T, 0]] is regular and its inverse is
// [[K_0^+, c], [c^T, 0]].  Returns K_0^+ (row-major, N0 x N0).
std::vector<double> coarse_pseudo_inverse(const Ref1D& r, int n0, double penalty_factor, int* N0_out);

}  // namespace smg
