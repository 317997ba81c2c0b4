// Host construction of the per-level stencil tables (FP64).
#pragma once

#include <string>
#include <vector>

#include "fe1d.hpp"

namespace smg {

struct LevelTables {
    int n = 0, k = 0, N1 = 0;
    double h = 0, gamma = 0;
    std::vector<double> stencil;   // layout of Tab<k> (stencil_tables.hpp)
    std::vector<double> patch;     // layout of PatchTab<k> (patch_tables.hpp); empty for n < 2
};

// Builds the stencil rows of one level (n cells per direction, h = 1/n).
// Throws std::runtime_error if the rows do not reproduce the assembled 1D
// matrices (a self-check run on every level).
LevelTables build_level_tables(const Ref1D& r, int n, double penalty_factor);

// Fast-diagonalization data of the vertex-patch matrices of one level
// (n >= 2): generalized eigenpairs of the restricted 1D stiffness/mass
// matrices per patch-boundary type, the restricted divergence block and the
// DG mass of a patch window.  Throws if an eigen-decomposition fails its
// self-check.
std::vector<double> build_patch_tables(const Ref1D& r, int n, double penalty_factor);

}  // namespace smg
