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
};

// Builds the stencil rows of one level (n cells per direction, h = 1/n).
// Throws std::runtime_error if the rows do not reproduce the assembled 1D
// matrices (a self-check run on every level).
LevelTables build_level_tables(const Ref1D& r, int n, double penalty_factor);

}  // namespace smg
