// The "Direct" local solver of Sec. 3.3 (host setup of its matrices).
#pragma once

#include <vector>

#include "fe1d.hpp"

namespace smg {

// Patch types: which outer faces of the vertex patch lie on the domain
// boundary, per direction d, as the 1D window type t_d = 0 (none), 1 (the
// lower face: vertex 1), 2 (the upper face: vertex n - 1); type index
// t_0 + 3 t_1 + 9 t_2.  Index 27 is the single patch of the 2^3-cell mesh
// (both faces in every direction).
constexpr int kDirectTypes = 28;

// The normalized exact local solve of a patch of the given type, t = M x with
// x = (F / h, G / h^2) and t = (U, h P) (the variables of the patch gather),
// as a dense d x d matrix, row-major [out][in], FP64.  The same on every
// level; built from the 4^3- and 8^3-cell patch tables, which must agree
// (throws otherwise).  Host cost grows like d^3: degrees 1..3.
std::vector<double> direct_type_map(const Ref1D& r, double penalty_factor, int type);

// All kDirectTypes maps, built on parallel host threads.
std::vector<std::vector<double>> direct_type_maps(const Ref1D& r, double penalty_factor);

}  // namespace smg
