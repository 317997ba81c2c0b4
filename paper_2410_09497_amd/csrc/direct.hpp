// The "Direct" local solver of Sec. 3.3 for interior patches (host setup).
#pragma once

#include <vector>

#include "fe1d.hpp"

namespace smg {

// The normalized exact local solve of an interior patch, t = M x with
// x = (F / h, G / h^2) and t = (U, h P) (the variables of the patch gather),
// as a dense d x d matrix, row-major [out][in], FP64.  The same on every
// level; built from the 4^3- and 8^3-cell patch tables, which must agree
// (throws otherwise).  Host cost grows like d^3: degrees 1..3.
std::vector<double> direct_interior_map(const Ref1D& r, double penalty_factor);

}  // namespace smg
