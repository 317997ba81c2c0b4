// Host-side launch policy shared by the operator kernels.
#include <algorithm>

#include "apply.hpp"

namespace smg {

int apply_chunk_layers(int k, int n, int blocks_xy) {
    // tile kernels, measured on MI355X at 64^3 cells (the z halo costs two extra layers per
    // chunk, and lengths dividing n avoid a short last chunk): 16 layers at k = 1, 8 at k = 2,
    // 32 at k = 3 and 4, 16 at k = 5.  From 8 cells on a level has at least two chunks, so
    // every level size exercises the chunk-boundary halo.
    (void)blocks_xy;
    const int pref = k == 2 ? 8 : ((k == 3 || k == 4) ? 32 : 16);
    const int cz = n >= 8 ? std::min(pref, n / 2) : pref;
    return std::min(cz, n);
}

}  // namespace smg
