// Host-side launch policy shared by the operator kernels.
#include <algorithm>
#include <cstdlib>

#include "apply.hpp"

namespace smg {

namespace {
int forced_chunk() {
    static const int forced = [] {
        const char* s = std::getenv("STOKESMG_APPLY_CZ");
        return s ? std::atoi(s) : 0;
    }();
    return forced;
}
}  // namespace

int apply_chunk_layers(int k, int n, int blocks_xy) {
    if (forced_chunk() > 0) return std::min(forced_chunk(), n);
    // tile kernels, measured on MI355X at 64^3 cells (the z halo costs two extra layers per
    // chunk, and lengths dividing n avoid a short last chunk): 16 layers at k = 1, 8 at k = 2,
    // 32 at k = 3 and 4, 16 at k = 5
    (void)blocks_xy;
    const int pref = k == 2 ? 8 : ((k == 3 || k == 4) ? 32 : 16);
    return std::min(pref, n);
}

int apply_chunk_layers_position(int n, int blocks_xy) {
    if (forced_chunk() > 0) return std::min(forced_chunk(), n);
    // wave-per-position kernel: at least 2048 workgroups, chunks of at least 4 layers
    const int chunks = (2048 + blocks_xy - 1) / blocks_xy;
    const int cz = std::max((n + chunks - 1) / chunks, std::min(4, n));
    return std::min(cz, n);
}

}  // namespace smg
