// Host-side launch policy shared by the operator kernels.
#include <algorithm>
#include <cstdlib>

#include "apply.hpp"

namespace smg {

int apply_chunk_layers(int n, int blocks_xy) {
    static const int forced = [] {
        const char* s = std::getenv("STOKESMG_APPLY_CZ");
        return s ? std::atoi(s) : 0;
    }();
    if (forced > 0) return std::min(forced, n);
    int chunks = (2048 + blocks_xy - 1) / blocks_xy;
    int cz = (n + chunks - 1) / chunks;
    cz = std::max(cz, std::min(4, n));
    return std::min(cz, n);
}

}  // namespace smg
