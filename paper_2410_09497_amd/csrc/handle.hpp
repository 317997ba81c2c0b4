// Library handle (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stokesmg.h"
#include "mg_tables.hpp"
#include "tables.hpp"

struct stokesmg {
    stokesmg_config cfg{};
    int n_levels = 0;
    std::vector<smg::LevelTables> lv;        // 0 = coarsest
    std::string err;

    // caller-owned device workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    // byte offsets inside the workspace
    std::vector<size_t> tab_f64, tab_f32;    // per level
    std::vector<size_t> ptab_f64, ptab_f32;  // per level (patch tables; unused for n < 2)
    size_t r_vec = 0;                        // residual vector of the finest level (8 B per unknown)
    size_t c_vec = 0;                        // finest-level vector: pair capture's correction (inside a
                                             // sweep), the transfers' intermediates (between sweeps)
    size_t cg_counter = 0;                   // two 64-bit counters: CG iterations, patch solves
    size_t ws_needed = 0;

    // multigrid: transfers between level l-1 and l (index l >= 1), coarse pseudo-inverse,
    // vectors x_l, b_l of the levels below the finest (8 B per unknown, either dtype)
    struct TransferOff {
        size_t pd_i, pd_w, pc_i, pc_w, rd_i, rd_w, rc_i, rc_w;
        int wpd, wpc, wrd, wrc;
    };
    std::vector<smg::Transfer1D> tr;          // host copies (index l >= 1)
    std::vector<TransferOff> tro;
    std::vector<double> coarse_pinv;          // empty if the coarsest level is too large
    int N0 = 0;
    size_t coarse_off = 0;
    std::vector<size_t> xl, bl;               // per level l < L-1
    size_t wg_off = 0;                        // Gauss weights (k+1 doubles)
    size_t scratch_off = 0;                   // reductions: kScratch doubles
    // scratch regions (in doubles): coefficients / dot results, pressure moment, multi-dot partials
    static constexpr int kCoef = 0, kMoment = 64, kPartial = 2048, kPartialBlocks = 1024;
    static constexpr int kScratch = kPartial + kPartialBlocks * 64;

    // learned local solver: caller-owned MLP workspace and offsets inside it (bytes)
    struct Mlp {
        char* ws = nullptr;
        size_t bytes = 0;
        int64_t rows = 0;          // max rows per batch / chunk
        int d = 0, H = 256;
        int64_t P = 0;             // parameter count
        size_t params, grads, m, v, Z1, H1, Z2, H2, Y, dY, dZ2, dZ1, X, s, split, lossp, loss, colp, brows, acc;
        size_t direct = 0;         // the Direct solver's maps per patch type, padded [out][in]: FP32, then BF16
        bool direct_ready = false; // stokesmg_direct_setup() has filled it
        size_t split_floats = 0;
        int64_t step = 0;          // Adam steps taken
        bool ready = false;        // parameters initialized or set
    } mlp;
    int local_solver = STOKESMG_LOCAL_EXACT;
    int pre_sweeps = 1, post_sweeps = 1;     // smoothing sweeps of the V-cycle before / after the coarse correction
    int mlp_mode = STOKESMG_MLP_BF16;
    double mlp_omega = 1.0;                  // damping of the learned corrections
    double rho_ref = 0.0;

    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
};

inline int64_t level_total(const stokesmg* h, int level) {
    const int64_t N1 = h->lv[level].N1;
    return 3 * (N1 - 1) * N1 * N1 + N1 * N1 * N1;
}

inline bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

#define SMG_HIP(h, call)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return (h)->fail(STOKESMG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
