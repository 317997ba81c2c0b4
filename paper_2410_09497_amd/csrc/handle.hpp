// Library handle (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/stokesmg.h"
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
    size_t cg_counter = 0;                   // two int counters: CG iterations, patch solves
    size_t ws_needed = 0;

    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
};

#define SMG_HIP(h, call)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return (h)->fail(STOKESMG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
