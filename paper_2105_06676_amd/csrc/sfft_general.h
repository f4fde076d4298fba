// Symbol power for stencils of any radius up to kMaxGeneralR, applied to a half
// spectrum between the forward and the inverse transform (unfused schedule).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_types.h"

namespace sfft {

constexpr int kMaxGeneralR = 8;

struct GeneralParams {
    void* ws;          // half spectrum, [rows][pitch] complex entries
    int64_t rows;      // spectrum rows (product of the extents of axes 0..d-2)
    int64_t pitch;     // complex entries per row
    const double* c;   // (2r+1)^d coefficients (normalised as fill_symbol does), device memory
    int r;
};

// sp: geometry of the unfused schedule (n, nlev, sub, sdim, hcount, eph) plus the
// symbol fields one_minus_sum, real_sym, switching, T and scale.
hipError_t launch_symbol_general(const GeneralParams& gp, const SymParams& sp, bool f64, hipStream_t st);

}  // namespace sfft
