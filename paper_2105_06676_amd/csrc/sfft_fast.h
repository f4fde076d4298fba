// Power-of-two fast pass kernels (sfft_fast.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "sfft_types.h"

namespace sfft {

// fast row pass kinds (PassDesc::fast_kind)
enum FastRowKind { ROW_R2C = 0, ROW_C2R = 1, ROW_MIDR = 2, ROW_MIDC = 3, ROW_CFWD = 4, ROW_CINV = 5,
                   // odd real lengths (register mixed-radix rows only)
                   ROW_R2C_ODD = 6, ROW_C2R_ODD = 7, ROW_MIDR_ODD = 8 };

constexpr int kFastMinL = 16;
constexpr int kFastMaxRowL = 4096;   // 256 threads x 16 points
constexpr int kFastMaxColL = 1024;   // at least 4 columns per tile

hipError_t launch_fast_pass(const PassDesc& pd, const SymParams& sp, bool f64, size_t lds, hipStream_t st);
// One launch running pass `proto`'s kernel variant over a work list (device memory).
hipError_t launch_fast_batch(const PassDesc& proto, const BatchItem* items, int n, const SymParams* syms,
                             int64_t tiles, bool f64, size_t lds, hipStream_t st);

// Threads of a column tile of length 2^logl: FP64 tiles of short columns use
// half-size workgroups, so that more of them share a compute unit's LDS.
constexpr bool col_half(bool f64, int logl) { return f64 && logl <= 7; }
template <typename R>
constexpr int col_threads(int logl) { return col_half(sizeof(R) == 8, logl) ? 128 : 256; }
}  // namespace sfft
