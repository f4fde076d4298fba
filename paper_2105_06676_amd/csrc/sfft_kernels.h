// Launch wrappers exported by sfft_kernels.hip to the host code.
#pragma once

#include <hip/hip_runtime.h>

#include "sfft_types.h"

namespace sfft {

hipError_t launch_pass(const PassDesc& pd, const SymParams& sp, bool f64, size_t lds, hipStream_t st);
hipError_t set_kernel_lds_limits(size_t bytes);
// One launch running the kernel variant of `proto` over a device work list.
hipError_t launch_pass_batch(const PassDesc& proto, const BatchItem* items, int n, const SymParams* syms,
                             int64_t tiles, bool f64, size_t lds, hipStream_t st);
hipError_t launch_twiddle_table(double2* t64, float2* t32, int64_t N, int64_t count, int64_t mult,
                                hipStream_t st);
hipError_t launch_phase_table(double2* E, int64_t n, hipStream_t st);
hipError_t launch_symbol_columns(void* tab, const SymParams& sp, int64_t total, hipStream_t st);
size_t symbol_column_bytes();
hipError_t launch_symbol_power(double2* out, const SymParams& sp, int64_t total, hipStream_t st);

}  // namespace sfft
