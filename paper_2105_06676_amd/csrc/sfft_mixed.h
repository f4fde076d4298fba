// Register mixed-radix pass kernels (sfft_mixed.hip): 7-smooth lengths held Q
// points per thread (Q of the length's family), a radix-Q stage first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_types.h"

namespace sfft {

// Stage radices are packed kMRadBits bits each into PassDesc::mrad, the first
// stage in the lowest bits.
constexpr int kMRadBits = 5;
constexpr uint64_t kMRadMask = (1u << kMRadBits) - 1;
__host__ __device__ inline int mixed_radix_at(int64_t packed, int s) {
    return (int)(((uint64_t)packed >> (kMRadBits * s)) & kMRadMask);
}

// points per thread of a length's family and its stage radices (packed as
// above); false when the length has no family or the tile shape does not fit
// (rows: P = L / Q <= 512 threads; columns: P <= 64).
bool mixed_family(int64_t L, bool column, bool f64, int* Q, int64_t* packed, int* nst);

// FP64 symbol chains are evaluated G at a time: the largest divisor of Q up to
// 7 (independent chains hide the FP64 latency; 14 points take two groups of
// seven rather than seven of two).
template <int Q>
constexpr int kMGroup() {
    return Q % 7 == 0 ? 7 : (Q % 6 == 0 ? 6 : (Q % 5 == 0 ? 5 : (Q % 4 == 0 ? 4 : (Q % 3 == 0 ? 3 : 2))));
}

hipError_t launch_mixed_pass(const PassDesc& pd, const SymParams& sp, bool f64, size_t lds, hipStream_t st);
hipError_t launch_mixed_batch(const PassDesc& proto, const BatchItem* items, int n, const SymParams* syms,
                              int64_t tiles, bool f64, size_t lds, hipStream_t st);

}  // namespace sfft
