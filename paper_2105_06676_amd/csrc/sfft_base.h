// Parameters of the RecursiveBoundary base-case kernel (sfft_base.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_types.h"

namespace sfft {

constexpr int kBaseThreads = 256;
constexpr int kBaseMaxCells = 8192;   // LDS cells per tile (64 KB in FP64)

// A box of interior cells, cut into tiles of `tile` cells per axis.
struct BaseStrip {
    int64_t lo[3], ext[3];     // interior coordinates (3 axes, unused leading axes have extent 1)
    int64_t tile[3];
    int64_t ntiles[3];
    int64_t first;             // index of the strip's first workgroup
};

struct BaseParams {
    int nstrip, steps, ncoef;
    int bc;                    // 0: fixed frame values; 1: reflecting (frame = mirror image of the interior)
    int64_t n[3];              // interior extents (padded to 3 axes)
    int64_t r3[3];             // frame width per axis (0 on unused axes)
    int64_t reach3[3];         // the stencil's largest offset along each axis
    int64_t halo3[3];          // reach * steps per axis (0 on unused axes)
    int64_t sstride[3];        // element strides of the stored array
    const void* src;           // values at the start time (interior)
    const void* frame;         // array whose frame holds the boundary values
    void* dst;                 // where the band cells at the end time go
    int off[kMaxCoef][3];      // non-zero stencil offsets
    double c[kMaxCoef];        // their coefficients
    BaseStrip strip[6];
};

hipError_t launch_base(const BaseParams& bp, bool f64, int64_t nblocks, size_t lds, hipStream_t st);

}  // namespace sfft
