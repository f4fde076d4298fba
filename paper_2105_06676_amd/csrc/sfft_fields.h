// Vector-valued fields: the per-mode m x m symbol matrix and its power (the
// appendix on vector-valued fields), applied to the forward spectra of the m
// fields between the forward and the inverse transform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_types.h"

namespace sfft {

constexpr int kMaxFields = 4;

struct FieldParams {
    int m;             // fields
    int nof;           // stencil offsets per block, (2r+1)^d
    int real_sym;      // every block point-symmetric: the symbol matrix is real
    int64_t rows;      // spectrum rows per field (product of the stored extents of axes 0..d-2)
    int64_t pitch;     // complex elements per row (half spectrum of the last axis, padded)
    int64_t fstride;   // complex elements per field
    void* ws;          // spectra, field-major
    const double* cK;  // K[i][j] = delta_ij - sum_o c_ij[o] (m*m), then c[i][j][o] (m*m*nof)
    // Implicit stencil (m = 1): Q a_{t+1} = S a_t, S given by cK; qK = 1 - sum_o q[o],
    // then q[o]; modes with |lambda_Q| <= qzero take lambda_R = 0 (pseudo-inverse).
    int implicit;
    const double* qK;
    double qzero;
    // 1: full spectrum of a complex transform (every axis, the last one included,
    // maps stored positions to frequencies through sp.nlev / sp.sub); 0: the half
    // spectrum of the real-data passes (last axis in natural order)
    int full;
};

hipError_t launch_fields_symbol(const FieldParams& fp, const SymParams& sp, bool f64, hipStream_t st);

}  // namespace sfft
