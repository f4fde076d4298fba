// Periodic solves on extents with a prime factor above 7: Bluestein's chirp-z
// form of the length-n DFT on those axes (a circular convolution of length M >=
// 2n - 1 done with 7-smooth FFTs), plain complex transforms on the others.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_types.h"

namespace sfft {

// Positions along an axis whose forward transform left them digit-reversed
// across `nlev` factor levels `sub` (nlev <= 1: natural order).
struct AxisOrder {
    int nlev;
    int64_t sub[3];
};

hipError_t launch_widen(const void* grid, void* ws, int64_t N, bool f64, hipStream_t st);
hipError_t launch_narrow(const void* ws, void* grid, int64_t N, bool f64, hipStream_t st);
// c[j] = exp(sign * i pi j^2 / n), j < n (FP64)
hipError_t launch_chirp(double2* c, int64_t n, int sign, hipStream_t st);
// h[m] = conj c[m] for |m| < n wrapped into [0, M), zero elsewhere (precision of the solve)
hipError_t launch_chirp_kernel(void* h, const double2* c, int64_t n, int64_t M, bool f64, hipStream_t st);
// dst[f(p)] = src[p] / M along a length-M digit-reversed transform (natural order out)
hipError_t launch_reorder_scale(const void* src, void* dst, int64_t M, AxisOrder ord, bool f64, hipStream_t st);
// dst[p] = src[f(p)]: a natural-order table laid out in a transform's position order
hipError_t launch_gather_order(const void* src, void* dst, int64_t M, AxisOrder ord, bool f64, hipStream_t st);
// [outer][n][inner] -> [outer][M][inner]: multiply by the chirp, zero-pad
hipError_t launch_pad_chirp(const void* src, void* dst, int64_t outer, int64_t n, int64_t inner, int64_t M,
                            const double2* c, bool f64, hipStream_t st);
// buf[o][p][i] *= H[f(p)] (f: position -> frequency by `ord`; identity for nlev <= 1)
hipError_t launch_mul_h(void* buf, int64_t outer, int64_t M, int64_t inner, const void* H, AxisOrder ord, bool f64,
                        hipStream_t st);
// [outer][M][inner] -> [outer][n][inner]: first n entries times the chirp
hipError_t launch_extract_chirp(const void* src, void* dst, int64_t outer, int64_t n, int64_t inner, int64_t M,
                                const double2* c, bool f64, hipStream_t st);
// ws (complex, dims sp.n[0..d-1], row-major) *= lambda(k)^T * scale, positions
// mapped to frequencies by sp.nlev / sp.sub per axis
hipError_t launch_symbol_full(void* ws, const SymParams& sp, int64_t N, bool f64, hipStream_t st);

}  // namespace sfft
