// Measurement probe, not part of the solver: is a small-radix DFT stage faster
// as a matrix product on the matrix cores (MFMA) than as the butterflies the
// pass kernels use?
//
// Both kernels apply a 16-point complex DFT (FP32) `reps` times to each of n
// vectors held in registers (loaded once, stored once), so the timing is the
// arithmetic of one DFT stage:
//  k_dft16_butterfly  one vector per thread, the pass kernels' composite 4 x 4
//                     in-register DFT (two radix-4 layers and 9 twiddles);
//  k_dft16_mfma       32 vectors per wave64 as a real 32 x 32 matrix times a
//                     32 x 32 block (Re and Im of 16 points stacked), 16
//                     v_mfma_f32_32x32x2f32 per application.  The matrix rows
//                     are permuted so that the product leaves every lane with
//                     the layout it started from (lane l < 32: Re of vector l,
//                     lane l >= 32: Im of vector l - 32), so repeated
//                     applications need no shuffles.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../csrc/sfft_device.h"

namespace sfft {
template <>
struct RootTab<16> {
    static constexpr double c[16] = {1.0, 0.9238795325112867, 0.7071067811865476, 0.38268343236508984,
                                     0.0, -0.38268343236508984, -0.7071067811865476, -0.9238795325112867,
                                     -1.0, -0.9238795325112867, -0.7071067811865476, -0.38268343236508984,
                                     0.0, 0.38268343236508984, 0.7071067811865476, 0.9238795325112867};
    static constexpr double s[16] = {0.0, 0.38268343236508984, 0.7071067811865476, 0.9238795325112867,
                                     1.0, 0.9238795325112867, 0.7071067811865476, 0.38268343236508984,
                                     0.0, -0.38268343236508984, -0.7071067811865476, -0.9238795325112867,
                                     -1.0, -0.9238795325112867, -0.7071067811865476, -0.38268343236508984};
};
}  // namespace sfft

using sfft::cx;

namespace {

__global__ __launch_bounds__(256) void k_dft16_butterfly(const float2* __restrict__ in, float2* __restrict__ out,
                                                         int64_t n, int reps) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    cx<float> x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float2 t = in[v * 16 + i];
        x[i] = cx<float>{t.x, t.y};
    }
    for (int r = 0; r < reps; ++r) sfft::dft_ab<float, 4, 4, false>(x);
#pragma unroll
    for (int i = 0; i < 16; ++i) out[v * 16 + i] = float2{x[i].x, x[i].y};
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Real 32 x 32 matrix of the 16-point DFT in the lane layout described above:
// A operand of MFMA j, lane l: M[l % 32][2j + l / 32] with
//   row (i / 4) * 8 + h * 4 + i % 4  = (h ? Im : Re) of output point i (i < 16),
//   column 2j + g                    = (g ? Im : Re) of input point j.
__device__ float dft_matrix_entry(int row, int col) {
    const int h = (row >> 2) & 1;
    const int i = (row >> 3) * 4 + (row & 3);
    const int j = col >> 1, g = col & 1;
    const int m = (i * j) & 15;
    const float c = (float)sfft::RootTab<16>::c[m], s = (float)sfft::RootTab<16>::s[m];
    // forward: Y_i = sum_j x_j (cos - i sin):  Re Y = c Re x + s Im x,  Im Y = -s Re x + c Im x
    if (!h) return g ? s : c;
    return g ? c : -s;
}

__global__ __launch_bounds__(256) void k_dft16_mfma(const float* __restrict__ in, float* __restrict__ out,
                                                    int64_t n, int reps) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t v = wave * 32 + (lane & 31);  // this lane's vector
    const int h = lane >> 5;                    // 0: real parts, 1: imaginary parts
    float a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = dft_matrix_entry(lane & 31, 2 * j + h);
    floatx16 x;
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = v < n ? in[v * 32 + 2 * i + h] : 0.0f;
    for (int r = 0; r < reps; ++r) {
        floatx16 y = {0};
        // B operand of MFMA j, lane l: X[2j + l / 32][l % 32] = component (2j + h) of this
        // lane's vector, i.e. its point j's Re (h = 0) or Im (h = 1) part: x[j]
#pragma unroll
        for (int j = 0; j < 16; ++j) y = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j], x[j], y, 0, 0, 0);
        x = y;
    }
    if (v < n) {
#pragma unroll
        for (int i = 0; i < 16; ++i) out[v * 32 + 2 * i + h] = x[i];
    }
}

}  // namespace

extern "C" {

// variant 0: butterflies, 1: MFMA.  in / out: device arrays of n vectors of 16
// complex FP32 values (interleaved re, im).  Returns the kernel time in
// milliseconds (HIP events on `stream`), or a negative value on error.
float sfft_probe_dft16(int variant, const void* in, void* out, int64_t n, int reps, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
    (void)hipEventRecord(e0, st);
    if (variant == 0) {
        const unsigned blocks = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_dft16_butterfly, dim3(blocks), dim3(256), 0, st, (const float2*)in, (float2*)out, n,
                           reps);
    } else {
        const int64_t waves = (n + 31) / 32;
        const unsigned blocks = (unsigned)((waves + 3) / 4);
        hipLaunchKernelGGL(k_dft16_mfma, dim3(blocks), dim3(256), 0, st, (const float*)in, (float*)out, n, reps);
    }
    (void)hipEventRecord(e1, st);
    float ms = -2.0f;
    if (hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

}  // extern "C"
