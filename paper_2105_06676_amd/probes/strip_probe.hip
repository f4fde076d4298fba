// Measurement probe, not part of the solver: the memory side of a one-pass
// strided transform of an 8192-point axis.
//
// The solver splits a strided axis of 8192 points into two passes (64 x 128)
// because one column of 8192 FP32 complex points already fills 64 KB of LDS: a
// workgroup can hold only W = 1 or 2 adjacent columns, so every wave access
// reads 8 or 16 bytes from each of 64 rows.  This kernel does exactly the
// memory work of such a pass and nothing else: W columns of a [8192][pitch]
// complex FP32 array, 16 points per thread (rows q + 512 i), one exchange
// through LDS (written at q * 16 + i, read back at q + 512 i, so every value
// moves between threads), and the values stored back to the rows they came
// from, into a second array.  Workgroups are optionally remapped so that each
// XCD takes a contiguous run of columns (neighbouring tiles then read the same
// 128-byte lines through one L2).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kRows = 8192, kP = 512;

__host__ __device__ constexpr int pad(int e) { return e + (e >> 4); }

template <int W>
__global__ __launch_bounds__(kP * W) void k_strip_copy(const float2* __restrict__ in, float2* __restrict__ out,
                                                       int pitch, int cols, int ntiles, int remap) {
    extern __shared__ float2 lds[];
    const int cl = threadIdx.x % W, q = threadIdx.x / W;
    unsigned tile = blockIdx.x;
    if (remap) {
        const unsigned per = (unsigned)ntiles / 8;
        if (tile < 8 * per) tile = (tile % 8) * per + tile / 8;
    }
    const int c = (int)tile * W + cl;
    const bool valid = c < cols;
    float2 v[16];
    const float2* src = in + (int64_t)q * pitch + (valid ? c : 0);
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = valid ? src[(int64_t)i * kP * pitch] : float2{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[pad(q * 16 + i) * W + cl] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[pad(q + kP * i) * W + cl];
    if (!valid) return;
    // LDS position e = q + 512 i holds the point that thread e / 16 loaded as its
    // point e % 16, i.e. row e / 16 + 512 (e % 16)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = q + kP * i;
        out[(int64_t)(e / 16 + kP * (e % 16)) * pitch + c] = v[i];
    }
}

template <int W>
hipError_t launch(const float2* in, float2* out, int pitch, int cols, int remap, hipStream_t st) {
    const int ntiles = (cols + W - 1) / W;
    const size_t lds = (size_t)pad(kRows) * W * sizeof(float2);
    hipError_t e = hipFuncSetAttribute((const void*)k_strip_copy<W>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_strip_copy<W>, dim3(ntiles), dim3(kP * W), lds, st, in, out, pitch, cols, ntiles, remap);
    return hipGetLastError();
}

}  // namespace

// Runs the probe `reps` times on `st` and returns milliseconds per launch (from
// HIP events), or a negative value on an error.  `in` and `out` are device
// arrays of 8192 * pitch float2; W is 1 or 2; cols <= pitch.
extern "C" float sfft_probe_strip(int W, int remap, const void* in, void* out, int pitch, int cols, int reps,
                                  hipStream_t st) {
    if ((W != 1 && W != 2) || cols < 1 || pitch < cols || reps < 1) return -1.f;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -2.f;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -2.f;
    }
    float ms = -3.f;
    hipError_t e = hipEventRecord(a, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = W == 1 ? launch<1>((const float2*)in, (float2*)out, pitch, cols, remap, st)
                   : launch<2>((const float2*)in, (float2*)out, pitch, cols, remap, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess) ms /= reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e == hipSuccess ? ms : -4.f;
}
