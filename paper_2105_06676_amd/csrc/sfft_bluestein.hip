// Elementwise kernels of the Bluestein path (see sfft_bluestein.h).
//
// Bluestein: with jk = (j^2 + k^2 - (k - j)^2) / 2 the DFT
//   X_k = sum_j x_j exp(-2 pi i jk / n) = c_k sum_j (c_j x_j) h_{k-j},
//   c_j = exp(-i pi j^2 / n), h_m = exp(+i pi m^2 / n) = conj c_m,
// a linear convolution that a length-M circular one (M >= 2n - 1) reproduces for
// k < n.  The inverse transform uses the conjugate chirp.  Chirp phases reduce
// j^2 modulo 2n in integers before sincospi, so they are exact to FP64 rounding.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sfft_bluestein.h"
#include "sfft_device.h"

namespace sfft {

namespace {

constexpr int kB = 256;

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kB - 1) / kB)); }

// I: index type (uint32_t when every index of the launch fits, else int64_t;
// 64-bit division costs several times the 32-bit one).
template <typename I>
__device__ __forceinline__ I order_freq(const AxisOrder& o, I p) {
    if (o.nlev <= 1) return p;
    const I s0 = (I)o.sub[0], s1 = (I)o.sub[1], s2 = (I)o.sub[2];
    if (o.nlev == 2) {
        const I d0 = p / s1, d1 = p - d0 * s1;
        return d0 + s0 * d1;
    }
    const I d0 = p / (s1 * s2);
    const I rem = p - d0 * s1 * s2;
    const I d1 = rem / s2, d2 = rem - d1 * s2;
    return d0 + s0 * (d1 + s1 * d2);
}

template <typename R>
__global__ void k_widen(const R* g, cx<R>* w, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < N) w[i] = cx<R>{g[i], R(0)};
}

template <typename R>
__global__ void k_narrow(const cx<R>* w, R* g, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < N) g[i] = w[i].x;
}

__global__ void k_chirp(double2* c, int64_t n, int sign) {
    const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (j >= n) return;
    const uint64_t q = ((uint64_t)j * (uint64_t)j) % (uint64_t)(2 * n);  // j < n < 2^31
    double s, co;
    sincospi((double)q / (double)n, &s, &co);
    c[j] = double2{co, sign * s};
}

template <typename R>
__global__ void k_chirp_kernel(cx<R>* h, const double2* c, int64_t n, int64_t M) {
    const int64_t m = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (m >= M) return;
    cx<R> v = {R(0), R(0)};
    if (m < n) v = cx<R>{R(c[m].x), R(-c[m].y)};
    else if (M - m < n) v = cx<R>{R(c[M - m].x), R(-c[M - m].y)};
    h[m] = v;
}

template <typename R>
__global__ void k_reorder_scale(const cx<R>* src, cx<R>* dst, int64_t M, AxisOrder ord) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= M) return;
    const R s = R(1.0 / (double)M);
    dst[order_freq<int64_t>(ord, p)] = scale(src[p], s);
}

template <typename R>
__global__ void k_gather_order(const cx<R>* src, cx<R>* dst, int64_t M, AxisOrder ord) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= M) return;
    dst[p] = src[order_freq<int64_t>(ord, p)];
}

template <typename R, typename I>
__global__ void k_pad_chirp(const cx<R>* src, cx<R>* dst, I outer, I n, I inner, I M, const double2* c) {
    const I e = (I)blockIdx.x * kB + threadIdx.x;
    if (e >= outer * M * inner) return;
    const I rest = e / inner, i = e - rest * inner;
    const I o = rest / M, j = rest - o * M;
    cx<R> v = {R(0), R(0)};
    if (j < n) {
        const cx<R> x = src[(o * n + j) * inner + i];
        const dcx y = dmul(dcx{(double)x.x, (double)x.y}, dcx{c[j].x, c[j].y});
        v = cx<R>{R(y.x), R(y.y)};
    }
    dst[e] = v;
}

template <typename R, typename I>
__global__ void k_mul_h(cx<R>* buf, I outer, I M, I inner, const cx<R>* H, AxisOrder ord) {
    const I e = (I)blockIdx.x * kB + threadIdx.x;
    if (e >= outer * M * inner) return;
    const I rest = e / inner;
    const I p = rest - (rest / M) * M;
    buf[e] = cmul(buf[e], H[order_freq<I>(ord, p)]);
}

template <typename R, typename I>
__global__ void k_extract_chirp(const cx<R>* src, cx<R>* dst, I outer, I n, I inner, I M, const double2* c) {
    const I e = (I)blockIdx.x * kB + threadIdx.x;
    if (e >= outer * n * inner) return;
    const I rest = e / inner, i = e - rest * inner;
    const I o = rest / n, k = rest - o * n;
    const cx<R> x = src[(o * M + k) * inner + i];
    const dcx y = dmul(dcx{(double)x.x, (double)x.y}, dcx{c[k].x, c[k].y});
    dst[e] = cx<R>{R(y.x), R(y.y)};
}

// Four elements per thread, 256 apart along the row-major index: their symbol
// powers run as independent chains (1-D spectra).
template <typename R>
__global__ void k_symbol_full(cx<R>* w, SymParams sp, int64_t N) {
    constexpr int G = 4;
    const int64_t e0 = (int64_t)blockIdx.x * kB * G + threadIdx.x;
    dcx mu[G], out[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t e = e0 + (int64_t)g * kB;
        int64_t f[3] = {0, 0, 0};
        int64_t rem = e < N ? e : 0;
        for (int a = sp.d - 1; a >= 0; --a) {
            const int64_t q = rem / sp.n[a];
            f[a] = pos_to_freq(sp, a, rem - q * sp.n[a]);
            rem = q;
        }
        const SymCol col = sp.d >= 2 ? symbol_column(sp, f) : symbol_column_1d(sp);
        mu[g] = symbol_mu(sp, col, f[0]);
    }
    if (sp.real_sym) {
        double m[G], o[G];
#pragma unroll
        for (int g = 0; g < G; ++g) m[g] = mu[g].x;
        power_real_dev<G>(m, o, sp.T, sp.switching);
#pragma unroll
        for (int g = 0; g < G; ++g) out[g] = dcx{o[g] * sp.scale, 0.0};
    } else {
        power_complex_dev<G>(mu, out, sp.T, sp.switching);
#pragma unroll
        for (int g = 0; g < G; ++g) out[g] = dcx{out[g].x * sp.scale, out[g].y * sp.scale};
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t e = e0 + (int64_t)g * kB;
        if (e >= N) continue;
        const cx<R> x = w[e];
        const dcx y = dmul(dcx{(double)x.x, (double)x.y}, out[g]);
        w[e] = cx<R>{R(y.x), R(y.y)};
    }
}

// d >= 2: the spectrum as rows (axis 0) x columns (axes 1..d-1, ncol of them);
// a thread takes one column, reads its part of the symbol once from the table
// (sp.coltab) and does four rows at a time as independent chains.
template <typename R>
__global__ void k_symbol_rows(cx<R>* w, SymParams sp, int64_t rows, int64_t ncol) {
    constexpr int G = 4;
    const int64_t c = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (c >= ncol) return;
    const SymCol col = ((const SymCol*)sp.coltab)[c];
    for (int64_t r0 = (int64_t)blockIdx.y * G; r0 < rows; r0 += (int64_t)gridDim.y * G) {
        dcx mu[G], out[G];
#pragma unroll
        for (int g = 0; g < G; ++g) mu[g] = symbol_mu(sp, col, pos_to_freq(sp, 0, min(r0 + g, rows - 1)));
        if (sp.real_sym) {
            double m[G], o[G];
#pragma unroll
            for (int g = 0; g < G; ++g) m[g] = mu[g].x;
            power_real_dev<G>(m, o, sp.T, sp.switching);
#pragma unroll
            for (int g = 0; g < G; ++g) out[g] = dcx{o[g] * sp.scale, 0.0};
        } else {
            power_complex_dev<G>(mu, out, sp.T, sp.switching);
#pragma unroll
            for (int g = 0; g < G; ++g) out[g] = dcx{out[g].x * sp.scale, out[g].y * sp.scale};
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (r0 + g >= rows) continue;
            const int64_t e = (r0 + g) * ncol + c;
            const cx<R> x = w[e];
            const dcx y = dmul(dcx{(double)x.x, (double)x.y}, out[g]);
            w[e] = cx<R>{R(y.x), R(y.y)};
        }
    }
}

}  // namespace

hipError_t launch_widen(const void* grid, void* ws, int64_t N, bool f64, hipStream_t st) {
    if (f64) hipLaunchKernelGGL(k_widen<double>, grid_for(N), dim3(kB), 0, st, (const double*)grid, (cx<double>*)ws, N);
    else hipLaunchKernelGGL(k_widen<float>, grid_for(N), dim3(kB), 0, st, (const float*)grid, (cx<float>*)ws, N);
    return hipGetLastError();
}

hipError_t launch_narrow(const void* ws, void* grid, int64_t N, bool f64, hipStream_t st) {
    if (f64) hipLaunchKernelGGL(k_narrow<double>, grid_for(N), dim3(kB), 0, st, (const cx<double>*)ws, (double*)grid, N);
    else hipLaunchKernelGGL(k_narrow<float>, grid_for(N), dim3(kB), 0, st, (const cx<float>*)ws, (float*)grid, N);
    return hipGetLastError();
}

hipError_t launch_chirp(double2* c, int64_t n, int sign, hipStream_t st) {
    hipLaunchKernelGGL(k_chirp, grid_for(n), dim3(kB), 0, st, c, n, sign);
    return hipGetLastError();
}

hipError_t launch_chirp_kernel(void* h, const double2* c, int64_t n, int64_t M, bool f64, hipStream_t st) {
    if (f64) hipLaunchKernelGGL(k_chirp_kernel<double>, grid_for(M), dim3(kB), 0, st, (cx<double>*)h, c, n, M);
    else hipLaunchKernelGGL(k_chirp_kernel<float>, grid_for(M), dim3(kB), 0, st, (cx<float>*)h, c, n, M);
    return hipGetLastError();
}

hipError_t launch_reorder_scale(const void* src, void* dst, int64_t M, AxisOrder ord, bool f64, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_reorder_scale<double>, grid_for(M), dim3(kB), 0, st, (const cx<double>*)src,
                           (cx<double>*)dst, M, ord);
    else
        hipLaunchKernelGGL(k_reorder_scale<float>, grid_for(M), dim3(kB), 0, st, (const cx<float>*)src,
                           (cx<float>*)dst, M, ord);
    return hipGetLastError();
}

hipError_t launch_gather_order(const void* src, void* dst, int64_t M, AxisOrder ord, bool f64, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_gather_order<double>, grid_for(M), dim3(kB), 0, st, (const cx<double>*)src,
                           (cx<double>*)dst, M, ord);
    else
        hipLaunchKernelGGL(k_gather_order<float>, grid_for(M), dim3(kB), 0, st, (const cx<float>*)src,
                           (cx<float>*)dst, M, ord);
    return hipGetLastError();
}

// 32-bit indices when every index of the launch fits
static bool fits32(int64_t total) { return total < ((int64_t)1 << 32) - 4 * kB; }

template <typename R, typename I>
static void pad_chirp_t(const void* src, void* dst, int64_t outer, int64_t n, int64_t inner, int64_t M,
                        const double2* c, hipStream_t st) {
    hipLaunchKernelGGL((k_pad_chirp<R, I>), grid_for(outer * M * inner), dim3(kB), 0, st, (const cx<R>*)src, (cx<R>*)dst,
                       (I)outer, (I)n, (I)inner, (I)M, c);
}

hipError_t launch_pad_chirp(const void* src, void* dst, int64_t outer, int64_t n, int64_t inner, int64_t M,
                            const double2* c, bool f64, hipStream_t st) {
    const bool s = fits32(outer * M * inner);
    if (f64) s ? pad_chirp_t<double, uint32_t>(src, dst, outer, n, inner, M, c, st)
               : pad_chirp_t<double, int64_t>(src, dst, outer, n, inner, M, c, st);
    else s ? pad_chirp_t<float, uint32_t>(src, dst, outer, n, inner, M, c, st)
           : pad_chirp_t<float, int64_t>(src, dst, outer, n, inner, M, c, st);
    return hipGetLastError();
}

template <typename R, typename I>
static void mul_h_t(void* buf, int64_t outer, int64_t M, int64_t inner, const void* H, AxisOrder ord, hipStream_t st) {
    hipLaunchKernelGGL((k_mul_h<R, I>), grid_for(outer * M * inner), dim3(kB), 0, st, (cx<R>*)buf, (I)outer, (I)M,
                       (I)inner, (const cx<R>*)H, ord);
}

hipError_t launch_mul_h(void* buf, int64_t outer, int64_t M, int64_t inner, const void* H, AxisOrder ord, bool f64,
                        hipStream_t st) {
    const bool s = fits32(outer * M * inner);
    if (f64) s ? mul_h_t<double, uint32_t>(buf, outer, M, inner, H, ord, st)
               : mul_h_t<double, int64_t>(buf, outer, M, inner, H, ord, st);
    else s ? mul_h_t<float, uint32_t>(buf, outer, M, inner, H, ord, st)
           : mul_h_t<float, int64_t>(buf, outer, M, inner, H, ord, st);
    return hipGetLastError();
}

template <typename R, typename I>
static void extract_t(const void* src, void* dst, int64_t outer, int64_t n, int64_t inner, int64_t M, const double2* c,
                      hipStream_t st) {
    hipLaunchKernelGGL((k_extract_chirp<R, I>), grid_for(outer * n * inner), dim3(kB), 0, st, (const cx<R>*)src,
                       (cx<R>*)dst, (I)outer, (I)n, (I)inner, (I)M, c);
}

hipError_t launch_extract_chirp(const void* src, void* dst, int64_t outer, int64_t n, int64_t inner, int64_t M,
                                const double2* c, bool f64, hipStream_t st) {
    // the source array is the larger one (M >= n)
    const bool s = fits32(outer * M * inner);
    if (f64) s ? extract_t<double, uint32_t>(src, dst, outer, n, inner, M, c, st)
               : extract_t<double, int64_t>(src, dst, outer, n, inner, M, c, st);
    else s ? extract_t<float, uint32_t>(src, dst, outer, n, inner, M, c, st)
           : extract_t<float, int64_t>(src, dst, outer, n, inner, M, c, st);
    return hipGetLastError();
}

hipError_t launch_symbol_full(void* ws, const SymParams& sp, int64_t N, bool f64, hipStream_t st) {
    if (sp.d >= 2 && sp.coltab) {
        const int64_t ncol = sp.ncol, rows = N / sp.ncol;
        const dim3 g((unsigned)((ncol + kB - 1) / kB), (unsigned)std::min<int64_t>(65535, (rows + 3) / 4));
        if (f64) hipLaunchKernelGGL(k_symbol_rows<double>, g, dim3(kB), 0, st, (cx<double>*)ws, sp, rows, ncol);
        else hipLaunchKernelGGL(k_symbol_rows<float>, g, dim3(kB), 0, st, (cx<float>*)ws, sp, rows, ncol);
        return hipGetLastError();
    }
    const dim3 g((unsigned)((N + 4 * kB - 1) / (4 * kB)));
    if (f64) hipLaunchKernelGGL(k_symbol_full<double>, g, dim3(kB), 0, st, (cx<double>*)ws, sp, N);
    else hipLaunchKernelGGL(k_symbol_full<float>, g, dim3(kB), 0, st, (cx<float>*)ws, sp, N);
    return hipGetLastError();
}

}  // namespace sfft
