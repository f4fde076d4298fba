// Symbol power for stencils of any radius (Sec. 3 Steps 1(i), 2 and 3), as an
// elementwise kernel between the forward and the inverse transform.
//
// The fused middle passes evaluate the symbol from per-radius unrolled code for
// radius <= 2.  Wider stencils take the unfused schedule (forward passes, this
// kernel over the half spectrum, inverse passes).  One thread per spectral entry
// forms mu = 1 - lambda(k) = (1 - sum c) - sum_o c_o (prod_a (1 + E_a(o_a k_a)) - 1),
// with E_a(m) = exp(2 pi i m / n_a) - 1 from the per-axis phase tables (the
// deviation form of the fused passes, so modes near lambda = 1 keep their relative
// accuracy), raises 1 - mu to the power T by binary repeated squaring in FP64 and
// multiplies the entry by the result times scale.  The radius is a template
// parameter so that the innermost axis' 2r + 1 phase values stay in registers.
#include <hip/hip_runtime.h>

#include "sfft_device.h"
#include "sfft_general.h"

namespace sfft {

namespace {

// (m + f) mod n for m < n, f < n
__device__ __forceinline__ uint32_t add_mod(uint32_t m, uint32_t f, uint32_t n) {
    const uint32_t s = m + f;
    return s >= n ? s - n : s;
}

// (-r f) mod n, the table index of offset -r
__device__ __forceinline__ uint32_t start_index(int r, uint32_t f, uint32_t n) {
    const uint64_t rf = ((uint64_t)r * f) % n;
    return rf == 0 ? 0u : (uint32_t)(n - rf);
}

template <typename R, int RR, int DIM>
__global__ __launch_bounds__(256) void k_symbol_general(GeneralParams gp, SymParams sp) {
    constexpr int W = 2 * RR + 1;
    const uint32_t cpr = (uint32_t)((sp.hcount + 255) / 256);  // workgroups per spectrum row
    const uint32_t row = blockIdx.x / cpr;
    const uint32_t kl = (blockIdx.x - row * cpr) * 256 + threadIdx.x;
    if (row >= (uint32_t)gp.rows || kl >= (uint32_t)sp.hcount) return;

    // frequency along every axis (stored position -> frequency; the last axis is natural)
    uint32_t f[3] = {0, 0, 0};
    if (DIM >= 2) {
        uint32_t rem = row;
#pragma unroll
        for (int a = DIM - 2; a >= 0; --a) {
            const uint32_t sd = (uint32_t)sp.sdim[a];
            const uint32_t q = rem / sd;
            f[a] = pos_to_freq32(sp, a, rem - q * sd);
            rem = q;
        }
    }
    f[DIM - 1] = kl;

    const dcx* E0 = (const dcx*)sp.eph[0];
    const dcx* E1 = (const dcx*)sp.eph[DIM >= 2 ? 1 : 0];
    const dcx* El = (const dcx*)sp.eph[DIM - 1];
    const uint32_t n0 = (uint32_t)sp.n[0], n1 = (uint32_t)sp.n[DIM >= 2 ? 1 : 0], nl = (uint32_t)sp.n[DIM - 1];
    // innermost axis: E_l(o f_l) for o = -r .. r
    dcx el[W];
    {
        uint32_t m = start_index(RR, f[DIM - 1], nl);
#pragma unroll
        for (int o = 0; o < W; ++o) {
            el[o] = El[m];
            m = add_mod(m, f[DIM - 1], nl);
        }
    }
    const double* c = gp.c;
    dcx mu = {sp.one_minus_sum, 0.0};
    if (DIM == 1) {
#pragma unroll
        for (int o = 0; o < W; ++o) {
            mu.x = fma(-c[o], el[o].x, mu.x);
            mu.y = fma(-c[o], el[o].y, mu.y);
        }
    } else if (DIM == 2) {
        uint32_t m0 = start_index(RR, f[0], n0);
        for (int o0 = 0; o0 < W; ++o0) {
            const dcx e0 = E0[m0];
            m0 = add_mod(m0, f[0], n0);
            const double* cr = c + o0 * W;
#pragma unroll
            for (int o1 = 0; o1 < W; ++o1) {
                // (1 + e0)(1 + e1) - 1 = e0 + e1 + e0 e1
                const dcx d = dadd(dadd(e0, el[o1]), dmul(e0, el[o1]));
                mu.x = fma(-cr[o1], d.x, mu.x);
                mu.y = fma(-cr[o1], d.y, mu.y);
            }
        }
    } else {
        uint32_t m0 = start_index(RR, f[0], n0);
        const uint32_t s1 = start_index(RR, f[1], n1);
        for (int o0 = 0; o0 < W; ++o0) {
            const dcx e0 = E0[m0];
            m0 = add_mod(m0, f[0], n0);
            uint32_t m1 = s1;
            for (int o1 = 0; o1 < W; ++o1) {
                const dcx e1 = E1[m1];
                m1 = add_mod(m1, f[1], n1);
                const dcx d01 = dadd(dadd(e0, e1), dmul(e0, e1));
                const double* cr = c + (o0 * W + o1) * W;
#pragma unroll
                for (int o2 = 0; o2 < W; ++o2) {
                    const dcx d = dadd(dadd(d01, el[o2]), dmul(d01, el[o2]));
                    mu.x = fma(-cr[o2], d.x, mu.x);
                    mu.y = fma(-cr[o2], d.y, mu.y);
                }
            }
        }
    }
    dcx v;
    if (sp.real_sym) {
        double m1[1] = {mu.x}, o1[1];
        power_real_dev<1>(m1, o1, sp.T, sp.switching);
        v = dcx{o1[0] * sp.scale, 0.0};
    } else {
        dcx o1[1];
        power_complex_dev<1>(&mu, o1, sp.T, sp.switching);
        v = dcx{o1[0].x * sp.scale, o1[0].y * sp.scale};
    }
    cx<R>* ws = (cx<R>*)gp.ws + (int64_t)row * gp.pitch + kl;
    *ws = cmul(*ws, cx<R>{R(v.x), R(v.y)});
}

template <typename R, int RR>
void launch_r(const GeneralParams& gp, const SymParams& sp, dim3 g, hipStream_t st) {
    if (sp.d == 1) hipLaunchKernelGGL((k_symbol_general<R, RR, 1>), g, dim3(256), 0, st, gp, sp);
    else if (sp.d == 2) hipLaunchKernelGGL((k_symbol_general<R, RR, 2>), g, dim3(256), 0, st, gp, sp);
    else hipLaunchKernelGGL((k_symbol_general<R, RR, 3>), g, dim3(256), 0, st, gp, sp);
}

template <typename R>
hipError_t launch_t(const GeneralParams& gp, const SymParams& sp, hipStream_t st) {
    const int64_t cpr = (sp.hcount + 255) / 256;
    const dim3 g((unsigned)(cpr * gp.rows));
    switch (gp.r) {
        case 0: launch_r<R, 0>(gp, sp, g, st); break;
        case 1: launch_r<R, 1>(gp, sp, g, st); break;
        case 2: launch_r<R, 2>(gp, sp, g, st); break;
        case 3: launch_r<R, 3>(gp, sp, g, st); break;
        case 4: launch_r<R, 4>(gp, sp, g, st); break;
        case 5: launch_r<R, 5>(gp, sp, g, st); break;
        case 6: launch_r<R, 6>(gp, sp, g, st); break;
        case 7: launch_r<R, 7>(gp, sp, g, st); break;
        case 8: launch_r<R, 8>(gp, sp, g, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_symbol_general(const GeneralParams& gp, const SymParams& sp, bool f64, hipStream_t st) {
    return f64 ? launch_t<double>(gp, sp, st) : launch_t<float>(gp, sp, st);
}

}  // namespace sfft
