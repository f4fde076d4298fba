// The fused middle passes' symbol step: multiply the points a thread holds by
// lambda(k)^T * scale (Sec. 3 Steps 1(i), 2 and 3), for the register pass kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sfft_device.h"

namespace sfft {

// Multiply the thread's NP points by lambda(f0_i)^T * scale, f0_i = fbase + fstep * i
// (axis-0 frequencies, below 2^31), for a stencil of radius RR.  Groups of G
// independent FP64 chains run in a loop that is not unrolled (one copy of their
// registers); the results pass through thread-private slots of the tile's LDS,
// which is idle between the forward and the inverse transform.
template <typename R, int NTH, int RR, int NP = 16, int G = 4>
__device__ __forceinline__ void apply_symbol_r(cx<R>* v, cx<R>* lds, const SymParams& sp, const SymCol& col,
                                               uint32_t fbase, uint32_t fstep) {
    static_assert(NP % G == 0, "groups of G points");
    constexpr int NR = RR > 0 ? RR : 1;
    // Phase-table entries of the current group.  For radius 1 the next group's
    // entries are fetched while this one's power chains run; for radius 2 that
    // would cost more registers than it saves.
    constexpr bool PIPE = RR <= 1;
    dcx ec[NR][G], en[PIPE ? NR : 1][G];
    if (PIPE) phases_n<G, RR>(sp, fbase, fstep, ec);  // in flight across the barrier
    __syncthreads();
    auto fetch = [&](int g) {
        if constexpr (PIPE) {
            phases_n<G, RR>(sp, fbase + fstep * (uint32_t)((g + G) % NP), fstep, en);
        } else {
            phases_n<G, RR>(sp, fbase + fstep * (uint32_t)g, fstep, ec);
        }
    };
    auto advance = [&]() {
        if constexpr (PIPE) {
#pragma unroll
            for (int a = 0; a < NR; ++a)
#pragma unroll
                for (int e = 0; e < G; ++e) ec[a][e] = en[a][e];
        }
    };
    if (sp.real_sym) {
        R* sl = reinterpret_cast<R*>(lds);
#pragma unroll 1
        for (int g = 0; g < NP; g += G) {
            fetch(g);
            double m[G], o[G];
            symbol_mu_real_e<G, RR>(col, ec, m);
            power_real_dev<G>(m, o, sp.T, sp.switching);
#pragma unroll
            for (int e = 0; e < G; ++e) sl[threadIdx.x + NTH * (g + e)] = R(o[e] * sp.scale);
            advance();
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = scale(v[i], sl[threadIdx.x + NTH * i]);
    } else {
#pragma unroll 1
        for (int g = 0; g < NP; g += G) {
            fetch(g);
            dcx m[G], o[G];
            symbol_mu_e<G, RR>(col, ec, m);
            power_complex_dev<G>(m, o, sp.T, sp.switching);
#pragma unroll
            for (int e = 0; e < G; ++e) lds[threadIdx.x + NTH * (g + e)] = cx<R>{R(o[e].x * sp.scale), R(o[e].y * sp.scale)};
            advance();
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = cmul(v[i], lds[threadIdx.x + NTH * i]);
    }
}

template <typename R, int NTH = kThreads, int NP = 16, int G = 4>
__device__ __forceinline__ void apply_symbol(cx<R>* v, cx<R>* lds, const SymParams& sp, const SymCol& col, uint32_t fbase,
                                             uint32_t fstep) {
    static_assert(kMaxR == 2, "radius dispatch below covers 0..2");
    if (sp.r <= 0) apply_symbol_r<R, NTH, 0, NP, G>(v, lds, sp, col, fbase, fstep);
    else if (sp.r == 1) apply_symbol_r<R, NTH, 1, NP, G>(v, lds, sp, col, fbase, fstep);
    else apply_symbol_r<R, NTH, 2, NP, G>(v, lds, sp, col, fbase, fstep);
}


}  // namespace sfft
