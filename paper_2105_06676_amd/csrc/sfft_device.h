// Device building blocks: complex arithmetic, small DFT butterflies, LDS
// Stockham stages, twiddle lookups and the FP64 symbol / symbol-power code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_types.h"

namespace sfft {

template <typename R>
struct cx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
// Products write their fused multiply-adds out: a * b - c * d could otherwise be
// contracted either way round, and kernels compiled separately (direct and
// batched launches) would then round differently.
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return {fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -(a.x * b.y))};
}
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV>
__device__ __forceinline__ cx<R> rot90(cx<R> a) {
    return INV ? cx<R>{-a.y, a.x} : cx<R>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers: X[k] = sum_t v[t] exp(-+2 pi i t k / RAD)
// (minus sign forward, plus sign inverse).
// ---------------------------------------------------------------------------

template <int RAD>
struct RootTab;  // cos(2 pi m / RAD), sin(2 pi m / RAD), m = 0..RAD-1
template <>
struct RootTab<3> {
    static constexpr double c[3] = {1.0, -0.5, -0.5};
    static constexpr double s[3] = {0.0, 0.8660254037844386, -0.8660254037844386};
};
template <>
struct RootTab<5> {
    static constexpr double c[5] = {1.0, 0.30901699437494745, -0.8090169943749475,
                                    -0.8090169943749475, 0.30901699437494745};
    static constexpr double s[5] = {0.0, 0.9510565162951535, 0.5877852522924731,
                                    -0.5877852522924731, -0.9510565162951535};
};
template <>
struct RootTab<7> {
    static constexpr double c[7] = {1.0, 0.6234898018587335, -0.2225209339563144, -0.9009688679024191,
                                    -0.9009688679024191, -0.2225209339563144, 0.6234898018587335};
    static constexpr double s[7] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.4338837391175581,
                                    -0.4338837391175581, -0.9749279121818236, -0.7818314824680298};
};

template <>
struct RootTab<9> {
    static constexpr double c[9] = {1.0, 0.766044443118978, 0.17364817766693036, -0.5, -0.9396926207859084,
                                    -0.9396926207859084, -0.5, 0.17364817766693036, 0.766044443118978};
    static constexpr double s[9] = {0.0, 0.6427876096865394, 0.984807753012208, 0.8660254037844386,
                                    0.3420201433256687, -0.3420201433256687, -0.8660254037844386,
                                    -0.984807753012208, -0.6427876096865394};
};
template <>
struct RootTab<6> {
    static constexpr double c[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    static constexpr double s[6] = {0.0, 0.8660254037844386, 0.8660254037844386, 0.0, -0.8660254037844386,
                                    -0.8660254037844386};
};
template <>
struct RootTab<10> {
    static constexpr double c[10] = {1.0, 0.8090169943749475, 0.30901699437494745, -0.30901699437494745,
                                     -0.8090169943749475, -1.0, -0.8090169943749475, -0.30901699437494745,
                                     0.30901699437494745, 0.8090169943749475};
    static constexpr double s[10] = {0.0, 0.5877852522924731, 0.9510565162951535, 0.9510565162951535,
                                     0.5877852522924731, 0.0, -0.5877852522924731, -0.9510565162951535,
                                     -0.9510565162951535, -0.5877852522924731};
};
template <>
struct RootTab<12> {
    static constexpr double c[12] = {1.0, 0.8660254037844386, 0.5, 0.0, -0.5, -0.8660254037844386,
                                     -1.0, -0.8660254037844386, -0.5, 0.0, 0.5, 0.8660254037844386};
    static constexpr double s[12] = {0.0, 0.5, 0.8660254037844386, 1.0, 0.8660254037844386, 0.5,
                                     0.0, -0.5, -0.8660254037844386, -1.0, -0.8660254037844386, -0.5};
};
template <>
struct RootTab<20> {
    static constexpr double c[20] = {1.0, 0.9510565162951535, 0.8090169943749475, 0.5877852522924731,
                                     0.30901699437494745, 0.0, -0.30901699437494745, -0.5877852522924731,
                                     -0.8090169943749475, -0.9510565162951535, -1.0, -0.9510565162951535,
                                     -0.8090169943749475, -0.5877852522924731, -0.30901699437494745, 0.0,
                                     0.30901699437494745, 0.5877852522924731, 0.8090169943749475,
                                     0.9510565162951535};
    static constexpr double s[20] = {0.0, 0.30901699437494745, 0.5877852522924731, 0.8090169943749475,
                                     0.9510565162951535, 1.0, 0.9510565162951535, 0.8090169943749475,
                                     0.5877852522924731, 0.30901699437494745, 0.0, -0.30901699437494745,
                                     -0.5877852522924731, -0.8090169943749475, -0.9510565162951535, -1.0,
                                     -0.9510565162951535, -0.8090169943749475, -0.5877852522924731,
                                     -0.30901699437494745};
};
template <>
struct RootTab<25> {
    static constexpr double c[25] = {1.0, 0.9685831611286311, 0.8763066800438636, 0.7289686274214116,
                                     0.5358267949789967, 0.30901699437494745, 0.06279051952931337,
                                     -0.18738131458572463, -0.42577929156507266, -0.6374239897486897,
                                     -0.8090169943749475, -0.9297764858882515, -0.9921147013144779,
                                     -0.9921147013144779, -0.9297764858882515, -0.8090169943749475,
                                     -0.6374239897486897, -0.42577929156507266, -0.18738131458572463,
                                     0.06279051952931337, 0.30901699437494745, 0.5358267949789967,
                                     0.7289686274214116, 0.8763066800438636, 0.9685831611286311};
    static constexpr double s[25] = {0.0, 0.2486898871648548, 0.48175367410171527, 0.6845471059286887,
                                     0.8443279255020151, 0.9510565162951535, 0.9980267284282716,
                                     0.9822872507286887, 0.9048270524660196, 0.7705132427757893,
                                     0.5877852522924731, 0.368124552684678, 0.12533323356430426,
                                     -0.12533323356430426, -0.368124552684678, -0.5877852522924731,
                                     -0.7705132427757893, -0.9048270524660196, -0.9822872507286887,
                                     -0.9980267284282716, -0.9510565162951535, -0.8443279255020151,
                                     -0.6845471059286887, -0.48175367410171527, -0.2486898871648548};
};

template <>
struct RootTab<14> {
    static constexpr double c[14] = {1.0, 0.9009688679024191, 0.6234898018587335,
                                     0.2225209339563144, -0.2225209339563144,
                                     -0.6234898018587335, -0.9009688679024191, -1.0,
                                     -0.9009688679024191, -0.6234898018587335,
                                     -0.2225209339563144, 0.2225209339563144,
                                     0.6234898018587335, 0.9009688679024191};
    static constexpr double s[14] = {0.0, 0.4338837391175581, 0.7818314824680298,
                                     0.9749279121818236, 0.9749279121818236, 0.7818314824680298,
                                     0.4338837391175581, 0.0, -0.4338837391175581,
                                     -0.7818314824680298, -0.9749279121818236,
                                     -0.9749279121818236, -0.7818314824680298,
                                     -0.4338837391175581};
};
template <>
struct RootTab<15> {
    static constexpr double c[15] = {1.0, 0.9135454576426009, 0.6691306063588582,
                                     0.30901699437494745, -0.10452846326765347, -0.5,
                                     -0.8090169943749475, -0.9781476007338057,
                                     -0.9781476007338057, -0.8090169943749475, -0.5,
                                     -0.10452846326765347, 0.30901699437494745,
                                     0.6691306063588582, 0.9135454576426009};
    static constexpr double s[15] = {0.0, 0.4067366430758002, 0.7431448254773942,
                                     0.9510565162951535, 0.9945218953682733, 0.8660254037844386,
                                     0.5877852522924731, 0.20791169081775934,
                                     -0.20791169081775934, -0.5877852522924731,
                                     -0.8660254037844386, -0.9945218953682733,
                                     -0.9510565162951535, -0.7431448254773942,
                                     -0.4067366430758002};
};
template <>
struct RootTab<21> {
    static constexpr double c[21] = {1.0, 0.9555728057861407, 0.8262387743159949,
                                     0.6234898018587335, 0.36534102436639504,
                                     0.07473009358642425, -0.2225209339563144, -0.5,
                                     -0.7330518718298263, -0.9009688679024191,
                                     -0.9888308262251285, -0.9888308262251285,
                                     -0.9009688679024191, -0.7330518718298263, -0.5,
                                     -0.2225209339563144, 0.07473009358642425,
                                     0.36534102436639504, 0.6234898018587335,
                                     0.8262387743159949, 0.9555728057861407};
    static constexpr double s[21] = {0.0, 0.2947551744109042, 0.5633200580636221,
                                     0.7818314824680298, 0.9308737486442042, 0.9972037971811801,
                                     0.9749279121818236, 0.8660254037844386, 0.6801727377709194,
                                     0.4338837391175581, 0.14904226617617444,
                                     -0.14904226617617444, -0.4338837391175581,
                                     -0.6801727377709194, -0.8660254037844386,
                                     -0.9749279121818236, -0.9972037971811801,
                                     -0.9308737486442042, -0.7818314824680298,
                                     -0.5633200580636221, -0.2947551744109042};
};

template <typename R, bool INV>
__device__ __forceinline__ void dft2(cx<R>* v) {
    cx<R> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cx<R>& v0, cx<R>& v1, cx<R>& v2, cx<R>& v3) {
    cx<R> t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = rot90<R, INV>(v1 - v3);
    v0 = t0 + t2;
    v2 = t0 - t2;
    v1 = t1 + t3;
    v3 = t1 - t3;
}

template <typename R, bool INV>
__device__ __forceinline__ void dft8(cx<R>* v) {
    constexpr R h = R(0.7071067811865476);
    cx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cx<R> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<R, INV>(e0, e1, e2, e3);
    dft4<R, INV>(o0, o1, o2, o3);
    // twiddles w^k, w = exp(-+ 2 pi i / 8)
    cx<R> w1 = INV ? cx<R>{h * (o1.x - o1.y), h * (o1.x + o1.y)} : cx<R>{h * (o1.x + o1.y), h * (o1.y - o1.x)};
    cx<R> w2 = rot90<R, INV>(o2);
    cx<R> w3 = INV ? cx<R>{-h * (o3.x + o3.y), h * (o3.x - o3.y)} : cx<R>{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + w1;
    v[5] = e1 - w1;
    v[2] = e2 + w2;
    v[6] = e2 - w2;
    v[3] = e3 + w3;
    v[7] = e3 - w3;
}

// Odd radix by the symmetric pairing of t and RAD - t.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft_odd(cx<R>* v) {
    constexpr int H = (RAD - 1) / 2;
    cx<R> a[H], b[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        a[j - 1] = v[j] + v[RAD - j];
        b[j - 1] = v[j] - v[RAD - j];
    }
    cx<R> out[RAD];
    cx<R> s0 = v[0];
#pragma unroll
    for (int j = 0; j < H; ++j) s0 = s0 + a[j];
    out[0] = s0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        cx<R> re = v[0];
        cx<R> im = {R(0), R(0)};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const R cc = R(RootTab<RAD>::c[(j * k) % RAD]);
            const R ss = R(RootTab<RAD>::s[(j * k) % RAD]);
            re = re + scale(a[j - 1], cc);
            im = im + scale(b[j - 1], ss);
        }
        // forward: X_k = re - i im, X_{RAD-k} = re + i im
        cx<R> r90 = rot90<R, INV>(im);
        out[k] = re + r90;
        out[RAD - k] = re - r90;
    }
#pragma unroll
    for (int k = 0; k < RAD; ++k) v[k] = out[k];
}

// a * exp(-+2 pi i m / N) for an m that is a constant once the caller's loops
// are unrolled (quarter turns exactly, the rest from the root table).
template <typename R, int N, bool INV>
__device__ __forceinline__ cx<R> twiddle_n(cx<R> a, int m) {
    m %= N;
    if (m == 0) return a;
    if ((4 * m) % N == 0) {
        const int qt = 4 * m / N;
        if (qt == 1) return rot90<R, INV>(a);
        if (qt == 2) return cx<R>{-a.x, -a.y};
        return rot90<R, !INV>(a);
    }
    const R c = R(RootTab<N>::c[m]), sn = R(RootTab<N>::s[m]);
    // forward: a (c - i s); inverse: a (c + i s)
    return INV ? cx<R>{fma(-a.y, sn, a.x * c), fma(a.x, sn, a.y * c)}
               : cx<R>{fma(a.y, sn, a.x * c), fma(-a.x, sn, a.y * c)};
}

template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cx<R>* v);

// Composite radix N = A B (Cooley-Tukey inside the registers): with n = B n1 + n2
// and k = k1 + A k2, X[k] = sum_n2 W_B^(n2 k2) W_N^(n2 k1) sum_n1 x[B n1 + n2] W_A^(n1 k1):
// B transforms of length A, the twiddles W_N^(n2 k1), then A transforms of length B.
template <typename R, int A, int B, bool INV>
__device__ __forceinline__ void dft_ab(cx<R>* v) {
    constexpr int N = A * B;
    cx<R> y[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) y[n2][n1] = v[B * n1 + n2];
        dft<R, A, INV>(y[n2]);
#pragma unroll
        for (int k1 = 1; k1 < A; ++k1)
            if (n2 > 0) y[n2][k1] = twiddle_n<R, N, INV>(y[n2][k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        cx<R> z[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) z[n2] = y[n2][k1];
        dft<R, B, INV>(z);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = z[k2];
    }
}

template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cx<R>* v) {
    if constexpr (RAD == 2) dft2<R, INV>(v);
    else if constexpr (RAD == 4) dft4<R, INV>(v[0], v[1], v[2], v[3]);
    else if constexpr (RAD == 8) dft8<R, INV>(v);
    else if constexpr (RAD == 6) dft_ab<R, 3, 2, INV>(v);
    else if constexpr (RAD == 9) dft_ab<R, 3, 3, INV>(v);
    else if constexpr (RAD == 10) dft_ab<R, 5, 2, INV>(v);
    else if constexpr (RAD == 12) dft_ab<R, 4, 3, INV>(v);
    else if constexpr (RAD == 14) dft_ab<R, 7, 2, INV>(v);
    else if constexpr (RAD == 15) dft_ab<R, 5, 3, INV>(v);
    else if constexpr (RAD == 20) dft_ab<R, 4, 5, INV>(v);
    else if constexpr (RAD == 21) dft_ab<R, 7, 3, INV>(v);
    else if constexpr (RAD == 25) dft_ab<R, 5, 5, INV>(v);
    else dft_odd<R, RAD, INV>(v);
}

// ---------------------------------------------------------------------------
// Division by a divisor n >= 1 that is the same for the whole workgroup, for
// dividends e < 2^22, through a float reciprocal: (e + 1/2) / n lies at least
// 1/(2n) away from the nearest integer, while the two float roundings of
// (e + 1/2) * fl(1/n) move it by at most (e + 1/2) / n * 2^-23 < 1/(2n), so
// truncation gives floor(e / n).  About 4 instructions instead of the ~20 of an
// integer division expansion.
struct UDiv {
    uint32_t n;
    float inv;
};
__device__ __forceinline__ UDiv udiv(uint32_t n) { return UDiv{n, 1.0f / (float)n}; }
__device__ __forceinline__ uint32_t udiv_q(uint32_t e, UDiv d) {
    return (uint32_t)(((float)e + 0.5f) * d.inv);
}
// q = e / n, returns e - q n
__device__ __forceinline__ uint32_t udiv_qr(uint32_t e, UDiv d, uint32_t* q) {
    *q = udiv_q(e, d);
    return e - *q * d.n;
}

// ---------------------------------------------------------------------------
// One Stockham radix-RAD stage over every transform of an LDS tile.
// Transform `tr` element `e` lives at lds[tr * ts + e * es].  With Ns the product
// of the radices already applied, butterfly j reads elements j + t * L/RAD,
// multiplies by exp(-+2 pi i t (j mod Ns) / (Ns RAD)), runs a RAD-point DFT and
// writes element (j / Ns) * Ns * RAD + (j mod Ns) + t * Ns (self-sorting order).
// TFAST: consecutive threads take consecutive transforms (column tiles);
// otherwise consecutive butterflies of one transform (row tiles).
// ---------------------------------------------------------------------------
template <typename R, int RAD, bool INV, bool TFAST>
__device__ __forceinline__ void stage(cx<R>* lds, int L, int ntrans, int ts, int es, int Ns,
                                      const cx<R>* __restrict__ tab, int tmul) {
    const int nb = L / RAD;
    const int total = nb * ntrans;
    constexpr int MAXIT = (kTileElems + RAD * gen_threads<R>() - 1) / (RAD * gen_threads<R>());
    cx<R> v[MAXIT][RAD];
    const int step = (L / (Ns * RAD)) * tmul;
    // (total <= kTileElems / RAD < 2^22)
    const UDiv dsplit = udiv((uint32_t)(TFAST ? ntrans : nb)), dns = udiv((uint32_t)Ns);
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int e = threadIdx.x + it * gen_threads<R>();
        if (e < total) {
            uint32_t tr, j;
            if (TFAST) tr = udiv_qr((uint32_t)e, dsplit, &j);
            else j = udiv_qr((uint32_t)e, dsplit, &tr);
            const cx<R>* base = lds + tr * ts;
#pragma unroll
            for (int t = 0; t < RAD; ++t) v[it][t] = base[(j + t * nb) * es];
            uint32_t jq;
            const int k = (int)udiv_qr(j, dns, &jq);
            if (Ns > 1 && k != 0) {
                const cx<R> w = tab[k * step];
                cx<R> wt = w;
#pragma unroll
                for (int t = 1; t < RAD; ++t) {
                    v[it][t] = INV ? cmulc(v[it][t], wt) : cmul(v[it][t], wt);
                    if (t + 1 < RAD) wt = cmul(wt, w);
                }
            }
            dft<R, RAD, INV>(v[it]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int e = threadIdx.x + it * gen_threads<R>();
        if (e < total) {
            uint32_t tr, j;
            if (TFAST) tr = udiv_qr((uint32_t)e, dsplit, &j);
            else j = udiv_qr((uint32_t)e, dsplit, &tr);
            cx<R>* base = lds + tr * ts;
            uint32_t jq;
            const int k = (int)udiv_qr(j, dns, &jq);
            const int dst = (int)jq * Ns * RAD + k;
#pragma unroll
            for (int t = 0; t < RAD; ++t) base[(dst + t * Ns) * es] = v[it][t];
        }
    }
    __syncthreads();
}

// Full transform of length L (radix list in the pass descriptor) on every
// transform of the tile.
template <typename R, bool INV, bool TFAST>
__device__ void tile_fft(cx<R>* lds, const PassDesc& pd, int ntrans, int ts, int es) {
    const cx<R>* tab = (const cx<R>*)pd.st_tab;
    int Ns = 1;
    for (int s = 0; s < pd.nst; ++s) {
        switch (pd.radix[s]) {
            case 2: stage<R, 2, INV, TFAST>(lds, pd.L, ntrans, ts, es, Ns, tab, pd.st_mul); break;
            case 3: stage<R, 3, INV, TFAST>(lds, pd.L, ntrans, ts, es, Ns, tab, pd.st_mul); break;
            case 4: stage<R, 4, INV, TFAST>(lds, pd.L, ntrans, ts, es, Ns, tab, pd.st_mul); break;
            case 5: stage<R, 5, INV, TFAST>(lds, pd.L, ntrans, ts, es, Ns, tab, pd.st_mul); break;
            case 7: stage<R, 7, INV, TFAST>(lds, pd.L, ntrans, ts, es, Ns, tab, pd.st_mul); break;
            default: stage<R, 8, INV, TFAST>(lds, pd.L, ntrans, ts, es, Ns, tab, pd.st_mul); break;
        }
        Ns *= pd.radix[s];
    }
}

// Twiddle between sub-transforms, exp(-2 pi i e / tw_n) from a two-level table.
template <typename R>
__device__ __forceinline__ cx<R> step_twiddle(const PassDesc& pd, int64_t e) {
    const cx<R>* lo = (const cx<R>*)pd.tw_lo;
    const cx<R>* hi = (const cx<R>*)pd.tw_hi;
    const uint32_t u = (uint32_t)e;  // e < tw_n <= 2^31
    cx<R> w = lo[u & (kTwSplit - 1)];
    const uint32_t q = u >> kTwSplitLog;
    if (q) w = cmul(w, hi[q]);
    return w;
}

// ---------------------------------------------------------------------------
// Region bookkeeping for the last pass: may local cell (b, i) be stored?
// ---------------------------------------------------------------------------
// The part of the test that is fixed along a row: distance and first face over
// the axes before the last one.
// a[i] for i in 0..2 through selects (a runtime index into a small array would
// place the array in scratch memory).
__device__ __forceinline__ int64_t pick3(const int64_t* a, int i) {
    return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}

struct RowKeep {
    int64_t epre;   // min face entry time over axes 0..d-2 (huge if none)
    int fpre;       // first face (in face order) with that entry time
};

// Entry time of a face at distance dist (1-based) along axis a.
__device__ __forceinline__ int64_t entry_time(const KeepRule& kr, int a, int64_t dist) {
    return ((kr.half_axes >> a) & 1) ? (dist + 1) >> 1 : dist;
}

__device__ __forceinline__ RowKeep keep_row(const KeepRule& kr, int d, int64_t b, const int64_t* i) {
    RowKeep rk{INT64_MAX, -1};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (a < d - 1) {
            const int64_t g = kr.gorg[a] + b * kr.gbstep[a] + i[a];
            const int64_t lo = entry_time(kr, a, g + 1), hi = entry_time(kr, a, kr.gdim[a] - g);
            if (lo < rk.epre) { rk.epre = lo; rk.fpre = 2 * a; }
            if (hi < rk.epre) { rk.epre = hi; rk.fpre = 2 * a + 1; }
        }
    }
    return rk;
}

// May cell m of the last axis of a row be stored?
__device__ __forceinline__ bool keep_last(const KeepRule& kr, const RowKeep& rk, int d, int64_t b, int64_t m) {
    const int L = d - 1;
    const int64_t g = pick3(kr.gorg, L) + b * pick3(kr.gbstep, L) + m;
    const int64_t lo = entry_time(kr, L, g + 1), hi = entry_time(kr, L, pick3(kr.gdim, L) - g);
    int64_t ell = rk.epre;
    int first = rk.fpre;
    if (lo < ell) { ell = lo; first = 2 * L; }
    if (hi < ell) { ell = hi; first = 2 * L + 1; }
    if (!(ell > kr.lo && ell <= kr.hi)) return false;
    if (kr.face_axis < 0) return true;
    if (first / 2 != kr.face_axis) return false;
    const int side = kr.face_side == 2 ? (int)b : kr.face_side;
    return side < 0 || (first & 1) == side;
}

// May any cell of a row along the last axis pass keep_last?  False only when none
// can: every cell's entry time is at most epre, and a last-axis face is the first
// face only when its entry time is strictly below epre.
__device__ __forceinline__ bool row_may_keep(const KeepRule& kr, const RowKeep& rk, int d, int64_t b) {
    if (rk.epre <= kr.lo) return false;
    if (kr.face_axis >= 0 && kr.face_axis != d - 1) {
        if (rk.epre > kr.hi) return false;
        if (rk.fpre / 2 != kr.face_axis) return false;
        const int side = kr.face_side == 2 ? (int)b : kr.face_side;
        if (side >= 0 && (rk.fpre & 1) != side) return false;
    }
    return true;
}

__device__ __forceinline__ bool keep_cell(const KeepRule& kr, int d, int64_t b, const int64_t* i) {
    if (!kr.enabled) return true;
    return keep_last(kr, keep_row(kr, d, b, i), d, b, pick3(i, d - 1));
}

// ---------------------------------------------------------------------------
// Symbol and symbol power, always FP64.
//
// lambda(k) = sum_o c[o] prod_a exp(2 pi i o_a k_a / n_a) (= (F s)[k], the DFT of
// the circulant matrix's first column; appendix, eigenvalue-FFT relation).  It is
// carried as mu = 1 - lambda so that modes with lambda close to 1, which
// dominate long runs, keep their relative accuracy: with E_a(m) = exp(2 pi i m /
// n_a) - 1 tabulated,
//   lambda = sum(c) + sum_{o0} D[o0] + sum_{o0} E_0(o0 k0) G[o0]
//   G[o0] = sum_{o'} c[o0, o'] prod_{a>0} (1 + E_a(o_a k_a))
//   D[o0] = sum_{o'} c[o0, o'] (prod_{a>0} (1 + E_a(o_a k_a)) - 1)
// so mu = (1 - sum c) - sum D - sum_{o0} E_0 G with no cancellation.
// ---------------------------------------------------------------------------
struct dcx {
    double x, y;
};
__device__ __forceinline__ dcx dmul(dcx a, dcx b) {
    return {fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ dcx dadd(dcx a, dcx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ dcx dsub(dcx a, dcx b) { return {a.x - b.x, a.y - b.y}; }

__device__ __forceinline__ int64_t pos_to_freq(const SymParams& sp, int a, int64_t p) {
    const int nl = sp.nlev[a];
    if (nl <= 1) return p;
    if (nl == 2) {
        const int64_t s0 = sp.sub[a][0], s1 = sp.sub[a][1];
        const int64_t d0 = p / s1, d1 = p - d0 * s1;
        return d0 + s0 * d1;
    }
    const int64_t s0 = sp.sub[a][0], s1 = sp.sub[a][1], s2 = sp.sub[a][2];
    const int64_t d0 = p / (s1 * s2);
    const int64_t rem = p - d0 * s1 * s2;
    const int64_t d1 = rem / s2, d2 = rem - d1 * s2;
    return d0 + s0 * (d1 + s1 * d2);
}

// Stored position -> frequency along axis a in 32-bit arithmetic (extents below 2^31).
__device__ __forceinline__ uint32_t pos_to_freq32(const SymParams& sp, int a, uint32_t p) {
    const int nl = sp.nlev[a];
    if (nl <= 1) return p;
    const uint32_t s0 = (uint32_t)sp.sub[a][0], s1 = (uint32_t)sp.sub[a][1];
    if (nl == 2) {
        const uint32_t d0 = p / s1, d1 = p - d0 * s1;
        return d0 + s0 * d1;
    }
    const uint32_t s2 = (uint32_t)sp.sub[a][2];
    const uint32_t d0 = p / (s1 * s2), rem = p - d0 * s1 * s2;
    const uint32_t d1 = rem / s2, d2 = rem - d1 * s2;
    return d0 + s0 * (d1 + s1 * d2);
}

// E_a((o * k) mod n_a) for offset o in [-r, r]
__device__ __forceinline__ dcx eph(const SymParams& sp, int a, int o, int64_t k) {
    const int64_t n = sp.n[a];
    int64_t m = ((int64_t)(o < 0 ? -o : o) * k) % n;
    const dcx* t = (const dcx*)sp.eph[a];
    dcx e = t[m];
    if (o < 0) e.y = -e.y;  // E(-m) = conj(E(m))
    return e;
}

// Per-column part of the symbol for the axis-1..d-1 frequencies f: G[o0] for
// o0 = +1..+r (Gp) and -1..-r (Gm), and K = (1 - sum c) - sum_{o0} D[o0].  All
// arrays are indexed by compile-time offsets so they stay in registers.
struct SymCol {
    dcx Gp[kMaxR + 1], Gm[kMaxR + 1];
    dcx K;
};

// E_a((o * f) mod n_a) for o in [-kMaxR, kMaxR] (32-bit index arithmetic).
// (o * f) mod n for 0 <= f < n <= 2^31 and 0 <= o <= kMaxR, by conditional
// subtraction (o * f < kMaxR * n) instead of an integer division.
__device__ __forceinline__ uint32_t mul_mod_small(uint32_t o, uint32_t f, uint32_t n) {
    uint32_t m = o * f;
#pragma unroll
    for (int k = 1; k < kMaxR; ++k) m = m >= n ? m - n : m;
    return m;
}

__device__ __forceinline__ dcx eph32(const SymParams& sp, int a, int o, uint32_t f) {
    const uint32_t n = (uint32_t)sp.n[a];
    const uint32_t m = mul_mod_small((uint32_t)(o < 0 ? -o : o), f, n);
    dcx e = ((const dcx*)sp.eph[a])[m];
    if (o < 0) e.y = -e.y;  // E(-m) = conj(E(m))
    return e;
}

__device__ inline SymCol symbol_column(const SymParams& sp, const int64_t* f) {
    SymCol out;
    const int r = sp.r, w = 2 * r + 1;
    // phases of axes 1 and 2 for every offset, looked up once
    dcx e1[2 * kMaxR + 1], e2[2 * kMaxR + 1];
#pragma unroll
    for (int o = -kMaxR; o <= kMaxR; ++o) {
        e1[o + kMaxR] = (sp.d >= 2 && o >= -r && o <= r) ? eph32(sp, 1, o, (uint32_t)f[1]) : dcx{0.0, 0.0};
        e2[o + kMaxR] = (sp.d >= 3 && o >= -r && o <= r) ? eph32(sp, 2, o, (uint32_t)f[2]) : dcx{0.0, 0.0};
    }
    dcx dsum = {0.0, 0.0};
#pragma unroll
    for (int o0 = -kMaxR; o0 <= kMaxR; ++o0) {
        dcx g = {0.0, 0.0}, dd = {0.0, 0.0};
        if (o0 >= -r && o0 <= r) {
            if (sp.d == 1) {
                g.x = sp.c[o0 + r];
            } else if (sp.d == 2) {
#pragma unroll
                for (int o1 = -kMaxR; o1 <= kMaxR; ++o1) {
                    if (o1 < -r || o1 > r) continue;
                    const double c = sp.c[(o0 + r) * w + (o1 + r)];
                    const dcx p = e1[o1 + kMaxR];
                    g = dadd(g, dcx{c * (1.0 + p.x), c * p.y});
                    dd = dadd(dd, dcx{c * p.x, c * p.y});
                }
            } else {
#pragma unroll
                for (int o1 = -kMaxR; o1 <= kMaxR; ++o1) {
                    if (o1 < -r || o1 > r) continue;
                    const dcx a1 = e1[o1 + kMaxR];
#pragma unroll
                    for (int o2 = -kMaxR; o2 <= kMaxR; ++o2) {
                        if (o2 < -r || o2 > r) continue;
                        const double c = sp.c[((o0 + r) * w + (o1 + r)) * w + (o2 + r)];
                        const dcx a2 = e2[o2 + kMaxR];
                        const dcx p = dadd(dadd(a1, a2), dmul(a1, a2));
                        g = dadd(g, dcx{c * (1.0 + p.x), c * p.y});
                        dd = dadd(dd, dcx{c * p.x, c * p.y});
                    }
                }
            }
            dsum = dadd(dsum, dd);
        }
        if (o0 > 0) out.Gp[o0] = g;
        if (o0 < 0) out.Gm[-o0] = g;
    }
    out.Gp[0] = out.Gm[0] = dcx{0.0, 0.0};
    out.K = dcx{sp.one_minus_sum - dsum.x, -dsum.y};
    return out;
}

// 1-D symbol: G = c, K = 1 - sum c.
__device__ inline SymCol symbol_column_1d(const SymParams& sp) {
    SymCol out;
#pragma unroll
    for (int o = 0; o <= kMaxR; ++o) {
        out.Gp[o] = dcx{o >= 1 && o <= sp.r ? sp.c[sp.r + o] : 0.0, 0.0};
        out.Gm[o] = dcx{o >= 1 && o <= sp.r ? sp.c[sp.r - o] : 0.0, 0.0};
    }
    out.K = dcx{sp.one_minus_sum, 0.0};
    return out;
}

// mu = 1 - lambda at axis-0 frequency f0 given the column part.
__device__ __forceinline__ dcx symbol_mu(const SymParams& sp, const SymCol& col, int64_t f0) {
    dcx mu = col.K;
    const uint32_t n = (uint32_t)sp.n[0];
    const dcx* t = (const dcx*)sp.eph[0];
    const uint32_t f = (uint32_t)f0;
#pragma unroll
    for (int o = 1; o <= kMaxR; ++o) {
        if (o <= sp.r) {
            const uint32_t m = mul_mod_small((uint32_t)o, f, n);
            const dcx e = t[m];
            const dcx ec = {e.x, -e.y};
            mu = dsub(mu, dadd(dmul(e, col.Gp[o]), dmul(ec, col.Gm[o])));
        }
    }
    return mu;
}

// mu for a point-symmetric stencil (c(-o) = c(o)), where lambda is real: the
// column parts of opposite axis-0 offsets are conjugate (Gm = conj Gp), so the
// two terms of an offset pair sum to 2 Re(E Gp).
__device__ __forceinline__ double symbol_mu_real(const SymParams& sp, const SymCol& col, uint32_t f) {
    double mu = col.K.x;
    const uint32_t n = (uint32_t)sp.n[0];
    const dcx* t = (const dcx*)sp.eph[0];
#pragma unroll
    for (int o = 1; o <= kMaxR; ++o) {
        if (o <= sp.r) {
            const uint32_t m = mul_mod_small((uint32_t)o, f, n);
            const dcx e = t[m];
            mu -= 2.0 * fma(e.x, col.Gp[o].x, -e.y * col.Gp[o].y);
        }
    }
    return mu;
}

// The same two quantities for G frequencies f + k * fstep (k < G) of one column,
// for a stencil of radius exactly RR, from phase-table entries fetched by
// phases_n.  The table lives in L2: fetching all RR * G entries of a group at
// once (and ahead of use) costs one round trip per group instead of one per mode.
// The arithmetic is that of symbol_mu / symbol_mu_real, term for term.
template <int G, int RR>
__device__ __forceinline__ void phases_n(const SymParams& sp, uint32_t f, uint32_t fstep, dcx (*e)[G]) {
    const uint32_t n = (uint32_t)sp.n[0];
    const dcx* t = (const dcx*)sp.eph[0];
#pragma unroll
    for (int o = 1; o <= RR; ++o)
#pragma unroll
        for (int k = 0; k < G; ++k) e[o - 1][k] = t[mul_mod_small((uint32_t)o, f + fstep * (uint32_t)k, n)];
}

template <int G, int RR>
__device__ __forceinline__ void symbol_mu_real_e(const SymCol& col, const dcx (*e)[G], double* mu) {
#pragma unroll
    for (int k = 0; k < G; ++k) {
        mu[k] = col.K.x;
#pragma unroll
        for (int o = 1; o <= RR; ++o)
            mu[k] -= 2.0 * fma(e[o - 1][k].x, col.Gp[o].x, -e[o - 1][k].y * col.Gp[o].y);
    }
}

template <int G, int RR>
__device__ __forceinline__ void symbol_mu_e(const SymCol& col, const dcx (*e)[G], dcx* mu) {
#pragma unroll
    for (int k = 0; k < G; ++k) {
        mu[k] = col.K;
#pragma unroll
        for (int o = 1; o <= RR; ++o) {
            const dcx ec = {e[o - 1][k].x, -e[o - 1][k].y};
            mu[k] = dsub(mu[k], dadd(dmul(e[o - 1][k], col.Gp[o]), dmul(ec, col.Gm[o])));
        }
    }
}

// (1 - mu)^T by binary repeated squaring (Sec. 3 Step 2), in deviation form:
// a factor 1 - m squares to 1 - (2m - m^2) and (1 - v)(1 - m) = 1 - (v + m - vm);
// a factor leaves the deviation form once |m| > 1/2, where plain products are
// just as accurate.
// Deviation-form steps on complex values, written out in fused multiply-adds:
//   square:   m <- 2m - m^2:   re = 2a - a^2 + b^2, im = 2b - 2ab = 2b (1 - a)
//   multiply: v <- v + m - vm: re = v.x + m.x - v.x m.x + v.y m.y,
//                              im = v.y + m.y - v.x m.y - v.y m.x
// (5 and 6 FP64 operations instead of the 8 of the complex-arithmetic form).
__device__ __forceinline__ dcx dev_square(dcx m) {
    const double a2 = m.x + m.x, b2 = m.y + m.y;
    return dcx{fma(-m.x, m.x, fma(m.y, m.y, a2)), fma(-b2, m.x, b2)};
}
__device__ __forceinline__ dcx dev_mul(dcx v, dcx m) {
    return dcx{fma(-v.x, m.x, fma(v.y, m.y, v.x + m.x)), fma(-v.x, m.y, fma(-v.y, m.x, v.y + m.y))};
}

__device__ inline dcx power_complex(dcx mu, int64_t T) {
    bool sq_dev = true, v_dev = true;
    dcx sq = mu, v = {0.0, 0.0};
    if (mu.x * mu.x + mu.y * mu.y > 0.25) { sq = dcx{1.0 - mu.x, -mu.y}; sq_dev = false; }
    int64_t R = T;
    while (R > 0) {
        if (R & 1) {
            if (v_dev && sq_dev) {
                v = dev_mul(v, sq);
            } else {
                const dcx a = v_dev ? dcx{1.0 - v.x, -v.y} : v;
                const dcx b = sq_dev ? dcx{1.0 - sq.x, -sq.y} : sq;
                v = dmul(a, b);
                v_dev = false;
            }
        }
        R >>= 1;
        if (R) {
            if (sq_dev) {
                sq = dev_square(sq);
                if (sq.x * sq.x + sq.y * sq.y > 0.25) { sq = dcx{1.0 - sq.x, -sq.y}; sq_dev = false; }
            } else {
                sq = dmul(sq, sq);
            }
        }
    }
    return v_dev ? dcx{1.0 - v.x, -v.y} : v;
}

__device__ inline double power_real(double mu, int64_t T) {
    bool sq_dev = true, v_dev = true;
    double sq = mu, v = 0.0;
    if (fabs(mu) > 0.5) { sq = 1.0 - mu; sq_dev = false; }
    int64_t R = T;
    while (R > 0) {
        if (R & 1) {
            if (v_dev && sq_dev) {
                v = (v + sq) - v * sq;
            } else {
                v = (v_dev ? 1.0 - v : v) * (sq_dev ? 1.0 - sq : sq);
                v_dev = false;
            }
        }
        R >>= 1;
        if (R) {
            if (sq_dev) {
                sq = 2.0 * sq - sq * sq;
                if (fabs(sq) > 0.5) { sq = 1.0 - sq; sq_dev = false; }
            } else {
                sq = sq * sq;
            }
        }
    }
    return v_dev ? 1.0 - v : v;
}

// lambda^T * scale for a mode, from its per-column part and axis-0 frequency.
__device__ __forceinline__ dcx symbol_power_at(const SymParams& sp, const SymCol& col, int64_t f0) {
    const dcx mu = symbol_mu(sp, col, f0);
    if (sp.real_sym) return dcx{power_real(mu.x, sp.T) * sp.scale, 0.0};
    const dcx v = power_complex(mu, sp.T);
    return dcx{v.x * sp.scale, v.y * sp.scale};
}


// Branch-free form for the solver's middle passes: the deviations of the running
// square (1 - lambda^(2^k)) and of the product are updated for N modes at once
// (independent chains for instruction-level parallelism) over the bits of T,
// which are the same for every lane.  Every mode keeps lambda^T within a few
// ulps of absolute error, which is relative accuracy for the dominant modes as
// long as the largest |lambda| is 1: the host guarantees that by dividing
// coefficients of one sign by lambda(0) = sum(c) (then |lambda(k)| <= lambda(0))
// and folding lambda(0)^T into the scale.  Stencils of mixed sign have no such
// bound and take the switching form per mode instead (SWITCHING = true), which
// keeps every mode's relative accuracy at the price of divergent branches.
template <int N>
__device__ __forceinline__ void power_real_dev(double* mu, double* out, int64_t T, bool switching) {
    if (switching) {
#pragma unroll
        for (int e = 0; e < N; ++e) out[e] = power_real(mu[e], T);
        return;
    }
    double v[N];
#pragma unroll
    for (int e = 0; e < N; ++e) v[e] = 0.0;
    for (int64_t R = T; R > 0; R >>= 1) {
        if (R & 1) {
#pragma unroll
            for (int e = 0; e < N; ++e) v[e] = fma(-v[e], mu[e], v[e] + mu[e]);
        }
        if (R > 1) {
#pragma unroll
            for (int e = 0; e < N; ++e) mu[e] = fma(-mu[e], mu[e], 2.0 * mu[e]);
        }
    }
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = 1.0 - v[e];
}

template <int N>
__device__ __forceinline__ void power_complex_dev(dcx* mu, dcx* out, int64_t T, bool switching) {
    if (switching) {
#pragma unroll
        for (int e = 0; e < N; ++e) out[e] = power_complex(mu[e], T);
        return;
    }
    dcx v[N];
#pragma unroll
    for (int e = 0; e < N; ++e) v[e] = dcx{0.0, 0.0};
    for (int64_t R = T; R > 0; R >>= 1) {
        if (R & 1) {
#pragma unroll
            for (int e = 0; e < N; ++e) v[e] = dev_mul(v[e], mu[e]);
        }
        if (R > 1) {
#pragma unroll
            for (int e = 0; e < N; ++e) mu[e] = dev_square(mu[e]);
        }
    }
#pragma unroll
    for (int e = 0; e < N; ++e) out[e] = dcx{1.0 - v[e].x, -v[e].y};
}

// lambda^T * scale for G modes of one column at axis-0 frequencies f[g] (below
// 2^31), for a stencil of radius exactly RR: the RR * G phase reads are issued
// before the first is used; the arithmetic is that of symbol_power_n.
template <int G, int RR>
__device__ __forceinline__ void symbol_power_g(const SymParams& sp, const SymCol& col, const uint32_t* f, dcx* out) {
    const uint32_t n = (uint32_t)sp.n[0];
    const dcx* t = (const dcx*)sp.eph[0];
    dcx e[RR > 0 ? RR : 1][G];
#pragma unroll
    for (int o = 1; o <= RR; ++o)
#pragma unroll
        for (int k = 0; k < G; ++k) e[o - 1][k] = t[mul_mod_small((uint32_t)o, f[k], n)];
    dcx mu[G];
    symbol_mu_e<G, RR>(col, e, mu);
    if (sp.real_sym) {
        double m[G], o[G];
#pragma unroll
        for (int k = 0; k < G; ++k) m[k] = mu[k].x;
        power_real_dev<G>(m, o, sp.T, sp.switching);
#pragma unroll
        for (int k = 0; k < G; ++k) out[k] = dcx{o[k] * sp.scale, 0.0};
    } else {
        dcx o[G];
        power_complex_dev<G>(mu, o, sp.T, sp.switching);
#pragma unroll
        for (int k = 0; k < G; ++k) out[k] = dcx{o[k].x * sp.scale, o[k].y * sp.scale};
    }
}

// lambda^T * scale for N modes of one column at axis-0 frequencies f0[e].
template <int N>
__device__ __forceinline__ void symbol_power_n(const SymParams& sp, const SymCol& col, const int64_t* f0, dcx* out) {
    dcx mu[N];
#pragma unroll
    for (int e = 0; e < N; ++e) mu[e] = symbol_mu(sp, col, f0[e]);
    if (sp.real_sym) {
        double m[N], o[N];
#pragma unroll
        for (int e = 0; e < N; ++e) m[e] = mu[e].x;
        power_real_dev<N>(m, o, sp.T, sp.switching);
#pragma unroll
        for (int e = 0; e < N; ++e) out[e] = dcx{o[e] * sp.scale, 0.0};
    } else {
        dcx o[N];
        power_complex_dev<N>(mu, o, sp.T, sp.switching);
#pragma unroll
        for (int e = 0; e < N; ++e) out[e] = dcx{o[e].x * sp.scale, o[e].y * sp.scale};
    }
}

}  // namespace sfft
