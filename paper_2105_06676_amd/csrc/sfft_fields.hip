// Symbol-matrix power for m coupled fields, applied to their spectra.
//
// Mode k of field i at time t+1 is sum_j Lambda_ij(k) x_j(k), Lambda_ij the symbol
// of stencil (i, j) (appendix on vector-valued fields), so the T-step map is the
// matrix power Lambda(k)^T, taken by binary repeated squaring of the matrix.  As
// in the scalar path the power starts in deviation form: D = I - Lambda,
// squaring I - D gives I - (2D - D^2) and (I - V)(I - D) = I - (V + D - V D); every
// matrix involved is a polynomial in Lambda, so the products commute.  The
// deviation entries come from the per-axis phase tables E(m) = exp(2 pi i m / n) - 1
// (a cell offset o contributes prod_a (1 + E_a) - 1, built axis by axis), so modes
// near Lambda = I keep their relative accuracy; a running square or product leaves
// the deviation form once its deviation is far from 0 (largest row sum above 1/2),
// so modes that decay keep theirs too.  One thread per mode, FP64 throughout;
// spectra are read and written in the solve's precision.
#include <hip/hip_runtime.h>

#include "sfft_device.h"
#include "sfft_fields.h"

namespace sfft {

namespace {

template <int M>
__device__ __forceinline__ void matmul(const dcx (&a)[M][M], const dcx (&b)[M][M], dcx (&c)[M][M]) {
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) {
            dcx s = dmul(a[i][0], b[0][j]);
#pragma unroll
            for (int k = 1; k < M; ++k) s = dadd(s, dmul(a[i][k], b[k][j]));
            c[i][j] = s;
        }
}

template <int M>
__device__ __forceinline__ void matmul_real(const double (&a)[M][M], const double (&b)[M][M], double (&c)[M][M]) {
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double s = a[i][0] * b[0][j];
#pragma unroll
            for (int k = 1; k < M; ++k) s = fma(a[i][k], b[k][j], s);
            c[i][j] = s;
        }
}

// Element operations shared by the real and the complex matrix power.
__device__ __forceinline__ double e_add(double a, double b) { return a + b; }
__device__ __forceinline__ dcx e_add(dcx a, dcx b) { return dadd(a, b); }
__device__ __forceinline__ double e_sub(double a, double b) { return a - b; }
__device__ __forceinline__ dcx e_sub(dcx a, dcx b) { return dsub(a, b); }
__device__ __forceinline__ double e_abs(double a) { return fabs(a); }
__device__ __forceinline__ double e_abs(dcx a) { return fabs(a.x) + fabs(a.y); }
__device__ __forceinline__ void e_set(double& a, double v) { a = v; }
__device__ __forceinline__ void e_set(dcx& a, double v) { a = dcx{v, 0.0}; }
template <int M>
__device__ __forceinline__ void mm(const double (&a)[M][M], const double (&b)[M][M], double (&c)[M][M]) { matmul_real<M>(a, b, c); }
template <int M>
__device__ __forceinline__ void mm(const dcx (&a)[M][M], const dcx (&b)[M][M], dcx (&c)[M][M]) { matmul<M>(a, b, c); }

// Largest row sum of |entries| (|re| + |im| for complex entries): a bound on the
// deviation's size that decides when to leave the deviation form.
template <int M, typename E>
__device__ __forceinline__ double row_norm(const E (&a)[M][M]) {
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) s += e_abs(a[i][j]);
        m = fmax(m, s);
    }
    return m;
}

// a <- I - a
template <int M, typename E>
__device__ __forceinline__ void one_minus(E (&a)[M][M]) {
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) {
            E id;
            e_set(id, i == j ? 1.0 : 0.0);
            a[i][j] = e_sub(id, a[i][j]);
        }
}

// P = (I - D)^T by binary repeated squaring (Sec. 3 Step 2 on the symbol
// matrix).  The running square and the product are kept as deviations from I
// while both are close to I (2D - D^2 and V + D - V D) and as plain matrices
// from the point where a deviation's row sum exceeds 1/2.  D is overwritten.
template <int M, typename E>
__device__ __forceinline__ void mat_power(E (&D)[M][M], E (&P)[M][M], int64_t T) {
    E V[M][M], Q[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) e_set(V[i][j], 0.0);
    bool sd = true, vd = true;
    if (row_norm<M>(D) > 0.5) { one_minus<M>(D); sd = false; }
    for (int64_t Rb = T; Rb > 0; Rb >>= 1) {
        if (Rb & 1) {
            if (vd && sd) {
                mm(V, D, Q);
#pragma unroll
                for (int i = 0; i < M; ++i)
#pragma unroll
                    for (int j = 0; j < M; ++j) V[i][j] = e_sub(e_add(V[i][j], D[i][j]), Q[i][j]);
            } else {
                if (vd) one_minus<M>(V);
                if (sd) one_minus<M>(D);
                mm(V, D, Q);
                if (sd) one_minus<M>(D);
#pragma unroll
                for (int i = 0; i < M; ++i)
#pragma unroll
                    for (int j = 0; j < M; ++j) V[i][j] = Q[i][j];
                vd = false;
            }
        }
        if (Rb > 1) {
            mm(D, D, Q);
            if (sd) {
#pragma unroll
                for (int i = 0; i < M; ++i)
#pragma unroll
                    for (int j = 0; j < M; ++j) D[i][j] = e_sub(e_add(D[i][j], D[i][j]), Q[i][j]);
                if (row_norm<M>(D) > 0.5) { one_minus<M>(D); sd = false; }
            } else {
#pragma unroll
                for (int i = 0; i < M; ++i)
#pragma unroll
                    for (int j = 0; j < M; ++j) D[i][j] = Q[i][j];
            }
        }
    }
    if (vd) one_minus<M>(V);
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) P[i][j] = V[i][j];
}


// E(o f) of one axis from its E(f), E(2f): zero for o = 0, conjugate for o < 0.
__device__ __forceinline__ dcx phase(const dcx (&Ea)[kMaxR + 1], int o) {
    dcx e = (o == 1 || o == -1) ? Ea[1] : Ea[kMaxR];
    if (o == 0) e = dcx{0.0, 0.0};
    if (o < 0) e.y = -e.y;  // E(-m) = conj E(m)
    return e;
}

// fn(q, dev) for the offsets of the (2r+1)^d box (DIM = d), q row-major over
// o_0..o_{d-1}, dev = prod_a (1 + E_a(o_a f_a)) - 1 built axis by axis.  HALF:
// only the offsets after the centre in that order (one of every pair o, -o), for
// point-symmetric blocks.
template <int DIM, bool HALF, typename F>
__device__ __forceinline__ void for_each_offset(const SymParams& sp, const dcx (&E)[3][kMaxR + 1], F&& fn) {
    const int r = sp.r, w = 2 * r + 1;
    const int r1 = DIM >= 2 ? r : 0, r2 = DIM >= 3 ? r : 0;
    for (int o0 = HALF ? 0 : -r; o0 <= r; ++o0) {
        const dcx e0 = phase(E[0], o0);
        for (int o1 = (HALF && o0 == 0) ? 0 : -r1; o1 <= r1; ++o1) {
            const dcx e1 = phase(E[1], o1);
            const dcx d01 = DIM >= 2 ? dadd(dadd(e0, e1), dmul(e0, e1)) : e0;
            const int q01 = DIM >= 2 ? (o0 + r) * w + (o1 + r) : o0 + r;
            for (int o2 = (HALF && o0 == 0 && o1 == 0) ? (DIM >= 3 ? 1 : 0) : -r2; o2 <= r2; ++o2) {
                if (HALF && DIM < 3 && o0 == 0 && o1 == 0) continue;  // the centre
                if (DIM >= 3) {
                    const dcx e2 = phase(E[2], o2);
                    fn(q01 * w + (o2 + r), dadd(dadd(d01, e2), dmul(d01, e2)));
                } else {
                    fn(q01, d01);
                }
            }
        }
    }
}

// A workgroup covers 256 consecutive entries of one spectrum row, so the row's
// position (and its frequencies on axes 0..d-2) is the same for the whole group.
template <typename R, int M, int DIM>
__global__ __launch_bounds__(256) void k_fields_symbol(FieldParams fp, SymParams sp) {
    const uint32_t cpr = (uint32_t)((sp.hcount + 255) / 256);  // workgroups per row
    const uint32_t row = blockIdx.x / cpr;
    const uint32_t kl = (blockIdx.x - row * cpr) * 256 + threadIdx.x;
    if (kl >= (uint32_t)sp.hcount) return;  // past the half spectrum
    const int64_t idx = (int64_t)row * fp.pitch + kl;

    // frequency of this position along every axis (stored order -> frequency)
    uint32_t f[3] = {0, 0, 0};
    {
        uint32_t rem = row;
#pragma unroll
        for (int a = 1; a >= 0; --a) {
            if (a <= sp.d - 2) {
                const uint32_t sd = (uint32_t)sp.sdim[a];
                const uint32_t q = rem / sd;
                f[a] = pos_to_freq32(sp, a, rem - q * sd);
                rem = q;
            }
        }
    }
    const int last = sp.d - 1;
    const uint32_t fl = fp.full ? pos_to_freq32(sp, last, kl) : kl;
    if (last == 0) f[0] = fl;
    else if (last == 1) f[1] = fl;
    else f[2] = fl;

    // E_a(o f_a) for o = 1..r on every axis
    dcx E[3][kMaxR + 1];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 0; o <= kMaxR; ++o) {
            E[a][o] = dcx{0.0, 0.0};
            if (a < sp.d && o >= 1 && o <= sp.r)
                E[a][o] = ((const dcx*)sp.eph[a])[mul_mod_small((uint32_t)o, f[a], (uint32_t)sp.n[a])];
        }

    const double* cc = fp.cK + M * M;
    cx<R>* ws = (cx<R>*)fp.ws;
    dcx x[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const cx<R> v = ws[j * fp.fstride + idx];
        x[j] = dcx{(double)v.x, (double)v.y};
    }

    if (M == 1 && fp.implicit) {
        // lambda_R = lambda_S / lambda_Q, or 0 where lambda_Q vanishes; in deviation
        // form mu_R = 1 - lambda_R = (mu_S - mu_Q) / (1 - mu_Q)
        dcx muS = {cc[-1], 0.0}, muQ = {fp.qK[0], 0.0};
        const double* qc = fp.qK + 1;
        for_each_offset<DIM, false>(sp, E, [&](int q, dcx dev) {
            muS.x = fma(-cc[q], dev.x, muS.x);
            muS.y = fma(-cc[q], dev.y, muS.y);
            muQ.x = fma(-qc[q], dev.x, muQ.x);
            muQ.y = fma(-qc[q], dev.y, muQ.y);
        });
        const dcx lq = {1.0 - muQ.x, -muQ.y};
        const double lq2 = lq.x * lq.x + lq.y * lq.y;
        dcx D = {1.0, 0.0};
        if (lq2 > fp.qzero * fp.qzero) {
            const dcx num = dsub(muS, muQ);
            D = dcx{(num.x * lq.x + num.y * lq.y) / lq2, (num.y * lq.x - num.x * lq.y) / lq2};
        }
        const dcx y = dmul(power_complex(D, sp.T), x[0]);
        ws[idx] = cx<R>{R(y.x * sp.scale), R(y.y * sp.scale)};
        return;
    }

    if (fp.real_sym) {
        // Point-symmetric blocks: the imaginary parts of offsets o and -o cancel,
        // the symbol matrix is real and so are its powers.
        double D[M][M], P[M][M];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) D[i][j] = fp.cK[i * M + j];
        // offsets o and -o share Re(dev) and their coefficient
        for_each_offset<DIM, true>(sp, E, [&](int q, dcx dev) {
            const double d2 = 2.0 * dev.x;
#pragma unroll
            for (int i = 0; i < M; ++i)
#pragma unroll
                for (int j = 0; j < M; ++j) D[i][j] = fma(-cc[(i * M + j) * fp.nof + q], d2, D[i][j]);
        });
        mat_power<M>(D, P, sp.T);
        // y = Lambda^T x * scale
#pragma unroll
        for (int i = 0; i < M; ++i) {
            dcx y = {0.0, 0.0};
#pragma unroll
            for (int j = 0; j < M; ++j) {
                y.x = fma(P[i][j], x[j].x, y.x);
                y.y = fma(P[i][j], x[j].y, y.y);
            }
            ws[i * fp.fstride + idx] = cx<R>{R(y.x * sp.scale), R(y.y * sp.scale)};
        }
        return;
    }

    // D = K - sum_o c_o * dev_o
    dcx D[M][M], P[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) D[i][j] = dcx{fp.cK[i * M + j], 0.0};
    for_each_offset<DIM, false>(sp, E, [&](int q, dcx dev) {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double c = cc[(i * M + j) * fp.nof + q];
                D[i][j].x = fma(-c, dev.x, D[i][j].x);
                D[i][j].y = fma(-c, dev.y, D[i][j].y);
            }
    });
    // P = Lambda^T by repeated squaring of I - D
    mat_power<M>(D, P, sp.T);
    // y = Lambda^T x * scale
#pragma unroll
    for (int i = 0; i < M; ++i) {
        dcx y = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < M; ++j) y = dadd(y, dmul(P[i][j], x[j]));
        ws[i * fp.fstride + idx] = cx<R>{R(y.x * sp.scale), R(y.y * sp.scale)};
    }
}

template <typename R>
hipError_t launch_m(const FieldParams& fp, const SymParams& sp, hipStream_t st) {
    const int64_t cpr = (sp.hcount + 255) / 256;
    if (fp.rows * cpr > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)(fp.rows * cpr)), b(256);
#define SFFT_FIELDS_M(MM)                                                                       \
    switch (sp.d) {                                                                              \
        case 1: hipLaunchKernelGGL((k_fields_symbol<R, MM, 1>), g, b, 0, st, fp, sp); break;      \
        case 2: hipLaunchKernelGGL((k_fields_symbol<R, MM, 2>), g, b, 0, st, fp, sp); break;      \
        case 3: hipLaunchKernelGGL((k_fields_symbol<R, MM, 3>), g, b, 0, st, fp, sp); break;      \
        default: return hipErrorInvalidValue;                                                    \
    }
    switch (fp.m) {
        case 1: SFFT_FIELDS_M(1) break;
        case 2: SFFT_FIELDS_M(2) break;
        case 3: SFFT_FIELDS_M(3) break;
        case 4: SFFT_FIELDS_M(4) break;
        default: return hipErrorInvalidValue;
    }
#undef SFFT_FIELDS_M
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fields_symbol(const FieldParams& fp, const SymParams& sp, bool f64, hipStream_t st) {
    return f64 ? launch_m<double>(fp, sp, st) : launch_m<float>(fp, sp, st);
}

}  // namespace sfft
