// HIP kernels of the FFT stencil solver (gfx950).
//
//  k_row  : transforms along the contiguous axis, whole rows staged in LDS.
//           Forward real-to-complex (first pass), inverse complex-to-real (last
//           pass), complex-to-complex (middle of a split 1-D problem), or the
//           whole periodic solve of a 1-D row in one launch.
//  k_col  : transforms along a strided axis on a tile of W adjacent columns,
//           forward / inverse with the twiddle of a split axis, or the fused
//           middle pass: forward transform, multiply by lambda^T / N (FP64 symbol
//           and repeated squaring), inverse transform.
//  table kernels: FP64 twiddles exp(-2 pi i m / N) and symbol phases
//           exp(2 pi i m / n) - 1 from sincospi with exact integer reduction.
//  k_symbol_power: lambda(k)^T in natural order (inspection entry point).
#include <hip/hip_runtime.h>

#include "sfft_device.h"
#include "sfft_fast.h"
#include "sfft_kernels.h"
#include "sfft_mixed.h"

namespace sfft {

__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

// (b, i_0 .. i_{d-2}) of row `row` of a row pass; rows are ordered [B][n_0]..[n_{d-2}].
// (Unrolled over the at most two leading axes with selects: a run-time index into
// the small array would place it in scratch memory.)
__device__ __forceinline__ int64_t row_coords(const PassDesc& pd, int64_t row, int64_t* i) {
    int64_t rem = row;
#pragma unroll
    for (int a = 1; a >= 0; --a) {
        if (a <= pd.d - 2) {
            const int64_t n = a == 1 ? pd.rdims[1] : pd.rdims[0];
            const int64_t q = rem / n;
            i[a] = rem - q * n;
            rem = q;
        }
    }
    return rem;
}

__device__ __forceinline__ bool prefix_inside(const RealView& v, int d, const int64_t* i) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
        if (a < d - 1 && i[a] >= v.ext[a]) return false;
    return true;
}

__device__ __forceinline__ int64_t prefix_offset(const RealView& v, int d, int64_t b, const int64_t* i) {
    int64_t off = b * v.boff;
#pragma unroll
    for (int a = 0; a < 2; ++a)
        if (a < d - 1) off += i[a] * v.stride[a];
    return off;
}

// ---------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------
template <typename R>
__device__ void r2c_untangle(cx<R>* lds, int nrows, int LS, int L, const cx<R>* tab) {
    // X[k] = (Z[k] + conj Z[L-k]) / 2 - i w^k (Z[k] - conj Z[L-k]) / 2, w = exp(-2 pi i / 2L)
    // tab holds exp(-2 pi i m / 2L).
    const int per = L / 2 + 1;
    const UDiv dper = udiv((uint32_t)per);
    for (int e = threadIdx.x; e < nrows * per; e += gen_threads<R>()) {
        uint32_t rr;
        const int k = (int)udiv_qr((uint32_t)e, dper, &rr);
        cx<R>* row = lds + rr * LS;
        const int kk = k == 0 ? 0 : L - k;
        const cx<R> zk = row[k], zm = row[kk];
        if (k == 0) {
            row[0] = cx<R>{zk.x + zk.y, R(0)};
            row[L] = cx<R>{zk.x - zk.y, R(0)};
            continue;
        }
        {
            const cx<R> e = scale(zk + conj(zm), R(0.5));
            const cx<R> o = scale(zk - conj(zm), R(0.5));
            const cx<R> w = tab[k];
            const cx<R> t = cmul(w, o);
            row[k] = cx<R>{e.x + t.y, e.y - t.x};  // e - i t
        }
        if (kk != k) {
            const cx<R> e = scale(zm + conj(zk), R(0.5));
            const cx<R> o = scale(zm - conj(zk), R(0.5));
            const cx<R> w = tab[kk];
            const cx<R> t = cmul(w, o);
            row[kk] = cx<R>{e.x + t.y, e.y - t.x};
        }
    }
}

template <typename R>
__device__ void c2r_tangle(cx<R>* lds, int nrows, int LS, int L, const cx<R>* tab) {
    // Z'[k] = (X[k] + conj X[L-k]) + i conj(w^k) (X[k] - conj X[L-k]), w as above.
    const int per = L / 2 + 1;
    const UDiv dper = udiv((uint32_t)per);
    for (int e = threadIdx.x; e < nrows * per; e += gen_threads<R>()) {
        uint32_t rr;
        const int k = (int)udiv_qr((uint32_t)e, dper, &rr);
        cx<R>* row = lds + rr * LS;
        const int kk = L - k;
        const cx<R> xk = row[k], xm = row[kk];
        {
            const cx<R> e = xk + conj(xm);
            const cx<R> o = cmulc(xk - conj(xm), tab[k]);
            row[k] = cx<R>{e.x - o.y, e.y + o.x};  // e + i o
        }
        if (k != 0 && kk != k) {
            const cx<R> e = xm + conj(xk);
            const cx<R> o = cmulc(xm - conj(xk), tab[kk]);
            row[kk] = cx<R>{e.x - o.y, e.y + o.x};
        }
    }
}

template <typename R>
__device__ __forceinline__ void row_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    const int L = pd.L;
    const int LS = pd.lds_stride;
    const int64_t row0 = (int64_t)bid * pd.W;
    const int nrows = (int)imin64(pd.W, pd.outer - row0);
    const cx<R>* buf = (const cx<R>*)pd.buf;
    const R* rin = (const R*)pd.rv.ptr;
    const cx<R>* htab = (const cx<R>*)pd.st_tab;  // exp(-2 pi i m / (L * st_mul))

    // Real views: each row's base offset (-1: outside the view) once per row when
    // the tile has few rows, instead of 64-bit divisions per element.
    constexpr int kRowCache = 64;
    __shared__ int64_t base_in[kRowCache], base_out[kRowCache];
    const bool cached = nrows <= kRowCache && (pd.in_real || pd.out_real);
    if (cached) {
        for (int rr = threadIdx.x; rr < nrows; rr += gen_threads<R>()) {
            int64_t idx[3];
            const int64_t b = row_coords(pd, row0 + rr, idx);
            if (pd.in_real) base_in[rr] = prefix_inside(pd.rv, pd.d, idx) ? prefix_offset(pd.rv, pd.d, b, idx) : -1;
            if (pd.out_real) base_out[rr] = prefix_inside(pd.rvo, pd.d, idx) ? prefix_offset(pd.rvo, pd.d, b, idx) : -1;
        }
        __syncthreads();
    }

    // ---- load
    if (pd.in_real) {
        const int64_t sl = pd.rv.stride[pd.d - 1];
        const int64_t el = pd.rv.ext[pd.d - 1];
        const UDiv dl = udiv((uint32_t)L);
        for (int e = threadIdx.x; e < nrows * L; e += gen_threads<R>()) {
            uint32_t rr;
            const int m = (int)udiv_qr((uint32_t)e, dl, &rr);
            int64_t base;
            if (cached) {
                base = base_in[rr];
            } else {
                int64_t idx[3];
                const int64_t b = row_coords(pd, row0 + rr, idx);
                base = prefix_inside(pd.rv, pd.d, idx) ? prefix_offset(pd.rv, pd.d, b, idx) : -1;
            }
            cx<R> v = {R(0), R(0)};
            if (base >= 0) {
                if (pd.rowtrans == RT_HALF) {
                    if (2 * m < el) v.x = rin[base + (int64_t)(2 * m) * sl];
                    if (2 * m + 1 < el) v.y = rin[base + (int64_t)(2 * m + 1) * sl];
                } else {
                    if (m < el) v.x = rin[base + (int64_t)m * sl];
                }
            }
            lds[rr * LS + m] = v;
        }
    } else {
        const int cnt = pd.rowtrans == RT_HALF ? L + 1 : L;
        const UDiv dc = udiv((uint32_t)cnt);
        for (int e = threadIdx.x; e < nrows * cnt; e += gen_threads<R>()) {
            uint32_t rr;
            const int m = (int)udiv_qr((uint32_t)e, dc, &rr);
            const cx<R>* src = buf + (row0 + rr) * pd.ostride;
            cx<R> v;
            if (pd.rowtrans == RT_ODD && m >= pd.hcount) v = conj(src[L - m]);
            else v = src[m];
            lds[rr * LS + m] = v;
        }
    }
    __syncthreads();

    const bool half = pd.rowtrans == RT_HALF;
    if (pd.mode == MODE_INV && half) {
        c2r_tangle<R>(lds, nrows, LS, L, htab);
        __syncthreads();
    }
    if (pd.mode != MODE_INV) {
        tile_fft<R, false, false>(lds, pd, nrows, LS, 1);
        if (half) {
            r2c_untangle<R>(lds, nrows, LS, L, htab);
            __syncthreads();
        }
    }
    if (pd.mode == MODE_MID) {
        // 1-D problems: axis 0 is the only axis, G[o] = c[o], K = 1 - sum c.
        const SymCol col = symbol_column_1d(sp);
        const int cnt = half ? L + 1 : L;
        const UDiv dc = udiv((uint32_t)cnt);
        for (int e = threadIdx.x; e < nrows * cnt; e += gen_threads<R>()) {
            uint32_t rr;
            const int k = (int)udiv_qr((uint32_t)e, dc, &rr);
            const int64_t p0 = ((row0 + rr) % pd.q_mod) * L + k;
            const int64_t f0 = pos_to_freq(sp, 0, p0);
            dcx v;
            symbol_power_n<1>(sp, col, &f0, &v);
            cx<R>& x = lds[rr * LS + k];
            x = cmul(x, cx<R>{R(v.x), R(v.y)});
        }
        __syncthreads();
        if (half) {
            c2r_tangle<R>(lds, nrows, LS, L, htab);
            __syncthreads();
        }
    }
    if (pd.mode != MODE_FWD) tile_fft<R, true, false>(lds, pd, nrows, LS, 1);

    // ---- store
    if (pd.out_real) {
        R* rout = (R*)pd.rvo.ptr;
        const int64_t sl = pd.rvo.stride[pd.d - 1];
        const int64_t el = pd.rvo.ext[pd.d - 1];
        const int per = half ? 2 * L : L;
        const UDiv dp = udiv((uint32_t)per);
        for (int e = threadIdx.x; e < nrows * per; e += gen_threads<R>()) {
            uint32_t rr;
            const int m = (int)udiv_qr((uint32_t)e, dp, &rr);
            if (m >= el) continue;
            int64_t base;
            if (cached && !pd.keep.enabled) {
                base = base_out[rr];
                if (base < 0) continue;
            } else {
                int64_t idx[3];
                const int64_t b = row_coords(pd, row0 + rr, idx);
                if (!prefix_inside(pd.rvo, pd.d, idx)) continue;
                if (pd.d == 1) idx[0] = m;
                else if (pd.d == 2) idx[1] = m;
                else idx[2] = m;
                if (!keep_cell(pd.keep, pd.d, b, idx)) continue;
                base = prefix_offset(pd.rvo, pd.d, b, idx);
            }
            const cx<R> z = lds[rr * LS + (half ? (m >> 1) : m)];
            rout[base + (int64_t)m * sl] = half ? ((m & 1) ? z.y : z.x) : z.x;
        }
    } else {
        cx<R>* dst = (cx<R>*)pd.buf;
        const int cnt = pd.rowtrans == RT_C2C ? L : pd.hcount;
        const UDiv dc = udiv((uint32_t)cnt);
        for (int e = threadIdx.x; e < nrows * cnt; e += gen_threads<R>()) {
            uint32_t rr;
            const int m = (int)udiv_qr((uint32_t)e, dc, &rr);
            dst[(row0 + rr) * pd.ostride + m] = lds[rr * LS + m];
        }
    }
}

// ---------------------------------------------------------------------------
// Column pass
// ---------------------------------------------------------------------------
// Multiply a column tile (W <= threads columns) by lambda^T * scale: tpc =
// threads / W threads share a column (the first tpc * W threads take part); each
// reads the column's part of the symbol once and takes every tpc-th row, four
// rows at a time as independent chains.
template <typename R, int RR>
__device__ __forceinline__ void symbol_cols(cx<R>* lds, const SymParams& sp, const SymCol* Cs, const int* Vs, int L,
                                            int W, int64_t qpre) {
    constexpr int G = 4;
    const int tpc = gen_threads<R>() / W;
    if ((int)threadIdx.x >= tpc * W) return;
    const int cc = threadIdx.x % W, k0 = threadIdx.x / W;
    if (!Vs[cc]) return;
    const SymCol col = Cs[cc];
    for (int k = k0; k < L; k += G * tpc) {
        uint32_t f[G];
#pragma unroll
        for (int g = 0; g < G; ++g) f[g] = pos_to_freq32(sp, 0, (uint32_t)(qpre + min(k + g * tpc, L - 1)));
        dcx v[G];
        symbol_power_g<G, RR>(sp, col, f, v);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int kg = k + g * tpc;
            if (kg >= L) continue;
            cx<R>& x = lds[kg * W + cc];
            x = cmul(x, cx<R>{R(v[g].x), R(v[g].y)});
        }
    }
}
template <typename R>
__device__ __forceinline__ void col_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    const int L = pd.L, W = pd.W;
    const int64_t tile = bid;
    const int64_t o = tile / pd.tiles_inner;
    const int64_t c0 = (tile - o * pd.tiles_inner) * W;
    const int wc = (int)imin64(W, pd.inner - c0);
    const cx<R>* buf = (const cx<R>*)pd.buf;
    // valid columns: inside inner and, when the last axis is padded, inside hcount
    auto col_valid = [&](int64_t c) -> bool {
        if (c - c0 >= wc) return false;
        if (pd.cpitch > 0 && (c % pd.cpitch) >= pd.hcount) return false;
        return true;
    };

    // Per-column validity and split-twiddle step once per tile column when the
    // tile is narrow enough, instead of 64-bit divisions per element (twj < 0:
    // column not valid).
    constexpr int kColCache = 256;
    __shared__ int64_t col_twj[kColCache];
    const bool cached = W <= kColCache;
    if (cached) {
        for (int cc = threadIdx.x; cc < W; cc += gen_threads<R>()) {
            const int64_t c = c0 + cc;
            col_twj[cc] = col_valid(c) ? (pd.tw ? c / pd.tw_div : 0) : -1;
        }
        __syncthreads();
    }
    auto column = [&](int cc, int64_t* twj) -> bool {
        if (cached) {
            *twj = col_twj[cc];
            return *twj >= 0;
        }
        const int64_t c = c0 + cc;
        if (!col_valid(c)) return false;
        *twj = pd.tw ? c / pd.tw_div : 0;
        return true;
    };

    // ---- load (inverse passes multiply by the conjugate split twiddle first)
    const UDiv dw = udiv((uint32_t)W);
    for (int e = threadIdx.x; e < L * W; e += gen_threads<R>()) {
        uint32_t k;
        const int cc = (int)udiv_qr((uint32_t)e, dw, &k);
        const int64_t c = c0 + cc;
        cx<R> v = {R(0), R(0)};
        int64_t twj;
        if (column(cc, &twj)) {
            if (pd.in_real) {
                const int64_t m = (int64_t)k * pd.kstride + c;
                if (m < pd.rv.ext[0]) v.x = ((const R*)pd.rv.ptr)[o * pd.rv.boff + m * pd.rv.stride[0]];
            } else {
                v = buf[o * pd.ostride + (int64_t)k * pd.kstride + c];
            }
            if (pd.mode == MODE_INV && pd.tw) v = cmulc(v, step_twiddle<R>(pd, (int64_t)k * twj));
        }
        lds[k * W + cc] = v;
    }
    __syncthreads();

    if (pd.mode != MODE_INV) tile_fft<R, false, true>(lds, pd, W, 1, W);

    if (pd.mode == MODE_MID) {
        __shared__ SymCol Cs[64];
        __shared__ int Vs[64];
        // per-column part of the symbol (axes 1..d-1 fixed along a column)
        for (int cc = threadIdx.x; cc < W; cc += gen_threads<R>()) {
            const int64_t c = c0 + cc;
            int valid = col_valid(c) ? 1 : 0;
            int64_t f[3] = {0, 0, 0};
            if (valid) {
                int64_t rem = c;
                for (int a = sp.d - 1; a >= 1; --a) {
                    const int64_t q = rem / sp.sdim[a];
                    const int64_t p = rem - q * sp.sdim[a];
                    rem = q;
                    f[a] = pos_to_freq(sp, a, p);
                }
            }
            Cs[cc] = symbol_column(sp, f);
            Vs[cc] = valid;
        }
        __syncthreads();
        const int64_t qpre = (o % pd.q_mod) * L;
        if (sp.r <= 0) symbol_cols<R, 0>(lds, sp, Cs, Vs, L, W, qpre);
        else if (sp.r == 1) symbol_cols<R, 1>(lds, sp, Cs, Vs, L, W, qpre);
        else symbol_cols<R, 2>(lds, sp, Cs, Vs, L, W, qpre);
        __syncthreads();
    }

    if (pd.mode != MODE_FWD) tile_fft<R, true, true>(lds, pd, W, 1, W);

    // ---- store (forward passes multiply by the split twiddle last)
    for (int e = threadIdx.x; e < L * W; e += gen_threads<R>()) {
        uint32_t k;
        const int cc = (int)udiv_qr((uint32_t)e, dw, &k);
        const int64_t c = c0 + cc;
        int64_t twj;
        if (!column(cc, &twj)) continue;
        cx<R> v = lds[k * W + cc];
        if (pd.mode == MODE_FWD && pd.tw) v = cmul(v, step_twiddle<R>(pd, (int64_t)k * twj));
        if (pd.out_real) {
            const int64_t m = (int64_t)k * pd.kstride + c;
            if (m >= pd.rvo.ext[0]) continue;
            int64_t idx[3] = {m, 0, 0};
            if (!keep_cell(pd.keep, 1, o, idx)) continue;
            ((R*)pd.rvo.ptr)[o * pd.rvo.boff + m * pd.rvo.stride[0]] = v.x;
        } else {
            ((cx<R>*)pd.buf)[o * pd.ostride + (int64_t)k * pd.kstride + c] = v;
        }
    }
}


__device__ __forceinline__ int batch_find_g(const BatchItem* it, int n, uint32_t bid) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (it[mid].first <= (int64_t)bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename R>
__global__ __launch_bounds__(gen_threads<R>()) void k_row(PassDesc pd, SymParams sp) {
    // The tile code indexes the descriptors' arrays with run-time indices; on the
    // kernel-argument copies that costs a private copy and several hundred VGPRs
    // (one wave per SIMD), on an LDS copy it is an LDS read.
    __shared__ PassDesc spd;
    __shared__ SymParams ssp;
    if (threadIdx.x == 0) {
        spd = pd;
        ssp = sp;
    }
    __syncthreads();
    row_tile<R>(spd, ssp, blockIdx.x);
}
template <typename R>
__global__ __launch_bounds__(gen_threads<R>()) void k_row_b(const BatchItem* it, int n, const SymParams* sy) {
    const int i = batch_find_g(it, n, blockIdx.x);
    row_tile<R>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
}
template <typename R>
__global__ __launch_bounds__(gen_threads<R>()) void k_col(PassDesc pd, SymParams sp) {
    __shared__ PassDesc spd;  // see k_row
    __shared__ SymParams ssp;
    if (threadIdx.x == 0) {
        spd = pd;
        ssp = sp;
    }
    __syncthreads();
    col_tile<R>(spd, ssp, blockIdx.x);
}
template <typename R>
__global__ __launch_bounds__(gen_threads<R>()) void k_col_b(const BatchItem* it, int n, const SymParams* sy) {
    const int i = batch_find_g(it, n, blockIdx.x);
    col_tile<R>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
}

// ---------------------------------------------------------------------------
// Tables
// ---------------------------------------------------------------------------
__global__ void k_twiddle_table(double2* t64, float2* t32, int64_t N, int64_t count, int64_t mult) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int64_t e = (i * mult) % N;
    if (2 * e > N) e -= N;
    double s, c;
    sincospi(2.0 * (double)e / (double)N, &s, &c);
    t64[i] = make_double2(c, -s);
    t32[i] = make_float2((float)c, (float)-s);
}

__global__ void k_phase_table(double2* E, int64_t n) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    int64_t mm = m;
    if (2 * mm > n) mm -= n;
    const double h = sinpi((double)mm / (double)n);
    const double s = sinpi(2.0 * (double)mm / (double)n);
    E[m] = make_double2(-2.0 * h * h, s);
}

// Per-column symbol parts for the middle pass: column c = position in the
// spectrum buffer over axes 1..d-1 (row-major, last axis padded).
__global__ void k_symbol_columns(SymCol* tab, SymParams sp, int64_t total) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= total) return;
    int64_t f[3] = {0, 0, 0};
    int64_t rem = c;
    for (int a = sp.d - 1; a >= 1; --a) {
        const int64_t q = rem / sp.sdim[a];
        f[a] = pos_to_freq(sp, a, rem - q * sp.sdim[a]);
        rem = q;
    }
    tab[c] = symbol_column(sp, f);
}

// lambda(k)^T in natural order over the full spectrum (row-major k).
__global__ void k_symbol_power(double2* out, SymParams sp, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int64_t f[3] = {0, 0, 0};
    int64_t rem = idx;
    for (int a = sp.d - 1; a >= 0; --a) {
        const int64_t q = rem / sp.n[a];
        f[a] = rem - q * sp.n[a];
        rem = q;
    }
    const SymCol col = symbol_column(sp, f);
    const dcx v = symbol_power_at(sp, col, f[0]);
    out[idx] = make_double2(v.x, v.y);
}

// ---------------------------------------------------------------------------
// Host-side launch helpers
// ---------------------------------------------------------------------------
template <typename R>
static hipError_t launch_pass_t(const PassDesc& pd, const SymParams& sp, size_t lds, hipStream_t st) {
    if (pd.kind == PASS_ROW)
        hipLaunchKernelGGL(k_row<R>, dim3((unsigned)pd.ntiles), dim3(gen_threads<R>()), lds, st, pd, sp);
    else
        hipLaunchKernelGGL(k_col<R>, dim3((unsigned)pd.ntiles), dim3(gen_threads<R>()), lds, st, pd, sp);
    return hipGetLastError();
}

hipError_t launch_pass(const PassDesc& pd, const SymParams& sp, bool f64, size_t lds, hipStream_t st) {
    if (pd.mq) return launch_mixed_pass(pd, sp, f64, lds, st);
    if (pd.fast) return launch_fast_pass(pd, sp, f64, lds, st);
    return f64 ? launch_pass_t<double>(pd, sp, lds, st) : launch_pass_t<float>(pd, sp, lds, st);
}

hipError_t launch_pass_batch(const PassDesc& proto, const BatchItem* items, int n, const SymParams* syms,
                             int64_t tiles, bool f64, size_t lds, hipStream_t st) {
    if (proto.mq) return launch_mixed_batch(proto, items, n, syms, tiles, f64, lds, st);
    if (proto.fast) return launch_fast_batch(proto, items, n, syms, tiles, f64, lds, st);
    const dim3 g((unsigned)tiles), b(f64 ? gen_threads<double>() : gen_threads<float>());
    if (proto.kind == PASS_ROW) {
        if (f64) hipLaunchKernelGGL(k_row_b<double>, g, b, lds, st, items, n, syms);
        else hipLaunchKernelGGL(k_row_b<float>, g, b, lds, st, items, n, syms);
    } else {
        if (f64) hipLaunchKernelGGL(k_col_b<double>, g, b, lds, st, items, n, syms);
        else hipLaunchKernelGGL(k_col_b<float>, g, b, lds, st, items, n, syms);
    }
    return hipGetLastError();
}

hipError_t set_kernel_lds_limits(size_t bytes) {
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_row<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_row<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_col<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_col<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_row_b<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_row_b<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_col_b<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_col_b<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    return hipSuccess;
}

hipError_t launch_twiddle_table(double2* t64, float2* t32, int64_t N, int64_t count, int64_t mult, hipStream_t st) {
    const int bs = 256;
    hipLaunchKernelGGL(k_twiddle_table, dim3((unsigned)((count + bs - 1) / bs)), dim3(bs), 0, st, t64, t32, N, count, mult);
    return hipGetLastError();
}

hipError_t launch_phase_table(double2* E, int64_t n, hipStream_t st) {
    const int bs = 256;
    hipLaunchKernelGGL(k_phase_table, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, E, n);
    return hipGetLastError();
}

size_t symbol_column_bytes() { return sizeof(SymCol); }

hipError_t launch_symbol_columns(void* tab, const SymParams& sp, int64_t total, hipStream_t st) {
    const int bs = 64;
    hipLaunchKernelGGL(k_symbol_columns, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, (SymCol*)tab, sp,
                       total);
    return hipGetLastError();
}

hipError_t launch_symbol_power(double2* out, const SymParams& sp, int64_t total, hipStream_t st) {
    const int bs = 256;
    hipLaunchKernelGGL(k_symbol_power, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, out, sp, total);
    return hipGetLastError();
}

}  // namespace sfft
