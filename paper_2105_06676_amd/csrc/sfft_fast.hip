// Power-of-two FFT passes with register radix-16 stages (gfx950).
//
// A transform of length L = 16^a * {1,2,4,8} (16 <= L <= 4096) is done by
// P = L/16 threads that each hold 16 points: thread q holds x[q + P i],
// i = 0..15, on entry and on exit (natural order).  The first Stockham stage is
// a radix-16 butterfly on those registers; every further stage exchanges the
// points through LDS once (written at their self-sorting positions, read back as
// the next stage's butterfly inputs), applies the stage twiddles from a
// two-level table and runs radix 16, 8, 4 or 2.  A 4096-point transform thus
// touches LDS twice.  Rows (contiguous axis) put 4096/L transforms in a
// 256-thread workgroup; columns put 4096/L adjacent columns in one workgroup so
// that every global access of a wave is a contiguous run across columns.
//
// Kernels:
//  k_frow<R, ROW_R2C>   first pass: real rows -> half spectrum (n/2 + 1 entries)
//  k_frow<R, ROW_C2R>   last pass: half spectrum -> real rows (keep rule applied)
//  k_frow<R, ROW_MIDR>  whole 1-D periodic solve of real rows in one launch
//  k_frow<R, ROW_MIDC>  complex row middle pass of a split 1-D axis
//  k_frow<R, ROW_CFWD>, k_frow<R, ROW_CINV>  plain complex forward / inverse rows
//  k_fcol<R, MODE>      strided-axis forward / inverse / fused middle pass
#include <hip/hip_runtime.h>

#include "sfft_device.h"
#include "sfft_fast.h"
#include "sfft_symapply.h"

namespace sfft {

namespace {

// ---------------------------------------------------------------------------
// 16-point DFT in registers: n = n1 + 4 n2, k = 4 k1 + k2.
// ---------------------------------------------------------------------------
template <typename R, bool INV>
__device__ __forceinline__ void dft16(cx<R>* v) {
    constexpr R c1 = R(0.9238795325112867), s1 = R(0.3826834323650898), h = R(0.7071067811865476);
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) dft4<R, INV>(v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]);
    // Y[n1][k2] sits at v[n1 + 4 k2]; multiply by exp(-+2 pi i n1 k2 / 16)
    auto tw = [](cx<R> a, R c, R s) -> cx<R> {  // a * (c - i s) forward, a * (c + i s) inverse
        return INV ? cx<R>{a.x * c - a.y * s, a.y * c + a.x * s} : cx<R>{a.x * c + a.y * s, a.y * c - a.x * s};
    };
    v[1 + 4] = tw(v[1 + 4], c1, s1);
    v[1 + 8] = tw(v[1 + 8], h, h);
    v[1 + 12] = tw(v[1 + 12], s1, c1);
    v[2 + 4] = tw(v[2 + 4], h, h);
    v[2 + 8] = rot90<R, INV>(v[2 + 8]);
    v[2 + 12] = tw(v[2 + 12], -h, h);
    v[3 + 4] = tw(v[3 + 4], s1, c1);
    v[3 + 8] = tw(v[3 + 8], -h, h);
    v[3 + 12] = tw(v[3 + 12], -c1, -s1);
    // DFT-4 over n1 for each k2; X[4 k1 + k2]
    cx<R> o[16];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        cx<R> a = v[4 * k2], b = v[1 + 4 * k2], c = v[2 + 4 * k2], d = v[3 + 4 * k2];
        dft4<R, INV>(a, b, c, d);
        o[k2] = a;
        o[4 + k2] = b;
        o[8 + k2] = c;
        o[12 + k2] = d;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft_r(cx<R>* v) {
    if constexpr (RAD == 16) dft16<R, INV>(v);
    else if constexpr (RAD == 8) dft8<R, INV>(v);
    else if constexpr (RAD == 4) dft4<R, INV>(v[0], v[1], v[2], v[3]);
    else dft2<R, INV>(v);
}

// exp(-2 pi i m / L) from the two-level table (lo: m mod 64, hi: m div 64)
template <typename R>
__device__ __forceinline__ cx<R> tw2(const cx<R>* lo, const cx<R>* hi, int m) {
    const cx<R> a = lo[m & 63];
    const int q = m >> 6;
    return q ? cmul(a, hi[q]) : a;
}

// LDS addressing: rows pad one point per 16, columns interleave W columns.
struct RowIdx {
    int base;
    __device__ __forceinline__ int operator()(int e) const { return base + e + (e >> 4); }
};
struct ColIdx {
    int c, ws;
    __device__ __forceinline__ int operator()(int e) const { return e * ws + c; }
};

// One Stockham stage on the thread's 16 points (all sizes compile-time).  Not
// the first stage: read the butterfly inputs from LDS and twiddle them.  Not the
// last stage: write the outputs back to LDS at their self-sorting positions.
template <typename R, int RAD, bool INV, int L, int NS, bool FIRST, bool LAST, typename IDX>
__device__ __forceinline__ void fstage(cx<R>* v, cx<R>* lds, IDX idx, int q, const cx<R>* tlo,
                                       const cx<R>* thi) {
    constexpr int P = L / 16;
    constexpr int NB = 16 / RAD;
    constexpr int SPAN = L / RAD;
    if (!FIRST) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = q + P * b;
#pragma unroll
            for (int t = 0; t < RAD; ++t) v[b * RAD + t] = lds[idx(j + t * SPAN)];
            const int k = j & (NS - 1);
            const cx<R> w1 = tw2<R>(tlo, thi, k * (L / (NS * RAD)));
            cx<R> w[RAD];
            w[1] = w1;
#pragma unroll
            for (int t = 2; t < RAD; ++t) w[t] = (t & 1) ? cmul(w[t - 1], w1) : cmul(w[t / 2], w[t / 2]);
#pragma unroll
            for (int t = 1; t < RAD; ++t) v[b * RAD + t] = INV ? cmulc(v[b * RAD + t], w[t]) : cmul(v[b * RAD + t], w[t]);
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) dft_r<R, RAD, INV>(v + b * RAD);
    if (!LAST) {
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = q + P * b;
            const int k = j & (NS - 1);
            const int d = (j - k) * RAD + k;
#pragma unroll
            for (int t = 0; t < RAD; ++t) lds[idx(d + t * NS)] = v[b * RAD + t];
        }
        __syncthreads();
    } else if (NB > 1) {
        // outputs y[q + P (b + t NB)] -> natural register order
        cx<R> o[16];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int t = 0; t < RAD; ++t) o[b + t * NB] = v[b * RAD + t];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = o[i];
    }
}

// Length-2^LOGL transform of the 16 points held by each of the L/16 threads;
// DONE = log2 of the radices already applied.
template <typename R, bool INV, int LOGL, int DONE = 0, typename IDX>
__device__ __forceinline__ void fast_fft(cx<R>* v, cx<R>* lds, IDX idx, int q, const cx<R>* tlo,
                                         const cx<R>* thi) {
    constexpr int REM = LOGL - DONE;
    if constexpr (REM > 0) {
        // the first stage is always radix 16 (the thread's 16 points); five bits
        // left after it go as radix 8 then 4, since a final radix-2 stage costs
        // more registers than it saves
        constexpr int LR = (DONE > 0 && REM == 5) ? 3 : (REM >= 4 ? 4 : REM);
        fstage<R, (1 << LR), INV, (1 << LOGL), (1 << DONE), DONE == 0, REM == LR>(v, lds, idx, q, tlo, thi);
        fast_fft<R, INV, LOGL, DONE + LR>(v, lds, idx, q, tlo, thi);
    }
}

// Row r of a row pass -> (batch b, i_0 .. i_{d-2}); returns b.
__device__ __forceinline__ int64_t row_split(const PassDesc& pd, int64_t row, int64_t* i) {
    int64_t rem = row;
#pragma unroll
    for (int a = 1; a >= 0; --a) {
        if (a <= pd.d - 2) {
            const int64_t qq = rem / pd.rdims[a];
            i[a] = rem - qq * pd.rdims[a];
            rem = qq;
        }
    }
    return rem;
}

// Base offset of a row in a real view, or -1 when the row lies outside its extents.
__device__ __forceinline__ int64_t row_base(const RealView& v, int d, int64_t b, const int64_t* i) {
    int64_t off = b * v.boff;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (a < d - 1) {
            if (i[a] >= v.ext[a]) return -1;
            off += i[a] * v.stride[a];
        }
    }
    return off;
}


}  // namespace

// ---------------------------------------------------------------------------
// Row passes
// ---------------------------------------------------------------------------
template <typename R, int KIND, int LOGL>
__device__ __forceinline__ void frow_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    constexpr int L = 1 << LOGL;
    constexpr int P = L / 16;
    constexpr int NTR = kThreads / P;
    constexpr int LS = L + L / 16 + 2;
    const int rr = threadIdx.x / P;
    const int q = threadIdx.x % P;
    const int64_t row = (int64_t)bid * NTR + rr;
    bool active = row < pd.outer;
    const RowIdx idx{rr * LS};
    const cx<R>* tlo = (const cx<R>*)pd.f_lo;
    const cx<R>* thi = (const cx<R>*)pd.f_hi;
    const cx<R>* hlo = (const cx<R>*)pd.h_lo;  // exp(-2 pi i m / 2L)
    const cx<R>* hhi = (const cx<R>*)pd.h_hi;
    cx<R> v[16];

    int64_t ii[3] = {0, 0, 0};
    const int64_t b = active ? row_split(pd, row, ii) : 0;
    // last pass under a keep rule: a row none of whose cells is kept is neither
    // read nor written (it still takes part in the tile's barriers)
    if (KIND == ROW_C2R && active && pd.keep.enabled && !row_may_keep(pd.keep, keep_row(pd.keep, pd.d, b, ii), pd.d, b))
        active = false;

    // ---------------- load
    if (KIND == ROW_R2C || KIND == ROW_MIDR) {
        const R* src = (const R*)pd.rv.ptr;
        const int64_t base = active ? row_base(pd.rv, pd.d, b, ii) : -1;
        const int64_t sl = pick3(pd.rv.stride, pd.d - 1), el = pick3(pd.rv.ext, pd.d - 1);
        const bool vec = base >= 0 && sl == 1 && el >= 2 * L && ((((uintptr_t)(src + base)) % (2 * sizeof(R))) == 0);
        if (vec) {
            const cx<R>* s2 = (const cx<R>*)(src + base) + q;
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = s2[P * i];
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int m = q + P * i;
                cx<R> z = {R(0), R(0)};
                if (base >= 0) {
                    if (2 * m < el) z.x = src[base + (int64_t)(2 * m) * sl];
                    if (2 * m + 1 < el) z.y = src[base + (int64_t)(2 * m + 1) * sl];
                }
                v[i] = z;
            }
        }
    } else {
        const cx<R>* src = (const cx<R>*)pd.buf + (active ? row : 0) * pd.ostride + q;
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = active ? src[P * i] : cx<R>{R(0), R(0)};
    }

    cx<R> xl = {R(0), R(0)};  // X[L] of a half-spectrum row (held by q == 0)
    if (KIND == ROW_C2R) {
        // X[L] goes straight to its LDS slot, which nothing touches before the
        // tangle reads it (holding it in registers across the loads made the
        // FP64 kernel spill it to scratch memory in every thread)
        if (q == 0) lds[idx(L)] = active ? ((const cx<R>*)pd.buf)[row * pd.ostride + L] : cx<R>{R(0), R(0)};
    } else if (KIND != ROW_CINV) {
        fast_fft<R, false, LOGL>(v, lds, idx, q, tlo, thi);
    }

    if (KIND == ROW_R2C || KIND == ROW_MIDR) {
        // untangle the half-length transform: X[k] from Z[k] and Z[L-k]
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[idx(q + P * i)] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = q + P * i;
            const cx<R> zk = v[i];
            if (k == 0) {
                v[i] = cx<R>{zk.x + zk.y, R(0)};
                xl = cx<R>{zk.x - zk.y, R(0)};
            } else {
                const cx<R> zm = lds[idx(L - k)];
                const cx<R> e = scale(zk + conj(zm), R(0.5));
                const cx<R> o = scale(zk - conj(zm), R(0.5));
                const cx<R> t = cmul(tw2<R>(hlo, hhi, k), o);
                v[i] = cx<R>{e.x + t.y, e.y - t.x};
            }
        }
        if (KIND == ROW_R2C) {
            if (active) {
                cx<R>* dst = (cx<R>*)pd.buf + row * pd.ostride + q;
#pragma unroll
                for (int i = 0; i < 16; ++i) dst[P * i] = v[i];
                if (q == 0) dst[L] = xl;
            }
            return;
        }
        // 1-D middle: multiply X[k], k = 0..L, by lambda^T / n
        const SymCol col = symbol_column_1d(sp);
        apply_symbol<R>(v, lds, sp, col, (uint32_t)q, (uint32_t)P);
        if (q == 0) {
            const int64_t fl = L;
            dcx s;
            symbol_power_n<1>(sp, col, &fl, &s);
            xl = cmul(xl, cx<R>{R(s.x), R(s.y)});
        }
    }

    if (KIND == ROW_C2R || KIND == ROW_MIDR) {
        // tangle for the half-length inverse:
        // Z'[k] = (X[k] + conj X[L-k]) + i conj(w^k) (X[k] - conj X[L-k]), w = exp(-2 pi i / 2L)
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[idx(q + P * i)] = v[i];
        if (KIND != ROW_C2R && q == 0) lds[idx(L)] = xl;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = q + P * i;
            const cx<R> xk = v[i], xm = lds[idx(L - k)];
            const cx<R> e = xk + conj(xm);
            const cx<R> o = cmulc(xk - conj(xm), tw2<R>(hlo, hhi, k));
            v[i] = cx<R>{e.x - o.y, e.y + o.x};
        }
        __syncthreads();
    }

    if (KIND == ROW_MIDC) {
        // position k of this row is axis-0 frequency (digit-reversed prefix) + (n0 / L) k
        const int64_t qd = active ? (row % pd.q_mod) : 0;
        const int64_t fp = pos_to_freq(sp, 0, qd * L);
        const int64_t M = sp.n[0] / L;
        const SymCol col = symbol_column_1d(sp);
        apply_symbol<R>(v, lds, sp, col, (uint32_t)(fp + M * q), (uint32_t)(M * P));
    }

    if (KIND != ROW_CFWD) fast_fft<R, true, LOGL>(v, lds, idx, q, tlo, thi);

    // ---------------- store
    if (KIND == ROW_MIDC || KIND == ROW_CFWD || KIND == ROW_CINV) {
        if (active) {
            cx<R>* dst = (cx<R>*)pd.buf + row * pd.ostride + q;
#pragma unroll
            for (int i = 0; i < 16; ++i) dst[P * i] = v[i];
        }
        return;
    }
    // real output: x[2m] = Re z[m], x[2m+1] = Im z[m]
    R* out = (R*)pd.rvo.ptr;
    const int64_t base = active ? row_base(pd.rvo, pd.d, b, ii) : -1;
    if (base < 0) return;
    const int64_t sl = pick3(pd.rvo.stride, pd.d - 1), el = pick3(pd.rvo.ext, pd.d - 1);
    const bool vec = !pd.keep.enabled && sl == 1 && el >= 2 * L &&
                     ((((uintptr_t)(out + base)) % (2 * sizeof(R))) == 0);
    if (vec) {
        cx<R>* d2 = (cx<R>*)(out + base) + q;
#pragma unroll
        for (int i = 0; i < 16; ++i) d2[P * i] = v[i];
        return;
    }
    const RowKeep rk = keep_row(pd.keep, pd.d, b, ii);
    // A slab whose face axis is not the last axis keeps, in a row that reaches
    // this point (row_may_keep held), exactly the cells whose last-axis faces
    // enter no earlier than epre: one interval [mlo, mhi] of the row.
    const bool interval = KIND == ROW_C2R && pd.keep.enabled && pd.keep.face_axis >= 0 && pd.keep.face_axis != pd.d - 1;
    int64_t mlo = 0, mhi = -1;
    if (interval) {
        const int la = pd.d - 1;
        const int64_t goff = pick3(pd.keep.gorg, la) + b * pick3(pd.keep.gbstep, la);
        // entry time >= epre along the last axis: distance above s (epre - 1) from both faces
        const int64_t s = 1 + ((pd.keep.half_axes >> la) & 1);
        mlo = s * (rk.epre - 1) - goff;
        mhi = pick3(pd.keep.gdim, la) - s * (rk.epre - 1) - 1 - goff;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = q + P * i;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t mm = 2 * m + h;
            if (mm >= el) continue;
            if (interval) {
                if (mm < mlo || mm > mhi) continue;
            } else if (pd.keep.enabled && !keep_last(pd.keep, rk, pd.d, b, mm)) {
                continue;
            }
            out[base + mm * sl] = h ? v[i].y : v[i].x;
        }
    }
}

// ---------------------------------------------------------------------------
// Column passes
// ---------------------------------------------------------------------------
template <typename R, int MODE, int LOGL>
__device__ __forceinline__ void fcol_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    constexpr int L = 1 << LOGL;
    constexpr int P = L / 16;
    constexpr int NTH = col_threads<R>(LOGL);
    constexpr int W = NTH / P;
    const int cl = threadIdx.x % W;
    const int q = threadIdx.x / W;
    uint32_t tile = bid;
    if (pd.xcd_remap) {
        // workgroups are dealt round-robin over the 8 XCDs; give each XCD a
        // contiguous run of tiles so neighbouring columns share its L2
        const uint32_t per = (uint32_t)(pd.ntiles / 8);
        if (tile < 8 * per) tile = (tile % 8) * per + tile / 8;
    }
    const uint32_t ti = (uint32_t)pd.tiles_inner;
    const uint32_t o32 = tile / ti;
    const int64_t o = o32;
    const int64_t c = (int64_t)(tile - o32 * ti) * W + cl;
    const bool valid = c < pd.inner && (pd.cpitch == 0 || ((uint32_t)c % (uint32_t)pd.cpitch) < (uint32_t)pd.hcount);
    const ColIdx idx{cl, W + 1};
    const cx<R>* tlo = (const cx<R>*)pd.f_lo;
    const cx<R>* thi = (const cx<R>*)pd.f_hi;
    const int64_t step = (int64_t)P * pd.kstride;
    // (columns past the last valid one take no twiddle: their index would run past the table)
    const uint32_t twj = (pd.tw && valid) ? (uint32_t)c / (uint32_t)pd.tw_div : 0;
    cx<R> v[16];

    // ---------------- load
    if (pd.in_real) {
        const R* src = (const R*)pd.rv.ptr;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t m = (int64_t)(q + P * i) * pd.kstride + c;
            v[i] = cx<R>{(valid && m < pd.rv.ext[0]) ? src[o * pd.rv.boff + m * pd.rv.stride[0]] : R(0), R(0)};
        }
    } else {
        const cx<R>* src = (const cx<R>*)pd.buf + o * pd.ostride + (int64_t)q * pd.kstride + (valid ? c : 0);
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = valid ? src[i * step] : cx<R>{R(0), R(0)};
    }
    if (MODE == MODE_INV && pd.tw) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = cmulc(v[i], step_twiddle<R>(pd, (int64_t)(q + P * i) * twj));
    }

    if (MODE != MODE_INV) fast_fft<R, false, LOGL>(v, lds, idx, q, tlo, thi);

    if (MODE == MODE_MID) {
        // per-column part of the symbol, tabulated for this solve by k_symbol_columns
        const SymCol col = valid ? ((const SymCol*)sp.coltab)[c] : SymCol{};
        const int64_t fp = pos_to_freq(sp, 0, (o % pd.q_mod) * L);
        const int64_t M = sp.n[0] / L;
        apply_symbol<R, NTH>(v, lds, sp, col, (uint32_t)(fp + M * q), (uint32_t)(M * P));
        fast_fft<R, true, LOGL>(v, lds, idx, q, tlo, thi);
    }
    if (MODE == MODE_INV) fast_fft<R, true, LOGL>(v, lds, idx, q, tlo, thi);
    if (MODE == MODE_FWD && pd.tw) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = cmul(v[i], step_twiddle<R>(pd, (int64_t)(q + P * i) * twj));
    }

    // ---------------- store
    if (!valid) return;
    if (pd.out_real) {
        R* dst = (R*)pd.rvo.ptr;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t m = (int64_t)(q + P * i) * pd.kstride + c;
            if (m >= pd.rvo.ext[0]) continue;
            if (pd.keep.enabled && !keep_last(pd.keep, RowKeep{INT64_MAX, -1}, 1, o, m)) continue;
            dst[o * pd.rvo.boff + m * pd.rvo.stride[0]] = v[i].x;
        }
    } else {
        cx<R>* dst = (cx<R>*)pd.buf + o * pd.ostride + (int64_t)q * pd.kstride + c;
#pragma unroll
        for (int i = 0; i < 16; ++i) dst[i * step] = v[i];
    }
}

// ---------------------------------------------------------------------------
// Direct launches (descriptor in kernel arguments) and batched launches (a
// sorted work list of problems' passes that share this kernel variant).
__device__ __forceinline__ int batch_find(const BatchItem* it, int n, uint32_t bid) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (it[mid].first <= (int64_t)bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename R, int KIND, int LOGL>
__global__ __launch_bounds__(kThreads) void k_frow(PassDesc pd, SymParams sp) {
    frow_tile<R, KIND, LOGL>(pd, sp, blockIdx.x);
}
template <typename R, int KIND, int LOGL>
__global__ __launch_bounds__(kThreads) void k_frow_b(const BatchItem* it, int n, const SymParams* sy) {
    const int i = batch_find(it, n, blockIdx.x);
    frow_tile<R, KIND, LOGL>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
}
template <typename R, int MODE, int LOGL>
__global__ __launch_bounds__(kThreads) void k_fcol(PassDesc pd, SymParams sp) {
    fcol_tile<R, MODE, LOGL>(pd, sp, blockIdx.x);
}
template <typename R, int MODE, int LOGL>
__global__ __launch_bounds__(kThreads) void k_fcol_b(const BatchItem* it, int n, const SymParams* sy) {
    const int i = batch_find(it, n, blockIdx.x);
    fcol_tile<R, MODE, LOGL>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
}

struct BatchArgs {
    const BatchItem* items;
    int n;
    const SymParams* syms;
    int64_t tiles;
};

template <typename R, int LOGL>
static void launch_row_l(const PassDesc& pd, const SymParams& sp, size_t lds, hipStream_t st, const BatchArgs* ba) {
    const dim3 g((unsigned)(ba ? ba->tiles : pd.ntiles)), b(kThreads);
#define SFFT_ROW(K)                                                                               \
    if (ba) hipLaunchKernelGGL((k_frow_b<R, K, LOGL>), g, b, lds, st, ba->items, ba->n, ba->syms); \
    else hipLaunchKernelGGL((k_frow<R, K, LOGL>), g, b, lds, st, pd, sp);
    switch (pd.fast_kind) {
        case ROW_R2C: SFFT_ROW(ROW_R2C) break;
        case ROW_C2R: SFFT_ROW(ROW_C2R) break;
        case ROW_CFWD: SFFT_ROW(ROW_CFWD) break;
        case ROW_CINV: SFFT_ROW(ROW_CINV) break;
        case ROW_MIDR: SFFT_ROW(ROW_MIDR) break;
        default: SFFT_ROW(ROW_MIDC) break;
    }
#undef SFFT_ROW
}

template <typename R, int LOGL>
static void launch_col_l(const PassDesc& pd, const SymParams& sp, size_t lds, hipStream_t st, const BatchArgs* ba) {
    const dim3 g((unsigned)(ba ? ba->tiles : pd.ntiles)), b(col_threads<R>(LOGL));
#define SFFT_COL(M)                                                                               \
    if (ba) hipLaunchKernelGGL((k_fcol_b<R, M, LOGL>), g, b, lds, st, ba->items, ba->n, ba->syms); \
    else hipLaunchKernelGGL((k_fcol<R, M, LOGL>), g, b, lds, st, pd, sp);
    switch (pd.mode) {
        case MODE_FWD: SFFT_COL(MODE_FWD) break;
        case MODE_INV: SFFT_COL(MODE_INV) break;
        default: SFFT_COL(MODE_MID) break;
    }
#undef SFFT_COL
}

template <typename R>
static hipError_t launch_fast_t(const PassDesc& pd, const SymParams& sp, size_t lds, hipStream_t st,
                                const BatchArgs* ba) {
    if (pd.kind == PASS_ROW) {
        switch (pd.logL) {
            case 4: launch_row_l<R, 4>(pd, sp, lds, st, ba); break;
            case 5: launch_row_l<R, 5>(pd, sp, lds, st, ba); break;
            case 6: launch_row_l<R, 6>(pd, sp, lds, st, ba); break;
            case 7: launch_row_l<R, 7>(pd, sp, lds, st, ba); break;
            case 8: launch_row_l<R, 8>(pd, sp, lds, st, ba); break;
            case 9: launch_row_l<R, 9>(pd, sp, lds, st, ba); break;
            case 10: launch_row_l<R, 10>(pd, sp, lds, st, ba); break;
            case 11: launch_row_l<R, 11>(pd, sp, lds, st, ba); break;
            case 12: launch_row_l<R, 12>(pd, sp, lds, st, ba); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (pd.logL) {
            case 4: launch_col_l<R, 4>(pd, sp, lds, st, ba); break;
            case 5: launch_col_l<R, 5>(pd, sp, lds, st, ba); break;
            case 6: launch_col_l<R, 6>(pd, sp, lds, st, ba); break;
            case 7: launch_col_l<R, 7>(pd, sp, lds, st, ba); break;
            case 8: launch_col_l<R, 8>(pd, sp, lds, st, ba); break;
            case 9: launch_col_l<R, 9>(pd, sp, lds, st, ba); break;
            case 10: launch_col_l<R, 10>(pd, sp, lds, st, ba); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_fast_pass(const PassDesc& pd, const SymParams& sp, bool f64, size_t lds, hipStream_t st) {
    return f64 ? launch_fast_t<double>(pd, sp, lds, st, nullptr) : launch_fast_t<float>(pd, sp, lds, st, nullptr);
}

hipError_t launch_fast_batch(const PassDesc& proto, const BatchItem* items, int n, const SymParams* syms,
                             int64_t tiles, bool f64, size_t lds, hipStream_t st) {
    const BatchArgs ba{items, n, syms, tiles};
    SymParams dummy;
    return f64 ? launch_fast_t<double>(proto, dummy, lds, st, &ba) : launch_fast_t<float>(proto, dummy, lds, st, &ba);
}

}  // namespace sfft
