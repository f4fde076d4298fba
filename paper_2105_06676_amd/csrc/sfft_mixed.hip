// Register mixed-radix pass kernels (gfx950) for 7-smooth lengths: 5, 7, 9, 10,
// 12, 14, 15, 20, 21 or 25 points per thread, by the length's family.
//
// A transform of L points is done by P = L/Q threads that each hold Q points
// (Q a compile-time constant of the length's family): thread q holds x[q + P i],
// i < Q, on entry and on exit (natural order).  The first Stockham stage has
// radix Q: a thread's Q registers are one butterfly, computed as a composite
// in-register DFT (Q = A B: B transforms of length A, the constant twiddles, A
// transforms of length B).  The last stage leaves its outputs in the registers
// when its radix divides Q; every stage in between exchanges the points through
// LDS once, with the stage twiddles read from the pass's table
// exp(-2 pi i m / (L st_mul)).  Middle stages whose radix does not divide Q
// spread their butterflies unevenly over the threads (guarded); a last radix that
// divides no Q runs like a middle stage and the threads read their outputs back
// from LDS (gather).  Most of a length is covered by radix-Q stages, so a
// transform takes few LDS exchanges and barriers.  The stage list is packed in
// PassDesc::mrad (5 bits per stage), so the kernels index no array at run time;
// divisions by the run-time, workgroup-uniform P, W and Ns go through the float
// reciprocal of sfft_device.h.  The same tile code (loads, the real-data
// untangling, the fused symbol step, keep rules, stores) as the power-of-two
// register kernels.
//
// Kernels:
//  k_mrow<R, KIND, Q, RL>  rows: R2C first pass, C2R last pass, whole 1-D real
//                          solve (even and odd real lengths), complex middle rows
//                          of split 1-D axes
//  k_mcol<R, MODE, Q, RL>  strided axis: forward / inverse / fused middle pass
// (RL: radix of the last stage; 1 for the gather form)
#include <hip/hip_runtime.h>

#include "sfft_device.h"
#include "sfft_fast.h"
#include "sfft_mixed.h"
#include "sfft_symapply.h"

namespace sfft {

namespace {

constexpr int kMRowThreads = 512;  // most threads of a mixed-radix row workgroup
constexpr int kMColThreads = 256;  // ... and of a column workgroup

struct MRowIdx {
    int base;
    __device__ __forceinline__ int operator()(int e) const { return base + e + (e >> 4); }
};
struct MColIdx {
    int c, ws;
    __device__ __forceinline__ int operator()(int e) const { return e * ws + c; }
};

// One Stockham stage of radix RAD on the Q points of each of the P threads of a
// transform (NS = product of the radices already applied).  FIRST: the inputs
// are the registers (NS = 1, no twiddles); otherwise they are read from LDS.
// LAST: the outputs go to the registers in natural order; otherwise to LDS at
// their self-sorting positions.  The flags are compile-time so that the point
// registers are dead between the first and the last stage.
template <typename R, int Q, int RAD, bool INV, bool FIRST, bool LAST, typename IDX>
__device__ __forceinline__ void mstage(cx<R> (&v)[Q], cx<R>* lds, IDX idx, int q, int P, int L, int NS,
                                       const cx<R>* tab, int tmul) {
    // A middle stage whose radix does not divide Q spreads its L / RAD butterflies
    // over the P threads unevenly: NB = ceil(Q / RAD) per thread, the last ones
    // guarded.  The first and the last stage hold the point registers and need
    // RAD | Q.
    constexpr bool EXACT = Q % RAD == 0;
    static_assert(EXACT || (!FIRST && !LAST), "register stages need a radix dividing Q");
    constexpr int NB = (Q + RAD - 1) / RAD;
    const int span = L / RAD;
    cx<R> w[NB][RAD];
    const UDiv dns = udiv((uint32_t)NS);
    if (FIRST) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int t = 0; t < RAD; ++t) w[b][t] = v[b + t * NB];
    } else {
        const int step = (L / (NS * RAD)) * tmul;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = q + P * b;
            if (!EXACT && j >= span) {
#pragma unroll
                for (int t = 0; t < RAD; ++t) w[b][t] = cx<R>{R(0), R(0)};
                continue;
            }
#pragma unroll
            for (int t = 0; t < RAD; ++t) w[b][t] = lds[idx(j + t * span)];
            uint32_t jq;
            const int k = (int)udiv_qr((uint32_t)j, dns, &jq);
            const cx<R> w1 = tab[k * step];
            if constexpr (RAD <= 5 || RAD == 7) {
                cx<R> wt = w1;
#pragma unroll
                for (int t = 1; t < RAD; ++t) {
                    w[b][t] = INV ? cmulc(w[b][t], wt) : cmul(w[b][t], wt);
                    if (t + 1 < RAD) wt = cmul(wt, w1);
                }
            } else {
                // w1^t for t = a BS + c as (w1^BS)^a w1^c, both factors by short
                // product chains from two table entries (a few roundings, not RAD)
                constexpr int BS = RAD % 7 == 0 ? 7 : (RAD % 5 == 0 ? 5 : (RAD % 4 == 0 ? 4 : 3));
                const cx<R> wb = tab[k * BS * step];
                cx<R> lo[BS];
                lo[0] = cx<R>{R(1), R(0)};
                lo[1] = w1;
#pragma unroll
                for (int c = 2; c < BS; ++c) lo[c] = cmul(lo[c - 1], w1);
                cx<R> hi = wb;
#pragma unroll
                for (int a = 0; a < RAD / BS; ++a) {
#pragma unroll
                    for (int c = 0; c < BS; ++c) {
                        if (a == 0 && c == 0) continue;
                        const cx<R> wt = a == 0 ? lo[c] : (c == 0 ? hi : cmul(hi, lo[c]));
                        w[b][a * BS + c] = INV ? cmulc(w[b][a * BS + c], wt) : cmul(w[b][a * BS + c], wt);
                    }
                    if (a > 0 && a + 1 < RAD / BS) hi = cmul(hi, wb);
                }
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) dft<R, RAD, INV>(w[b]);
    if (!LAST) {
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = q + P * b;
            if (!EXACT && j >= span) continue;
            uint32_t jq;
            const int k = (int)udiv_qr((uint32_t)j, dns, &jq);
            const int d = (int)jq * NS * RAD + k;
#pragma unroll
            for (int t = 0; t < RAD; ++t) lds[idx(d + t * NS)] = w[b][t];
        }
        __syncthreads();
    } else {
        // outputs y[q + P (b + t NB)] -> natural register order
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int t = 0; t < RAD; ++t) v[b + t * NB] = w[b][t];
    }
}

// Middle stages: the radices that divide Q, and for the families that mix 3, 5
// and 7 (Q = 7, 9, 12, 14, 15, 21) also 2, 3, 4, 5 and 7 with guarded butterflies;
// X4: also a guarded radix 4 (10-point first-pass rows, where it replaces two
// radix-2 exchanges by one; a separate kernel variant, so the other 10-point
// kernels keep their registers).
template <typename R, int Q, bool INV, bool FIRST, bool LAST, bool X4 = false, typename IDX>
__device__ __forceinline__ void mstage_rad(int rad, cx<R> (&v)[Q], cx<R>* lds, IDX idx, int q, int P, int L, int NS,
                                           const cx<R>* tab, int tmul) {
#define SFFT_MST(RAD)                                                                                      if constexpr (Q % RAD == 0) mstage<R, Q, RAD, INV, FIRST, LAST>(v, lds, idx, q, P, L, NS, tab, tmul);
#define SFFT_MSTG(RAD)                                                                                     \
    if constexpr (Q % RAD == 0 || Q == 7 || Q == 9 || Q == 12 || Q == 14 || Q == 15 || Q == 21 || (X4 && RAD == 4)) \
        mstage<R, Q, RAD, INV, FIRST, LAST>(v, lds, idx, q, P, L, NS, tab, tmul);
    switch (rad) {
        case 2: SFFT_MSTG(2) break;
        case 3: SFFT_MSTG(3) break;
        case 4: SFFT_MSTG(4) break;
        case 5: SFFT_MSTG(5) break;
        case 7: SFFT_MSTG(7) break;
        case 6: SFFT_MST(6) break;
        case 9: SFFT_MST(9) break;
        case 10: SFFT_MST(10) break;
        case 12: SFFT_MST(12) break;
        case 14: SFFT_MST(14) break;
        case 15: SFFT_MST(15) break;
        case 20: SFFT_MST(20) break;
        case 21: SFFT_MST(21) break;
        default: SFFT_MST(25) break;
    }
#undef SFFT_MST
#undef SFFT_MSTG
}

// Stage lists (the planner's canonical order): the first stage has radix Q (a
// thread's Q registers form one butterfly, computed as a composite in-register
// DFT), then the middle stages, then a last stage of radix RL (Q again when the
// length holds two factors Q).  The first and last radices are compile-time, so
// no stage that touches the point registers sits behind a run-time switch
// (which would move the registers to scratch memory); radix-Q stages keep the
// number of LDS exchanges (and workgroup barriers) per transform small.

// Length-L transform of the Q points held by each of the P threads (stage
// radices in pd.mrad, pd.nst >= 2 stages, the first of radix Q, the last RL).
// RL = 1 (gather): the last radix does not divide Q, so every stage after the
// first goes through LDS like a middle one; Stockham's self-sorting order leaves
// the outputs in natural order there, and each thread reads its Q points back
// (one more exchange, for lengths no register family takes otherwise, such as
// 35, 42 or 210 points).
template <typename R, int Q, int RL, bool INV, bool X4 = false, typename IDX>
__device__ __forceinline__ void mfft(cx<R> (&v)[Q], cx<R>* lds, IDX idx, int q, int P, const PassDesc& pd) {
    const cx<R>* tab = (const cx<R>*)pd.st_tab;
    const int L = pd.L, tmul = pd.st_mul, nst = pd.nst;
    const uint64_t rads = (uint64_t)pd.mrad;
    mstage<R, Q, Q, INV, true, false>(v, lds, idx, q, P, L, 1, tab, tmul);
    int NS = Q;
    constexpr int NMID_END = RL == 1 ? 0 : 1;  // stages left for the register stage
    for (int s = 1; s < nst - NMID_END; ++s) {
        const int rad = mixed_radix_at((int64_t)rads, s);
        mstage_rad<R, Q, INV, false, false, X4>(rad, v, lds, idx, q, P, L, NS, tab, tmul);
        NS *= rad;
    }
    if constexpr (RL == 1) {
        // (the last stage's barrier orders its LDS writes before these reads; every
        // later writer of this LDS starts with a barrier)
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = lds[idx(q + P * i)];
    } else {
        mstage<R, Q, RL, INV, false, true>(v, lds, idx, q, P, L, NS, tab, tmul);
    }
}

// ---------------------------------------------------------------------------
// Row passes
// ---------------------------------------------------------------------------
template <typename R, int KIND, int Q, int RL, bool X4 = false>
__device__ __forceinline__ void mrow_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    const int L = pd.L;
    const int P = L / Q;
    const int NTR = pd.W;
    const int LS = L + L / 16 + 2;
    // the workgroup has exactly NTR * P threads
    uint32_t rr_u;
    const int q = (int)udiv_qr((uint32_t)threadIdx.x, udiv((uint32_t)P), &rr_u);
    const int rr = (int)rr_u;
    const int64_t row = (int64_t)bid * NTR + rr;
    bool active = row < pd.outer;
    const MRowIdx idx{rr * LS};
    // exp(-2 pi i m / 2L) for the real-data untangling (the pass table has 2L entries)
    const cx<R>* htab = (const cx<R>*)pd.st_tab;
    cx<R> v[Q];

    int64_t ii[3] = {0, 0, 0};
    int64_t b = 0;
    {
        int64_t rem = active ? row : 0;
#pragma unroll
        for (int a = 1; a >= 0; --a) {
            if (a <= pd.d - 2) {
                const int64_t n = a == 1 ? pd.rdims[1] : pd.rdims[0];
                const int64_t qq = rem / n;
                ii[a] = rem - qq * n;
                rem = qq;
            }
        }
        b = rem;
    }
    if (KIND == ROW_C2R && active && pd.keep.enabled && !row_may_keep(pd.keep, keep_row(pd.keep, pd.d, b, ii), pd.d, b))
        active = false;
    auto row_base = [&](const RealView& rv) -> int64_t {
        int64_t off = b * rv.boff;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (a < pd.d - 1) {
                if (ii[a] >= rv.ext[a]) return -1;
                off += ii[a] * rv.stride[a];
            }
        }
        return off;
    };

    // ---------------- load
    if (KIND == ROW_R2C || KIND == ROW_MIDR) {
        const R* src = (const R*)pd.rv.ptr;
        const int64_t base = active ? row_base(pd.rv) : -1;
        const int64_t sl = pick3(pd.rv.stride, pd.d - 1), el = pick3(pd.rv.ext, pd.d - 1);
        const bool vec = base >= 0 && sl == 1 && el >= 2 * L && ((((uintptr_t)(src + base)) % (2 * sizeof(R))) == 0);
        if (vec) {
            const cx<R>* s2 = (const cx<R>*)(src + base) + q;
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = s2[P * i];
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
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
        for (int i = 0; i < Q; ++i) v[i] = active ? src[P * i] : cx<R>{R(0), R(0)};
    }

    cx<R> xl = {R(0), R(0)};  // X[L] of a half-spectrum row (held by q == 0)
    if (KIND == ROW_C2R) {
        if (q == 0) lds[idx(L)] = active ? ((const cx<R>*)pd.buf)[row * pd.ostride + L] : cx<R>{R(0), R(0)};
    } else {
        mfft<R, Q, RL, false, X4>(v, lds, idx, q, P, pd);
    }

    if (KIND == ROW_R2C || KIND == ROW_MIDR) {
        // untangle the half-length transform: X[k] from Z[k] and Z[L-k]
        __syncthreads();
#pragma unroll
        for (int i = 0; i < Q; ++i) lds[idx(q + P * i)] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int k = q + P * i;
            const cx<R> zk = v[i];
            if (k == 0) {
                v[i] = cx<R>{zk.x + zk.y, R(0)};
                xl = cx<R>{zk.x - zk.y, R(0)};
            } else {
                const cx<R> zm = lds[idx(L - k)];
                const cx<R> e = scale(zk + conj(zm), R(0.5));
                const cx<R> o = scale(zk - conj(zm), R(0.5));
                const cx<R> t = cmul(htab[k], o);
                v[i] = cx<R>{e.x + t.y, e.y - t.x};
            }
        }
        if (KIND == ROW_R2C) {
            if (active) {
                cx<R>* dst = (cx<R>*)pd.buf + row * pd.ostride + q;
#pragma unroll
                for (int i = 0; i < Q; ++i) dst[P * i] = v[i];
                if (q == 0) dst[L] = xl;
            }
            return;
        }
        // 1-D middle: multiply X[k], k = 0..L, by lambda^T / n
        const SymCol col = symbol_column_1d(sp);
        apply_symbol<R, kMRowThreads, Q, kMGroup<Q>()>(v, lds, sp, col, (uint32_t)q, (uint32_t)P);
        if (q == 0) {
            const int64_t fl = L;
            dcx s;
            symbol_power_n<1>(sp, col, &fl, &s);
            xl = cmul(xl, cx<R>{R(s.x), R(s.y)});
        }
    }

    // tangle for the half-length inverse:
    // Z'[k] = (X[k] + conj X[L-k]) + i conj(w^k) (X[k] - conj X[L-k]), w = exp(-2 pi i / 2L)
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) lds[idx(q + P * i)] = v[i];
    if (KIND != ROW_C2R && q == 0) lds[idx(L)] = xl;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int k = q + P * i;
        const cx<R> xk = v[i], xm = lds[idx(L - k)];
        const cx<R> e = xk + conj(xm);
        const cx<R> o = cmulc(xk - conj(xm), htab[k]);
        v[i] = cx<R>{e.x - o.y, e.y + o.x};
    }
    __syncthreads();

    mfft<R, Q, RL, true, X4>(v, lds, idx, q, P, pd);

    // ---------------- store: x[2m] = Re z[m], x[2m+1] = Im z[m]
    if (!active) return;
    R* out = (R*)pd.rvo.ptr;
    const int64_t base = row_base(pd.rvo);
    if (base < 0) return;
    const int64_t sl = pick3(pd.rvo.stride, pd.d - 1), el = pick3(pd.rvo.ext, pd.d - 1);
    const bool vec = !pd.keep.enabled && sl == 1 && el >= 2 * L &&
                     ((((uintptr_t)(out + base)) % (2 * sizeof(R))) == 0);
    if (vec) {
        cx<R>* d2 = (cx<R>*)(out + base) + q;
#pragma unroll
        for (int i = 0; i < Q; ++i) d2[P * i] = v[i];
        return;
    }
    const RowKeep rk = keep_row(pd.keep, pd.d, b, ii);
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
    for (int i = 0; i < Q; ++i) {
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

// Rows of odd real length n (RT_ODD): one n-point complex transform of (x, 0)
// per row.  The first pass stores the h = (n + 1) / 2 entries of the half
// spectrum; the last pass takes the others as the conjugates of their mirrors
// X[n - k], read straight from the stored half (no exchange), transforms back and
// keeps the real parts; the whole 1-D solve multiplies all n modes by the symbol
// power between the two transforms.  Odd Q only (an odd length has no even factor).
template <typename R, int KIND, int Q, int RL>
__device__ __forceinline__ void mrow_odd_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    const int L = pd.L;
    const int P = L / Q;
    const int NTR = pd.W;
    const int LS = L + L / 16 + 2;
    uint32_t rr_u;
    const int q = (int)udiv_qr((uint32_t)threadIdx.x, udiv((uint32_t)P), &rr_u);
    const int rr = (int)rr_u;
    const int64_t row = (int64_t)bid * NTR + rr;
    bool active = row < pd.outer;
    const MRowIdx idx{rr * LS};
    cx<R> v[Q];

    int64_t ii[3] = {0, 0, 0};
    int64_t b = 0;
    {
        int64_t rem = active ? row : 0;
#pragma unroll
        for (int a = 1; a >= 0; --a) {
            if (a <= pd.d - 2) {
                const int64_t n = a == 1 ? pd.rdims[1] : pd.rdims[0];
                const int64_t qq = rem / n;
                ii[a] = rem - qq * n;
                rem = qq;
            }
        }
        b = rem;
    }
    if (KIND == ROW_C2R_ODD && active && pd.keep.enabled &&
        !row_may_keep(pd.keep, keep_row(pd.keep, pd.d, b, ii), pd.d, b))
        active = false;
    auto row_base = [&](const RealView& rv) -> int64_t {
        int64_t off = b * rv.boff;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (a < pd.d - 1) {
                if (ii[a] >= rv.ext[a]) return -1;
                off += ii[a] * rv.stride[a];
            }
        }
        return off;
    };

    // ---------------- load
    if (KIND == ROW_C2R_ODD) {
        const cx<R>* src = (const cx<R>*)pd.buf + (active ? row : 0) * pd.ostride;
        const int h = pd.hcount;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int k = q + P * i;
            v[i] = !active ? cx<R>{R(0), R(0)} : (k < h ? src[k] : conj(src[L - k]));
        }
    } else {
        const R* src = (const R*)pd.rv.ptr;
        const int64_t base = active ? row_base(pd.rv) : -1;
        const int64_t sl = pick3(pd.rv.stride, pd.d - 1), el = pick3(pd.rv.ext, pd.d - 1);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int m = q + P * i;
            v[i] = cx<R>{(base >= 0 && m < el) ? src[base + (int64_t)m * sl] : R(0), R(0)};
        }
        mfft<R, Q, RL, false>(v, lds, idx, q, P, pd);
    }

    if (KIND == ROW_R2C_ODD) {
        if (active) {
            cx<R>* dst = (cx<R>*)pd.buf + row * pd.ostride;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int k = q + P * i;
                if (k < pd.hcount) dst[k] = v[i];
            }
        }
        return;
    }
    if (KIND == ROW_MIDR_ODD) {
        // 1-D whole solve: thread q holds frequencies q + P i of all n
        const SymCol col = symbol_column_1d(sp);
        apply_symbol<R, kMRowThreads, Q, kMGroup<Q>()>(v, lds, sp, col, (uint32_t)q, (uint32_t)P);
    }
    mfft<R, Q, RL, true>(v, lds, idx, q, P, pd);

    // ---------------- store the real parts
    if (!active) return;
    R* out = (R*)pd.rvo.ptr;
    const int64_t base = row_base(pd.rvo);
    if (base < 0) return;
    const int64_t sl = pick3(pd.rvo.stride, pd.d - 1), el = pick3(pd.rvo.ext, pd.d - 1);
    const RowKeep rk = keep_row(pd.keep, pd.d, b, ii);
    const bool interval = KIND == ROW_C2R_ODD && pd.keep.enabled && pd.keep.face_axis >= 0 &&
                          pd.keep.face_axis != pd.d - 1;
    int64_t mlo = 0, mhi = -1;
    if (interval) {
        const int la = pd.d - 1;
        const int64_t goff = pick3(pd.keep.gorg, la) + b * pick3(pd.keep.gbstep, la);
        const int64_t s = 1 + ((pd.keep.half_axes >> la) & 1);
        mlo = s * (rk.epre - 1) - goff;
        mhi = pick3(pd.keep.gdim, la) - s * (rk.epre - 1) - 1 - goff;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t m = q + P * i;
        if (m >= el) continue;
        if (interval) {
            if (m < mlo || m > mhi) continue;
        } else if (pd.keep.enabled && !keep_last(pd.keep, rk, pd.d, b, m)) {
            continue;
        }
        out[base + m * sl] = v[i].x;
    }
}

// Complex middle rows of a 1-D axis split into strided levels and a row level
// (ROW_MIDC): load the row, forward transform, multiply position k by the symbol
// power of its axis-0 frequency (the digit-reversed prefix of the strided levels
// plus (n / L) k), inverse transform, store.
template <typename R, int Q, int RL, bool X4 = false>
__device__ __forceinline__ void mrow_c2c_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    const int L = pd.L;
    const int P = L / Q;
    const int NTR = pd.W;
    const int LS = L + L / 16 + 2;
    uint32_t rr_u;
    const int q = (int)udiv_qr((uint32_t)threadIdx.x, udiv((uint32_t)P), &rr_u);
    const int rr = (int)rr_u;
    const int64_t row = (int64_t)bid * NTR + rr;
    const bool active = row < pd.outer;
    const MRowIdx idx{rr * LS};
    cx<R> v[Q];
    const cx<R>* src = (const cx<R>*)pd.buf + (active ? row : 0) * pd.ostride + q;
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] = active ? src[P * i] : cx<R>{R(0), R(0)};
    mfft<R, Q, RL, false, X4>(v, lds, idx, q, P, pd);
    const int64_t qd = active ? (row % pd.q_mod) : 0;
    const int64_t fp = pos_to_freq(sp, 0, qd * L);
    const int64_t M = sp.n[0] / L;
    const SymCol col = symbol_column_1d(sp);
    apply_symbol<R, kMRowThreads, Q, kMGroup<Q>()>(v, lds, sp, col, (uint32_t)(fp + M * q), (uint32_t)(M * P));
    mfft<R, Q, RL, true, X4>(v, lds, idx, q, P, pd);
    if (!active) return;
    cx<R>* dst = (cx<R>*)pd.buf + row * pd.ostride + q;
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[P * i] = v[i];
}

// ---------------------------------------------------------------------------
// Column passes
// ---------------------------------------------------------------------------
template <typename R, int MODE, int Q, int RL>
__device__ __forceinline__ void mcol_tile(const PassDesc& pd, const SymParams& sp, uint32_t bid) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);
    const int L = pd.L;
    const int P = L / Q;
    const int W = pd.W;
    // the workgroup has exactly W * P threads
    uint32_t q_u;
    const int cl = (int)udiv_qr((uint32_t)threadIdx.x, udiv((uint32_t)W), &q_u);
    const int q = (int)q_u;
    uint32_t tile = bid;
    if (pd.xcd_remap) {
        const uint32_t per = (uint32_t)(pd.ntiles / 8);
        if (tile < 8 * per) tile = (tile % 8) * per + tile / 8;
    }
    const uint32_t ti = (uint32_t)pd.tiles_inner;
    const uint32_t o32 = tile / ti;
    const int64_t o = o32;
    const int64_t c = (int64_t)(tile - o32 * ti) * W + cl;
    const bool valid = c < pd.inner &&
                       (pd.cpitch == 0 || ((uint32_t)c % (uint32_t)pd.cpitch) < (uint32_t)pd.hcount);
    const MColIdx idx{cl, W + 1};
    const int64_t step = (int64_t)P * pd.kstride;
    // (columns past the last valid one take no twiddle: their index would run past the table)
    const uint32_t twj = (pd.tw && valid) ? (uint32_t)c / (uint32_t)pd.tw_div : 0;
    const int qq = q;
    cx<R> v[Q];

    // ---------------- load
    if (pd.in_real) {
        const R* src = (const R*)pd.rv.ptr;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t m = (int64_t)(qq + P * i) * pd.kstride + c;
            v[i] = cx<R>{(valid && m < pd.rv.ext[0]) ? src[o * pd.rv.boff + m * pd.rv.stride[0]] : R(0), R(0)};
        }
    } else {
        const cx<R>* src = (const cx<R>*)pd.buf + o * pd.ostride + (int64_t)qq * pd.kstride + (valid ? c : 0);
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = valid ? src[i * step] : cx<R>{R(0), R(0)};
    }
    if (MODE == MODE_INV && pd.tw) {
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = cmulc(v[i], step_twiddle<R>(pd, (int64_t)(qq + P * i) * twj));
    }

    if (MODE != MODE_INV) mfft<R, Q, RL, false>(v, lds, idx, qq, P, pd);

    if (MODE == MODE_MID) {
        const SymCol col = valid ? ((const SymCol*)sp.coltab)[c] : SymCol{};
        const int64_t fp = pos_to_freq(sp, 0, (o % pd.q_mod) * L);
        const int64_t M = sp.n[0] / L;
        apply_symbol<R, kMColThreads, Q, kMGroup<Q>()>(v, lds, sp, col, (uint32_t)(fp + M * qq), (uint32_t)(M * P));
        mfft<R, Q, RL, true>(v, lds, idx, qq, P, pd);
    }
    if (MODE == MODE_INV) mfft<R, Q, RL, true>(v, lds, idx, qq, P, pd);
    if (MODE == MODE_FWD && pd.tw) {
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = cmul(v[i], step_twiddle<R>(pd, (int64_t)(qq + P * i) * twj));
    }

    // ---------------- store
    if (!valid) return;
    if (pd.out_real) {
        R* dst = (R*)pd.rvo.ptr;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t m = (int64_t)(qq + P * i) * pd.kstride + c;
            if (m >= pd.rvo.ext[0]) continue;
            if (pd.keep.enabled && !keep_last(pd.keep, RowKeep{INT64_MAX, -1}, 1, o, m)) continue;
            dst[o * pd.rvo.boff + m * pd.rvo.stride[0]] = v[i].x;
        }
    } else {
        cx<R>* dst = (cx<R>*)pd.buf + o * pd.ostride + (int64_t)qq * pd.kstride + c;
#pragma unroll
        for (int i = 0; i < Q; ++i) dst[i * step] = v[i];
    }
}

__device__ __forceinline__ int batch_find_m(const BatchItem* it, int n, uint32_t bid) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (it[mid].first <= (int64_t)bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Waves per SIMD the row kernels are compiled for.  A long row is one workgroup
// of L / Q threads; at 10 FP32 points per thread the unconstrained kernels take
// about 110 VGPRs, four waves per SIMD, so only two 7-wave rows fit a CU.  Six
// waves per SIMD (80 VGPRs, a few words of spill) fit three.
template <typename R, int KIND, int Q>
constexpr int mrow_waves() { return (sizeof(R) == 4 && Q == 10 && KIND != ROW_MIDR && KIND != ROW_MIDC) ? 6 : 1; }

template <typename R, int KIND, int Q, int RL, bool X4 = false>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kMRowThreads), amdgpu_waves_per_eu(mrow_waves<R, KIND, Q>())))
void k_mrow(PassDesc pd, SymParams sp) {
    if constexpr (KIND >= ROW_R2C_ODD) mrow_odd_tile<R, KIND, Q, RL>(pd, sp, blockIdx.x);
    else if constexpr (KIND == ROW_MIDC) mrow_c2c_tile<R, Q, RL, X4>(pd, sp, blockIdx.x);
    else mrow_tile<R, KIND, Q, RL, X4>(pd, sp, blockIdx.x);
}
template <typename R, int KIND, int Q, int RL, bool X4 = false>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kMRowThreads), amdgpu_waves_per_eu(mrow_waves<R, KIND, Q>())))
void k_mrow_b(const BatchItem* it, int n, const SymParams* sy) {
    const int i = batch_find_m(it, n, blockIdx.x);
    if constexpr (KIND >= ROW_R2C_ODD)
        mrow_odd_tile<R, KIND, Q, RL>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
    else if constexpr (KIND == ROW_MIDC)
        mrow_c2c_tile<R, Q, RL, X4>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
    else
        mrow_tile<R, KIND, Q, RL, X4>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
}
// The 20- and 25-point FP32 fused middle passes take about 190 VGPRs unconstrained
// (two waves per SIMD); three waves per SIMD fit one more workgroup per CU.
template <typename R, int MODE, int Q>
constexpr int mcol_waves() { return (sizeof(R) == 4 && Q >= 20 && MODE == MODE_MID) ? 3 : 1; }

template <typename R, int MODE, int Q, int RL>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kMColThreads), amdgpu_waves_per_eu(mcol_waves<R, MODE, Q>())))
void k_mcol(PassDesc pd, SymParams sp) {
    mcol_tile<R, MODE, Q, RL>(pd, sp, blockIdx.x);
}
template <typename R, int MODE, int Q, int RL>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kMColThreads), amdgpu_waves_per_eu(mcol_waves<R, MODE, Q>())))
void k_mcol_b(const BatchItem* it, int n, const SymParams* sy) {
    const int i = batch_find_m(it, n, blockIdx.x);
    mcol_tile<R, MODE, Q, RL>(it[i].pd, sy[it[i].sym], (uint32_t)(blockIdx.x - it[i].first));
}

struct MBatch {
    const BatchItem* items;
    int n;
    const SymParams* syms;
    int64_t tiles;
};

template <typename R, int Q, int RL>
hipError_t launch_q(const PassDesc& pd, const SymParams& sp, size_t lds, hipStream_t st, const MBatch* ba) {
    const dim3 g((unsigned)(ba ? ba->tiles : pd.ntiles)), b((unsigned)pd.mthreads);
    if (pd.kind == PASS_ROW) {
        // rows take at most 10 points per thread when the length has a factor 2:
        // there are no 20-point row kernels
        if constexpr (Q == 20) {
            return hipErrorInvalidValue;
        } else {
#define SFFT_MROW(K)                                                                               \
    if (ba) hipLaunchKernelGGL((k_mrow_b<R, K, Q, RL>), g, b, lds, st, ba->items, ba->n, ba->syms);     \
    else hipLaunchKernelGGL((k_mrow<R, K, Q, RL>), g, b, lds, st, pd, sp);
            if constexpr (Q == 10 && RL == 10) {
                bool x4 = false;
                for (int s = 1; s + 1 < pd.nst; ++s) x4 = x4 || mixed_radix_at(pd.mrad, s) == 4;
                if (x4) {
#define SFFT_MROW4(K)                                                                                \
    if (ba) hipLaunchKernelGGL((k_mrow_b<R, K, Q, RL, true>), g, b, lds, st, ba->items, ba->n, ba->syms); \
    else hipLaunchKernelGGL((k_mrow<R, K, Q, RL, true>), g, b, lds, st, pd, sp);
                    // (the planner gives radix-4 stages to first-pass rows only)
                    if (pd.fast_kind != ROW_R2C) return hipErrorInvalidValue;
                    SFFT_MROW4(ROW_R2C)
#undef SFFT_MROW4
                    return hipGetLastError();
                }
            }
            switch (pd.fast_kind) {
                case ROW_R2C: SFFT_MROW(ROW_R2C) break;
                case ROW_C2R: SFFT_MROW(ROW_C2R) break;
                case ROW_MIDR: SFFT_MROW(ROW_MIDR) break;
                case ROW_MIDC: SFFT_MROW(ROW_MIDC) break;
                default:
                    // odd real lengths: odd Q only
                    if constexpr (Q % 2 == 1) {
                        switch (pd.fast_kind) {
                            case ROW_R2C_ODD: SFFT_MROW(ROW_R2C_ODD) break;
                            case ROW_C2R_ODD: SFFT_MROW(ROW_C2R_ODD) break;
                            case ROW_MIDR_ODD: SFFT_MROW(ROW_MIDR_ODD) break;
                            default: return hipErrorInvalidValue;
                        }
                    } else {
                        return hipErrorInvalidValue;
                    }
            }
#undef SFFT_MROW
        }
    } else {
#define SFFT_MCOL(M)                                                                               \
    if (ba) hipLaunchKernelGGL((k_mcol_b<R, M, Q, RL>), g, b, lds, st, ba->items, ba->n, ba->syms);     \
    else hipLaunchKernelGGL((k_mcol<R, M, Q, RL>), g, b, lds, st, pd, sp);
        switch (pd.mode) {
            case MODE_FWD: SFFT_MCOL(MODE_FWD) break;
            case MODE_INV: SFFT_MCOL(MODE_INV) break;
            default: SFFT_MCOL(MODE_MID) break;
        }
#undef SFFT_MCOL
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_m(const PassDesc& pd, const SymParams& sp, size_t lds, hipStream_t st, const MBatch* ba) {
    if (pd.nst < 2) return hipErrorInvalidValue;
    const int rl = mixed_radix_at(pd.mrad, pd.nst - 1);
    // every middle radix must have a stage in the kernel variant chosen below (a
    // radix without one would be skipped, not reported)
    const int Q = pd.mq;
    const bool guarded = Q == 7 || Q == 9 || Q == 12 || Q == 14 || Q == 15 || Q == 21;
    const bool x4 = Q == 10 && rl == 10 && pd.kind == PASS_ROW && pd.fast_kind == ROW_R2C;
    for (int s = 1; s < pd.nst - (Q % rl ? 0 : 1); ++s) {
        const int rad = mixed_radix_at(pd.mrad, s);
        const bool small = rad == 2 || rad == 3 || rad == 4 || rad == 5 || rad == 7;
        const bool listed = rad == 6 || rad == 9 || rad == 10 || rad == 12 || rad == 14 || rad == 15 ||
                            rad == 20 || rad == 21 || rad == 25;
        const bool ok = (Q % rad == 0 && (small || listed)) || (guarded && small) || (x4 && rad == 4);
        if (!ok) return hipErrorInvalidValue;
    }
    // (Q, last radix) pairs the planner's canonical order produces
    // (FP32 only for 20 and 25 points per thread: FP64 would hold one wave per SIMD)
    // last radix not dividing Q: the gather form (families 7, 9, 12, 14, 15, 21)
    if (pd.mq % rl != 0) {
        if (pd.mq == 7) return launch_q<R, 7, 1>(pd, sp, lds, st, ba);
        if (pd.mq == 9) return launch_q<R, 9, 1>(pd, sp, lds, st, ba);
        if (pd.mq == 12) return launch_q<R, 12, 1>(pd, sp, lds, st, ba);
        if (pd.mq == 14) return launch_q<R, 14, 1>(pd, sp, lds, st, ba);
        if (pd.mq == 15) return launch_q<R, 15, 1>(pd, sp, lds, st, ba);
        if constexpr (sizeof(R) == 4) {
            if (pd.mq == 21) return launch_q<R, 21, 1>(pd, sp, lds, st, ba);
        }
        return hipErrorInvalidValue;
    }
    if (pd.mq == 5 && rl == 5) return launch_q<R, 5, 5>(pd, sp, lds, st, ba);
    if (pd.mq == 7 && rl == 7) return launch_q<R, 7, 7>(pd, sp, lds, st, ba);
    if (pd.mq == 9 && rl == 9) return launch_q<R, 9, 9>(pd, sp, lds, st, ba);
    if (pd.mq == 9 && rl == 3) return launch_q<R, 9, 3>(pd, sp, lds, st, ba);
    if (pd.mq == 10 && rl == 10) return launch_q<R, 10, 10>(pd, sp, lds, st, ba);
    if (pd.mq == 10 && rl == 2) return launch_q<R, 10, 2>(pd, sp, lds, st, ba);
    if (pd.mq == 10 && rl == 5) return launch_q<R, 10, 5>(pd, sp, lds, st, ba);
    if (pd.mq == 12 && rl == 12) return launch_q<R, 12, 12>(pd, sp, lds, st, ba);
    if (pd.mq == 12 && rl == 2) return launch_q<R, 12, 2>(pd, sp, lds, st, ba);
    if (pd.mq == 12 && rl == 3) return launch_q<R, 12, 3>(pd, sp, lds, st, ba);
    if (pd.mq == 14 && rl == 14) return launch_q<R, 14, 14>(pd, sp, lds, st, ba);
    if (pd.mq == 14 && rl == 2) return launch_q<R, 14, 2>(pd, sp, lds, st, ba);
    if (pd.mq == 14 && rl == 7) return launch_q<R, 14, 7>(pd, sp, lds, st, ba);
    if (pd.mq == 15 && rl == 15) return launch_q<R, 15, 15>(pd, sp, lds, st, ba);
    if (pd.mq == 15 && rl == 3) return launch_q<R, 15, 3>(pd, sp, lds, st, ba);
    if (pd.mq == 15 && rl == 5) return launch_q<R, 15, 5>(pd, sp, lds, st, ba);
    if constexpr (sizeof(R) == 4) {
        if (pd.mq == 20 && rl == 20) return launch_q<R, 20, 20>(pd, sp, lds, st, ba);
        if (pd.mq == 20 && rl == 2) return launch_q<R, 20, 2>(pd, sp, lds, st, ba);
        if (pd.mq == 20 && rl == 5) return launch_q<R, 20, 5>(pd, sp, lds, st, ba);
        if (pd.mq == 25 && rl == 25) return launch_q<R, 25, 25>(pd, sp, lds, st, ba);
        if (pd.mq == 25 && rl == 5) return launch_q<R, 25, 5>(pd, sp, lds, st, ba);
        if (pd.mq == 21 && rl == 21) return launch_q<R, 21, 21>(pd, sp, lds, st, ba);
        if (pd.mq == 21 && rl == 3) return launch_q<R, 21, 3>(pd, sp, lds, st, ba);
        if (pd.mq == 21 && rl == 7) return launch_q<R, 21, 7>(pd, sp, lds, st, ba);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_mixed_pass(const PassDesc& pd, const SymParams& sp, bool f64, size_t lds, hipStream_t st) {
    return f64 ? launch_m<double>(pd, sp, lds, st, nullptr) : launch_m<float>(pd, sp, lds, st, nullptr);
}

hipError_t launch_mixed_batch(const PassDesc& proto, const BatchItem* items, int n, const SymParams* syms,
                              int64_t tiles, bool f64, size_t lds, hipStream_t st) {
    const MBatch ba{items, n, syms, tiles};
    SymParams dummy;
    return f64 ? launch_m<double>(proto, dummy, lds, st, &ba) : launch_m<float>(proto, dummy, lds, st, &ba);
}

}  // namespace sfft
