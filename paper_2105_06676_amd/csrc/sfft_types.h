// Descriptors shared by the host planner and the HIP kernels.
//
// A periodic solve is a short list of passes over one complex spectrum buffer
// (Sec. 3, StencilFFT-P): a forward pass per axis (the first one real-to-complex
// along the contiguous axis), one fused middle pass that finishes the forward
// transform of axis 0, multiplies by lambda^T / N (Steps 1(i), 2 and 3) and
// starts the inverse transform, then inverse passes in reverse order (Step 4).
// Every pass is "rows" (transform along the contiguous axis, whole rows in LDS)
// or "columns" (transform along a strided axis, a tile of W adjacent columns
// in LDS).  Long strided axes are split into up to three sub-transforms with
// twiddles between them (Cooley-Tukey, Sec. 2); the forward output is left in
// digit-reversed order, which the symbol lookup undoes and the inverse passes
// consume directly, so no transposes are needed.
#pragma once

#include <stdint.h>

namespace sfft {

constexpr int kThreads = 256;     // threads per FFT workgroup (four wave64s)
// threads per generic (mixed-radix) tile of up to 8192 points: 16 points each in
// FP32, 8 in FP64 (the registers a stage holds across its barrier)
template <typename R>
constexpr int gen_threads() { return sizeof(R) == 8 ? 1024 : 512; }
constexpr int kMaxStages = 16;    // radix stages per sub-transform
constexpr int kMaxCoef = 125;     // (2r+1)^d for r <= 2, d <= 3
constexpr int kMaxR = 2;          // largest stencil radius with a fused symbol
constexpr int kTileElems = 8192;  // complex elements one FFT tile may hold
constexpr int kTwSplit = 1024;    // split twiddles: exp(-2 pi i e / N) = lo[e mod 1024] * hi[e div 1024]
constexpr int kTwSplitLog = 10;

enum PassKind { PASS_ROW = 0, PASS_COL = 1 };
enum PassMode { MODE_FWD = 0, MODE_INV = 1, MODE_MID = 2 };
// How a row pass maps real data to its complex transform.
//  RT_C2C : the row is complex already (1-D problems split over rows)
//  RT_HALF: even real length n, transformed as n/2 complex points plus an
//           even/odd untangling step (n/2+1 spectral entries stored)
//  RT_ODD : odd real length n, transformed as n complex points with zero
//           imaginary part ((n+1)/2 spectral entries stored)
enum RowTrans { RT_C2C = 0, RT_HALF = 1, RT_ODD = 2 };

// A strided real array: the first pass reads it, the last pass writes it.
struct RealView {
    void* ptr;            // float* or double*, per the pass precision
    int64_t boff;         // element offset between consecutive batch items
    int64_t stride[3];    // element stride of axes 0..d-1
    int64_t ext[3];       // cells at index >= ext along an axis read as zero and are never written
};

// Which output cells the last pass stores (Sec. 4 region bookkeeping, with the
// entry times of the appendix on l-shells).  A face at index distance dist_f - 1
// from global interior cell g enters it after ell_f = ceil(dist_f / s_a) steps,
// s_a the stencil's reach per step along the face's axis a (1 or 2: 2 for the axes
// in half_axes); ell(g) = min over faces.  A cell is stored iff lo < ell <= hi
// and, when face_axis >= 0, the first face (axis 0 low, axis 0 high, axis 1 low,
// ...) with that entry time is the slab's own face.
struct KeepRule {
    int enabled;
    int face_axis;        // -1: no face test
    int face_side;        // 0 low, 1 high, -1 either side, 2 = the batch index
    int half_axes;        // bit a: entry time along axis a is ceil(dist / 2)
    int64_t lo, hi;
    int64_t gdim[3];      // interior extents
    int64_t gorg[3];      // global coordinate of local cell 0 of batch item 0
    int64_t gbstep[3];    // added per batch item
};

// Everything the fused middle pass needs to form lambda(k)^T / N in FP64.
struct SymParams {
    int d, r, ncoef, real_sym;
    // 0: coefficients of one sign, normalised on the host by lambda(0) = sum(c)
    //    (the largest |lambda| of all modes), so the branch-free deviation-form
    //    power keeps the accuracy of the dominant modes; 1: mixed signs, every
    //    mode leaves the deviation form once it is far from 1 (relative accuracy
    //    per mode, data-dependent branches)
    int switching;
    int pad_sym;
    int64_t T;
    double one_minus_sum;     // 1 - sum(c), exact (host TwoSum); 0 after normalisation
    double scale;             // lambda(0)^T / prod(n) after normalisation, else 1 / prod(n)
    int64_t n[3];             // transform extents per axis
    int nlev[3];              // sub-transform levels per axis
    int64_t sub[3][3];        // sub-lengths per axis in pass order
    int64_t sdim[3];          // spectrum buffer extents per axis (last axis padded)
    int64_t hcount;           // valid entries along the last axis (d >= 2)
    const void* eph[3];       // per-axis tables exp(2 pi i m / n_a) - 1, FP64 complex
    const void* coltab;       // d >= 2: per-column symbol parts (SymCol) of the middle pass
    int64_t ncol;             // entries of coltab
    double c[kMaxCoef];       // coefficients, row-major over offsets
};

struct PassDesc {
    int kind, mode, rowtrans;
    int in_real, out_real;
    int L;                    // complex transform length of this (sub-)pass
    int nreal;                // row passes: real length (RT_HALF / RT_ODD)
    int hcount;               // row passes: stored spectral entries per row
    int W;                    // columns per tile (col) or rows per tile (row)
    int lds_stride;           // row passes: LDS stride between rows (complex elements)
    int64_t outer, inner;     // col: [outer][L][inner]; row: outer = number of rows
    int64_t ostride, kstride; // complex buffer strides (col: o, k; row: row, -)
    int64_t ntiles;           // workgroups of this pass
    int64_t tiles_inner;      // col: tiles per outer index
    // twiddle between sub-transforms: w = exp(-+2 pi i (k * (c / tw_div)) / tw_n)
    int tw;                   // 0 none, 1 multiply after forward / before inverse
    int tw_B;                 // two-level table split: e = q * tw_B + l
    int64_t tw_n, tw_div;
    const void* tw_lo;        // exp(-2 pi i l / tw_n), l < tw_B
    const void* tw_hi;        // exp(-2 pi i q tw_B / tw_n)
    // radix stages; stage twiddles read exp(-2 pi i m / st_n) at m = e * st_mul
    const void* st_tab;
    int st_mul;
    int nst;
    int radix[kMaxStages];
    void* buf;                // complex spectrum buffer
    RealView rv;              // real input of the first pass
    RealView rvo;             // real output of the last pass
    KeepRule keep;
    // problem geometry for addressing real views and the symbol
    int d;
    int pad2_;
    int64_t B;                // batch items
    int64_t rdims[3];         // transform extents per axis
    int64_t q_mod;            // mid pass: prefix digits of axis 0 = (outer or row) % q_mod
    int64_t cpitch;           // col passes: padded pitch of the last axis inside `inner`
                              // (columns with (c % cpitch) >= hcount are padding); 0 = none
    // power-of-two fast kernels
    int fast;                 // 1: run the register radix-16 kernels
    int fast_kind;            // row passes: R2C / C2R / 1-D real middle / complex middle
    int logL;
    int xcd_remap;            // column passes: place consecutive tiles on one XCD
    const void* f_lo;         // exp(-2 pi i m / L): m mod 64 ...
    const void* f_hi;         // ... and 64 * (m div 64)
    const void* h_lo;         // exp(-2 pi i m / 2L) for the real-data untangling
    const void* h_hi;
    // register mixed-radix kernels: points per thread (0: not used), threads per
    // workgroup, stage radices packed 4 bits each (first stage lowest)
    int mq;
    int mthreads;
    int64_t mrad;
};

// One problem's pass inside a batched launch: workgroups [first, first + pd.ntiles)
// of the launch run this pass with symbol parameters syms[sym].
struct BatchItem {
    PassDesc pd;
    int64_t first;
    int sym;
    int pad_;
};

// The host fills these structs and the kernels read them (by value in kernel
// arguments, or from device memory in batched launches), so both compilation
// passes must agree on their layout; a change here is checked in both.
static_assert(sizeof(void*) == 8 && sizeof(int64_t) == 8, "LP64 layout assumed");
static_assert(sizeof(RealView) == 64 && alignof(RealView) == 8, "RealView layout");
static_assert(sizeof(KeepRule) == 104 && alignof(KeepRule) == 8, "KeepRule layout");
static_assert(sizeof(SymParams) == 1232 && alignof(SymParams) == 8, "SymParams layout");
static_assert(sizeof(PassDesc) == 568 && alignof(PassDesc) == 8, "PassDesc layout");
static_assert(sizeof(BatchItem) == 584 && alignof(BatchItem) == 8, "BatchItem layout");
static_assert(__builtin_offsetof(PassDesc, rvo) == 280 && __builtin_offsetof(PassDesc, keep) == 344 &&
              __builtin_offsetof(PassDesc, mq) == 552, "PassDesc field offsets");
static_assert(__builtin_offsetof(SymParams, eph) == 192 && __builtin_offsetof(SymParams, c) == 232,
              "SymParams field offsets");
// one direct launch passes a PassDesc and a SymParams by value: well inside the
// 4 KiB of kernel arguments
static_assert(sizeof(PassDesc) + sizeof(SymParams) + 64 <= 4096, "kernel argument budget");

}  // namespace sfft
