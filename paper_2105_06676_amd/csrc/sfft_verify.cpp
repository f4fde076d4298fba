// Host-side verification of pass schedules (no device needed).
//
// Every index a pass kernel forms is an affine function of its loop indices
// (row or tile, point, column, batch item) with non-negative coefficients (the
// descriptor's strides), each index running over a box given by the
// descriptor's bounds.  The largest address a pass can touch is therefore that
// function at the upper corner of the box, and the smallest is the buffer's
// origin.  This file evaluates those corners for every pass of a schedule and
// checks them against the buffers the solve hands the passes: the spectrum
// workspace, the real input and output views, the symbol column table, and the
// twiddle and stage tables of each pass.  The aperiodic solver runs its whole
// bookkeeping in this mode with no device work (every slab, interior and
// recursion-level solve is checked with its real views and keep rules).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/stencil_fft.h"
#include "sfft_plan.h"
#include "sfft_runtime.h"
#include "sfft_verify.h"

namespace sfft {

void Verifier::add(const void* base, size_t bytes, const std::string& name) {
    bufs.push_back({(uintptr_t)base, bytes, name});
}

void Verifier::fail(const std::string& what) {
    if (errors.size() < 64) errors.push_back(what);
    ++nerr;
}

void Verifier::range(const void* p, int64_t hi_elem, size_t esz, const std::string& what) {
    ++checked;
    if (hi_elem < 0) return;  // nothing addressed
    const uintptr_t lo = (uintptr_t)p, hi = lo + (uintptr_t)(hi_elem + 1) * esz;
    for (const Buf& b : bufs)
        if (lo >= b.base && lo < b.base + b.bytes) {
            if (hi > b.base + b.bytes)
                fail(what + ": reaches " + std::to_string(hi - b.base) + " bytes into " + b.name + " of " +
                     std::to_string(b.bytes));
            return;
        }
    fail(what + ": starts outside every buffer");
}

namespace {

// Largest element offset of a real view over `rows` iterated row coordinates
// (axes 0..d-2, clipped to the view's extents), `B` batch items and `last`
// elements along the last axis.
int64_t view_max(const RealView& v, int d, int64_t B, const int64_t* rdims, int64_t last) {
    int64_t m = (B - 1) * v.boff;
    for (int a = 0; a < d - 1; ++a) m += (std::min(rdims[a], v.ext[a]) - 1) * v.stride[a];
    m += (std::min(last, v.ext[d - 1]) - 1) * v.stride[d - 1];
    return m;
}

}  // namespace

void Verifier::schedule(const Schedule& s, const void* ws, const RealView& in, const RealView& out,
                        const void* coltab, int64_t ncol, const std::string& tag) {
    const size_t esz = s.f64 ? 8 : 4, csz = 2 * esz;
    for (size_t i = 0; i < s.passes.size(); ++i) {
        const PassPlan& pp = s.passes[i];
        const PassDesc& pd = pp.pd;
        const std::string w = tag + " pass " + std::to_string(i) + " (" + pp.name + ")";
        const int64_t L = pd.L;
        if (pd.kind == PASS_ROW) {
            // rows of a real view are the batch items times the transform extents of
            // axes 0..d-2 (rows of a split axis' complex middle pass are sub-transforms)
            int64_t rows = pd.B;
            for (int a = 0; a < pd.d - 1; ++a) rows *= pd.rdims[a];
            ++checked;
            if ((pd.in_real || pd.out_real) && rows != pd.outer)
                fail(w + ": row count " + std::to_string(pd.outer) + " != " + std::to_string(rows));
            const int64_t entries = pd.rowtrans == RT_HALF ? L + 1 : (pd.rowtrans == RT_ODD ? pd.hcount : L);
            if (!(pd.in_real && pd.out_real)) range(ws, (pd.outer - 1) * pd.ostride + entries - 1, csz, w + " spectrum");
            if (pd.ostride < entries && pd.outer > 1 && !(pd.in_real && pd.out_real))
                fail(w + ": spectrum rows overlap (stride " + std::to_string(pd.ostride) + ")");
            const int64_t len = pd.rowtrans == RT_HALF ? 2 * L : (pd.rowtrans == RT_ODD ? pd.nreal : L);
            if (pd.in_real) range(in.ptr, view_max(in, pd.d, pd.B, pd.rdims, len), esz, w + " real input");
            if (pd.out_real) range(out.ptr, view_max(out, pd.d, pd.B, pd.rdims, len), esz, w + " real output");
        } else {
            const int64_t tiles = pd.outer * pd.tiles_inner;
            if (tiles != pd.ntiles) fail(w + ": tile count mismatch");
            if (pd.tiles_inner * pd.W < pd.inner) fail(w + ": tiles do not cover the columns");
            if (!(pd.in_real && pd.out_real))
                range(ws, (pd.outer - 1) * pd.ostride + (L - 1) * pd.kstride + pd.inner - 1, csz, w + " spectrum");
            // a real view along the (only) strided axis: element m = k kstride + c < ext[0]
            // (k < L, c < inner)
            const int64_t mmax = (L - 1) * pd.kstride + pd.inner;
            if (pd.in_real) range(in.ptr, (pd.outer - 1) * in.boff + (std::min(mmax, in.ext[0]) - 1) * in.stride[0],
                                  esz, w + " real input");
            if (pd.out_real)
                range(out.ptr, (pd.outer - 1) * out.boff + (std::min(mmax, out.ext[0]) - 1) * out.stride[0], esz,
                      w + " real output");
            if (pd.tw) {
                // twiddle exp(-2 pi i k (c / tw_div) / tw_n) for k < L, c < inner
                const int64_t e = (L - 1) * ((pd.inner - 1) / pd.tw_div);
                ++checked;
                if (e >= pd.tw_n) fail(w + ": twiddle index " + std::to_string(e) + " >= " + std::to_string(pd.tw_n));
                if (pp.has_tw && (e / pd.tw_B) >= pp.tw_hi.count) fail(w + ": twiddle table too short");
            }
            if (pd.mode == MODE_MID && s.fused && s.d >= 2) {
                ++checked;
                if (coltab && pd.inner > ncol)
                    fail(w + ": " + std::to_string(pd.inner) + " columns, symbol table of " + std::to_string(ncol));
            }
        }
        // stage table of the generic and mixed-radix kernels: exp(-2 pi i m / (L st_mul)), m < L st_mul
        if (!pd.fast) {
            ++checked;
            if (pp.stage_tab.count < (int64_t)L * pd.st_mul) fail(w + ": stage table shorter than the transform");
        }
    }
}

}  // namespace sfft
