// Base case of RecursiveBoundary (Sec. 4): loop `steps` stencil steps near the
// fixed frame, in LDS, and store the cells of entry time <= steps.
//
// The band to produce (face f's cells within sig_f * steps of it, for every face
// the stencil reads toward) is cut into disjoint boxes ("strips", one per such
// face, later faces excluding what earlier faces cover) and each strip into
// tiles.  A workgroup loads its tile plus a halo of reach * steps cells per axis
// (clipped to the stored array, whose frame is fixed and read from the frame
// source), runs the steps in LDS (cells whose neighbourhood is not loaded keep
// stale values; the stale margin grows by at most the reach per step and never
// reaches the tile), and stores the tile.  Reads stay inside entry times
// <= 2 * steps, where the recursion guarantees valid input.
//
// Boundary condition (Sec. 4 leaves it to the base case): with a fixed frame the
// frame cells keep the values of the stored array; with a reflecting (zero-flux)
// boundary every frame cell in LDS is, at the start and after every step, a copy
// of its mirror image about the cell faces (interior cell r + k for frame cell
// r - 1 - k along each axis it lies outside of).  The copy of a frame cell is
// exactly as current as its mirror, which is nearer the tile than the frame cell
// itself, so every value a kept cell reads is still current.
#include <hip/hip_runtime.h>

#include "sfft_base.h"

namespace sfft {

// MAXC: LDS cells per thread, at least the largest loaded region / kBaseThreads.
// NC > 0: the stencil's coefficients and LDS offsets are unrolled into registers
// (NC entries, the ones past bp.ncoef zero with offset 0, adding +0), so a term
// costs one LDS read and one multiply-add; NC = 0 reads them from LDS per term.
template <typename R, int MAXC, int NC>
__global__ __launch_bounds__(kBaseThreads) void k_base(BaseParams bp) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R* A = reinterpret_cast<R*>(smem_raw);
    __shared__ int offs[kMaxCoef];
    __shared__ R coef[kMaxCoef];

    // which strip and tile
    const int64_t bid = blockIdx.x;
    int s = 0;
    while (s + 1 < bp.nstrip && bid >= bp.strip[s + 1].first) ++s;
    const BaseStrip& st = bp.strip[s];
    int64_t t = bid - st.first;
    int64_t org[3], ext[3];
    for (int a = 2; a >= 0; --a) {
        const int64_t ti = t % st.ntiles[a];
        t /= st.ntiles[a];
        org[a] = st.lo[a] + ti * st.tile[a];
        ext[a] = min(st.tile[a], st.lo[a] + st.ext[a] - org[a]);
    }
    // LDS region in storage coordinates: [rlo, rlo + rext)
    int64_t rlo[3], rext[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t slo = org[a] + bp.r3[a] - bp.halo3[a];
        const int64_t shi = org[a] + bp.r3[a] + ext[a] + bp.halo3[a];
        rlo[a] = slo < 0 ? 0 : slo;
        const int64_t sx = bp.n[a] + 2 * bp.r3[a];
        rext[a] = (shi > sx ? sx : shi) - rlo[a];
    }
    const int le1 = (int)rext[2];
    const int le0 = (int)(rext[1] * rext[2]);
    const int cells = (int)(rext[0] * rext[1] * rext[2]);

    if constexpr (NC == 0) {
        for (int i = threadIdx.x; i < bp.ncoef; i += kBaseThreads) {
            offs[i] = bp.off[i][0] * le0 + bp.off[i][1] * le1 + bp.off[i][2];
            coef[i] = (R)bp.c[i];
        }
    }
    constexpr int NR = NC > 0 ? NC : 1;
    int roff[NR];
    R rcoef[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const bool use = NC > 0 && j < bp.ncoef;
        roff[j] = use ? bp.off[j][0] * le0 + bp.off[j][1] * le1 + bp.off[j][2] : 0;
        rcoef[j] = use ? (R)bp.c[j] : R(0);
    }

    const R* src = (const R*)bp.src;
    const R* frame = (const R*)bp.frame;
    // load
    for (int i = threadIdx.x; i < cells; i += kBaseThreads) {
        const int x0 = i / le0, rem = i - x0 * le0, x1 = rem / le1, x2 = rem - x1 * le1;
        const int64_t g0 = rlo[0] + x0, g1 = rlo[1] + x1, g2 = rlo[2] + x2;
        const bool fr = g0 < bp.r3[0] || g0 >= bp.n[0] + bp.r3[0] || g1 < bp.r3[1] || g1 >= bp.n[1] + bp.r3[1] ||
                        g2 < bp.r3[2] || g2 >= bp.n[2] + bp.r3[2];
        const int64_t gi = g0 * bp.sstride[0] + g1 * bp.sstride[1] + g2 * bp.sstride[2];
        A[i] = fr ? (bp.bc ? R(0) : frame[gi]) : src[gi];
    }
    // per-thread cells and the last step at which each is updated (-1: never;
    // <= -2: a reflected frame cell copying LDS cell -2 - lim).
    // An interior cell whose whole neighbourhood is loaded is updated while it
    // can still reach the tile: a cell delta_a cells outside the tile along axis
    // a influences the tile's values after the last step only through steps
    // 0 .. steps - 1 - max_a ceil(delta_a / reach_a).  The cells such a cell reads
    // are at most one reach further out, so they are updated one step longer,
    // and every value a kept cell reads is current.
    int idx[MAXC];
    int lim[MAXC];
#pragma unroll
    for (int k = 0; k < MAXC; ++k) {
        const int i = threadIdx.x + k * kBaseThreads;
        idx[k] = i;
        lim[k] = -1;
        if (i < cells) {
            const int x0 = i / le0, rem = i - x0 * le0, x1 = rem / le1, x2 = rem - x1 * le1;
            const int64_t xs[3] = {x0, x1, x2};
            bool ok = true;
            bool frame_cell = false, mirror_in = true;
            int64_t need = 0, mli = 0;
            for (int a = 0; a < 3; ++a) {
                const int64_t g = rlo[a] + xs[a];
                const int64_t lo = bp.r3[a], hi = bp.n[a] + bp.r3[a];
                const int64_t gm = g < lo ? 2 * lo - 1 - g : (g >= hi ? 2 * hi - 1 - g : g);
                mirror_in = mirror_in && gm >= rlo[a] && gm < rlo[a] + rext[a];
                mli = mli * rext[a] + (gm - rlo[a]);
                if (g < lo || g >= hi) { ok = false; frame_cell = true; }           // frame cell
                if (xs[a] < bp.reach3[a] || xs[a] + bp.reach3[a] >= rext[a]) ok = false;  // neighbourhood not loaded
                const int64_t t0 = org[a] + bp.r3[a], t1 = t0 + ext[a] - 1;
                const int64_t delta = g < t0 ? t0 - g : (g > t1 ? g - t1 : 0);
                if (delta > 0 && bp.reach3[a] > 0) need = max(need, (delta + bp.reach3[a] - 1) / bp.reach3[a]);
            }
            if (ok) lim[k] = bp.steps - 1 - (int)need;
            if (bp.bc && frame_cell && mirror_in) lim[k] = -2 - (int)mli;
        }
    }
    __syncthreads();
    // reflecting boundary: frame cells := their mirror images (interior cells,
    // never written in this phase)
    auto reflect = [&]() {
#pragma unroll
        for (int k = 0; k < MAXC; ++k)
            if (lim[k] <= -2) A[idx[k]] = A[-2 - lim[k]];
        __syncthreads();
    };
    if (bp.bc) reflect();

    for (int step = 0; step < bp.steps; ++step) {
        R nv[MAXC];
#pragma unroll
        for (int k = 0; k < MAXC; ++k) {
            if (step <= lim[k]) {
                R acc = R(0);
                if constexpr (NC > 0) {
#pragma unroll
                    for (int j = 0; j < NC; ++j) acc += rcoef[j] * A[idx[k] + roff[j]];
                } else {
                    for (int j = 0; j < bp.ncoef; ++j) acc += coef[j] * A[idx[k] + offs[j]];
                }
                nv[k] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MAXC; ++k)
            if (step <= lim[k]) A[idx[k]] = nv[k];
        __syncthreads();
        if (bp.bc) reflect();
    }

    // store the tile (every tile cell lies in the band dist <= wout)
    R* dst = (R*)bp.dst;
    const int64_t tcells = ext[0] * ext[1] * ext[2];
    for (int64_t i = threadIdx.x; i < tcells; i += kBaseThreads) {
        const int64_t y0 = i / (ext[1] * ext[2]);
        const int64_t rem = i - y0 * ext[1] * ext[2];
        const int64_t y1 = rem / ext[2], y2 = rem - y1 * ext[2];
        const int64_t s0 = org[0] + bp.r3[0] + y0, s1 = org[1] + bp.r3[1] + y1, s2 = org[2] + bp.r3[2] + y2;
        const int li = (int)(((s0 - rlo[0]) * rext[1] + (s1 - rlo[1])) * rext[2] + (s2 - rlo[2]));
        dst[s0 * bp.sstride[0] + s1 * bp.sstride[1] + s2 * bp.sstride[2]] = A[li];
    }
}

template <typename R, int NC>
hipError_t launch_nc(const BaseParams& bp, int64_t nblocks, size_t lds, hipStream_t st) {
    // per-thread slots for the largest region (lds bytes of R cells): unused slots
    // still cost issue slots in the unrolled step loop, so use the smallest that fits
    const int64_t cells = (int64_t)(lds / sizeof(R));
    const dim3 g((unsigned)nblocks), b(kBaseThreads);
    if (cells <= 4 * kBaseThreads) hipLaunchKernelGGL((k_base<R, 4, NC>), g, b, lds, st, bp);
    else if (cells <= 8 * kBaseThreads) hipLaunchKernelGGL((k_base<R, 8, NC>), g, b, lds, st, bp);
    else if (cells <= 16 * kBaseThreads) hipLaunchKernelGGL((k_base<R, 16, NC>), g, b, lds, st, bp);
    else if (cells <= kBaseMaxCells) hipLaunchKernelGGL((k_base<R, kBaseMaxCells / kBaseThreads, NC>), g, b, lds, st, bp);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R>
hipError_t launch_r(const BaseParams& bp, int64_t nblocks, size_t lds, hipStream_t st) {
    // the stencils' common term counts (1-D, 5- and 7-point stars, 3 x 3 and
    // 3 x 3 x 3 boxes, 5 x 5 boxes; shorter lists pad up with zero terms)
    const int n = bp.ncoef;
    if (n <= 3) return launch_nc<R, 3>(bp, nblocks, lds, st);
    if (n <= 5) return launch_nc<R, 5>(bp, nblocks, lds, st);
    if (n <= 7) return launch_nc<R, 7>(bp, nblocks, lds, st);
    if (n <= 9) return launch_nc<R, 9>(bp, nblocks, lds, st);
    if (n <= 25) return launch_nc<R, 25>(bp, nblocks, lds, st);
    if (n <= 27) return launch_nc<R, 27>(bp, nblocks, lds, st);
    return launch_nc<R, 0>(bp, nblocks, lds, st);
}

hipError_t launch_base(const BaseParams& bp, bool f64, int64_t nblocks, size_t lds, hipStream_t st) {
    return f64 ? launch_r<double>(bp, nblocks, lds, st) : launch_r<float>(bp, nblocks, lds, st);
}

}  // namespace sfft
