// Periodic solves on any extents (Sec. 3 Steps 1-4 with the DFT of a length
// that has a prime factor above 7 taken by Bluestein's chirp-z algorithm).
//
// The grid is widened to a complex array; each axis is transformed in turn (a
// 7-smooth axis by the complex pass kernels in place, digit-reversed across its
// factor levels; any other axis by chirp-multiply and zero-pad to a 7-smooth
// length M >= 2n - 1, forward transform, product with the transformed chirp
// kernel, inverse transform, extract and chirp-multiply: natural order); every
// spectral element is multiplied by lambda(k)^T / N; the inverse runs the same way
// in reverse order with conjugate chirps; the real part is stored back.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <map>
#include <tuple>
#include <vector>

#include "sfft_bluestein.h"
#include "sfft_fields.h"
#include "sfft_kernels.h"
#include "sfft_runtime.h"
#include "sfft_solvers.h"

namespace sfft {

namespace {

int64_t smooth_at_least(int64_t n) {
    while (!is_7smooth(n)) ++n;
    return n;
}

// Convolution length for an axis of n points: a power of two (whose transforms
// run on the register radix-16 kernels, several times faster than the generic
// mixed-radix ones) unless that pads more than 2x the next 7-smooth length.
int64_t conv_len(int64_t n) {
    const int64_t need = 2 * n - 1;
    int64_t p = 1;
    while (p < need) p *= 2;
    const int64_t s = smooth_at_least(need);
    return p <= 2 * s ? p : s;
}

struct BlueTables {
    double2* chirp[2] = {nullptr, nullptr};  // forward (sign -1), inverse (sign +1)
    void* H[2] = {nullptr, nullptr};         // transformed chirp kernels / M, natural order
};

std::mutex g_blue_mu;
std::map<std::tuple<int, int64_t, int64_t, bool>, BlueTables> g_blue;

AxisOrder order_of(const Plan& p) {
    AxisOrder o;
    std::memset(&o, 0, sizeof(o));
    o.nlev = p.s.sym.nlev[0];
    for (int i = 0; i < 3; ++i) o.sub[i] = p.s.sym.sub[0][i];
    return o;
}

// Enqueue one elementwise launch, timed under `name` when profiling is on.
template <typename F>
void timed(hipStream_t st, const char* name, bool f64, int64_t bytes, F&& launch) {
    hipEvent_t ev = nullptr;
    const bool prof = profiling();
    if (prof) profile_launch_begin(st, &ev);
    check_hip(launch(), name);
    if (prof) profile_launch_end(st, ev, std::string(name) + (f64 ? "_f64" : "_f32"), bytes);
}

void run_passes(const Plan& p, void* buf, hipStream_t st) {
    if (p.pd.empty()) return;
    RealView v;
    std::memset(&v, 0, sizeof(v));
    KeepRule keep;
    std::memset(&keep, 0, sizeof(keep));
    SymParams sp;
    std::memset(&sp, 0, sizeof(sp));
    run_plan(p, buf, v, v, keep, sp, st);
}

// Tables of an axis of n points convolved at length M (built once per device).
const BlueTables& blue_tables(int64_t n, int64_t M, bool f64, hipStream_t st) {
    DevCtx& ctx = device_ctx();
    const auto key = std::make_tuple(ctx.device, n, M, f64);
    std::lock_guard<std::mutex> g(g_blue_mu);
    auto it = g_blue.find(key);
    if (it != g_blue.end()) return it->second;
    BlueTables t;
    const size_t csz = f64 ? 16 : 8;
    auto fwd = ctx.axis_plan(1, M, 1, f64, false);
    void* tmp = nullptr;
    check_hip(hipMalloc(&tmp, (size_t)M * csz), "hipMalloc(chirp kernel)");
    for (int k = 0; k < 2; ++k) {
        check_hip(hipMalloc(&t.chirp[k], sizeof(double2) * (size_t)n), "hipMalloc(chirp)");
        check_hip(hipMalloc(&t.H[k], (size_t)M * csz), "hipMalloc(chirp spectrum)");
        check_hip(launch_chirp(t.chirp[k], n, k == 0 ? -1 : 1, st), "chirp");
        check_hip(launch_chirp_kernel(tmp, t.chirp[k], n, M, f64, st), "chirp kernel");
        run_passes(*fwd, tmp, st);
        check_hip(launch_reorder_scale(tmp, t.H[k], M, order_of(*fwd), f64, st), "chirp spectrum order");
    }
    check_hip(hipStreamSynchronize(st), "hipStreamSynchronize(chirp tables)");
    check_hip(hipFree(tmp), "hipFree(chirp kernel)");
    return g_blue.emplace(key, t).first->second;
}

// The transformed kernel H of direction k laid out in the position order `o` of
// the length-M forward transform (built once per device and order), so that the
// product reads it contiguously.
std::map<std::tuple<int, int64_t, int64_t, bool, int, int, int64_t, int64_t, int64_t>, void*> g_hpos;

const void* h_positions(const BlueTables& t, int k, int64_t n, int64_t M, bool f64, const AxisOrder& o,
                        hipStream_t st) {
    if (o.nlev <= 1) return t.H[k];
    DevCtx& ctx = device_ctx();
    const auto key = std::make_tuple(ctx.device, n, M, f64, k, o.nlev, o.sub[0], o.sub[1], o.sub[2]);
    std::lock_guard<std::mutex> g(g_blue_mu);
    auto it = g_hpos.find(key);
    if (it != g_hpos.end()) return it->second;
    void* d = nullptr;
    check_hip(hipMalloc(&d, (size_t)M * (f64 ? 16 : 8)), "hipMalloc(chirp spectrum positions)");
    check_hip(launch_gather_order(t.H[k], d, M, o, f64, st), "chirp spectrum positions");
    check_hip(hipStreamSynchronize(st), "hipStreamSynchronize(chirp spectrum positions)");
    return g_hpos.emplace(key, d).first->second;
}

// Forward (inverse = false) or inverse DFT along axis a of the complex array ws.
void axis_transform(void* ws, void* tmp, int64_t outer, int64_t n, int64_t inner, bool f64, bool inverse,
                    SymParams* sp, int a, hipStream_t st) {
    DevCtx& ctx = device_ctx();
    if (is_7smooth(n)) {
        auto p = ctx.axis_plan(outer, n, inner, f64, inverse);
        run_passes(*p, ws, st);
        if (sp) {
            sp->nlev[a] = p->s.sym.nlev[0];
            for (int i = 0; i < 3; ++i) sp->sub[a][i] = p->s.sym.sub[0][i];
        }
        return;
    }
    const int64_t M = conv_len(n);
    const BlueTables& t = blue_tables(n, M, f64, st);
    const int k = inverse ? 1 : 0;
    auto fwd = ctx.axis_plan(outer, M, inner, f64, false);
    auto inv = ctx.axis_plan(outer, M, inner, f64, true);
    const int64_t csz = f64 ? 16 : 8;
    timed(st, "chirp_pad", f64, outer * inner * (n + M) * csz,
          [&] { return launch_pad_chirp(ws, tmp, outer, n, inner, M, t.chirp[k], f64, st); });
    run_passes(*fwd, tmp, st);
    const void* Hp = h_positions(t, k, n, M, f64, order_of(*fwd), st);
    AxisOrder natural;
    std::memset(&natural, 0, sizeof(natural));
    timed(st, "chirp_product", f64, 2 * outer * inner * M * csz,
          [&] { return launch_mul_h(tmp, outer, M, inner, Hp, natural, f64, st); });
    run_passes(*inv, tmp, st);
    timed(st, "chirp_extract", f64, 2 * outer * inner * n * csz,
          [&] { return launch_extract_chirp(tmp, ws, outer, n, inner, M, t.chirp[k], f64, st); });
    if (sp) {
        sp->nlev[a] = 1;  // natural frequency order
        sp->sub[a][0] = n;
    }
}

}  // namespace

namespace {
// Byte offsets of the solve's buffers inside one region: workspace, convolution
// scratch, column table.
struct AnyLayout {
    size_t ws, tmp, col, total;
};
AnyLayout any_layout(bool f64, int d, const int64_t* dims) {
    const size_t csz = f64 ? 16 : 8;
    int64_t N = 1;
    for (int a = 0; a < d; ++a) N *= dims[a];
    int64_t tmp_elems = 1;
    for (int a = 0; a < d; ++a) {
        if (is_7smooth(dims[a])) continue;
        tmp_elems = std::max(tmp_elems, N / dims[a] * conv_len(dims[a]));
    }
    int64_t ncol = 1;
    for (int a = 1; a < d; ++a) ncol *= dims[a];
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    AnyLayout l;
    l.ws = 0;
    l.tmp = up((size_t)N * csz);
    l.col = l.tmp + up((size_t)tmp_elems * csz);
    l.total = l.col + (d >= 2 ? up((size_t)ncol * symbol_column_bytes()) : 0);
    return l;
}
}  // namespace

size_t periodic_any_footprint(bool f64, int d, const int64_t* dims) { return any_layout(f64, d, dims).total; }

void solve_periodic_any(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r, int64_t T,
                        hipStream_t st, void* pool) {
    DevCtx& ctx = device_ctx();
    const size_t csz = f64 ? 16 : 8;
    int64_t N = 1;
    for (int a = 0; a < d; ++a) N *= dims[a];
    const AnyLayout lay = any_layout(f64, d, dims);
    void* ws = pool ? pool : ctx.workspace(st, lay.tmp);
    void* tmp = pool ? (char*)pool + lay.tmp : ctx.scratch(st, 70, lay.col - lay.tmp);
    SymParams sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.d = d;
    for (int a = 0; a < 3; ++a) sp.n[a] = a < d ? dims[a] : 1;
    fill_symbol(sp, coeffs, r, d, T, 1.0 / (double)N);
    for (int a = 0; a < d; ++a) sp.eph[a] = ctx.phase_table(dims[a]);

    const int64_t esz = f64 ? 8 : 4;
    timed(st, "widen", f64, N * (esz + (int64_t)csz), [&] { return launch_widen(grid, ws, N, f64, st); });
    for (int a = 0; a < d; ++a) {
        int64_t outer = 1, inner = 1;
        for (int b = 0; b < a; ++b) outer *= dims[b];
        for (int b = a + 1; b < d; ++b) inner *= dims[b];
        axis_transform(ws, tmp, outer, dims[a], inner, f64, false, &sp, a, st);
    }
    if (d >= 2) {
        // the part of the symbol that depends on axes 1..d-1, once per column
        for (int a = 0; a < d; ++a) sp.sdim[a] = dims[a];
        int64_t ncol = 1;
        for (int a = 1; a < d; ++a) ncol *= dims[a];
        build_symbol_columns(sp, pool ? (char*)pool + lay.col : ctx.scratch(st, 71, (size_t)ncol * symbol_column_bytes()),
                             f64, st);
    }
    timed(st, "symbol_full", f64, 2 * N * (int64_t)csz, [&] { return launch_symbol_full(ws, sp, N, f64, st); });
    for (int a = d - 1; a >= 0; --a) {
        int64_t outer = 1, inner = 1;
        for (int b = 0; b < a; ++b) outer *= dims[b];
        for (int b = a + 1; b < d; ++b) inner *= dims[b];
        axis_transform(ws, tmp, outer, dims[a], inner, f64, true, nullptr, a, st);
    }
    timed(st, "narrow", f64, N * (esz + (int64_t)csz), [&] { return launch_narrow(ws, grid, N, f64, st); });
}

// m coupled fields (appendix on vector-valued fields), or an implicit stencil on
// one field (appendix on implicit stencils), on any extents: the m fields are one
// more outer axis of the widened array, every axis is transformed as above, and
// the symbol-matrix power (sfft_fields.hip) runs over the full spectrum with every
// axis's stored positions mapped to frequencies.
void solve_fields_any(void* grid, bool f64, int m, int d, const int64_t* dims, const double* coeffs, int r,
                      int64_t T, hipStream_t st, const double* q_coeffs) {
    DevCtx& ctx = device_ctx();
    const size_t csz = f64 ? 16 : 8;
    int64_t N = 1;
    for (int a = 0; a < d; ++a) N *= dims[a];
    int64_t tmp_elems = 1;
    for (int a = 0; a < d; ++a)
        if (!is_7smooth(dims[a])) tmp_elems = std::max(tmp_elems, (int64_t)m * (N / dims[a]) * conv_len(dims[a]));
    void* ws = ctx.workspace(st, (size_t)m * N * csz);
    void* tmp = ctx.scratch(st, 72, (size_t)tmp_elems * csz);
    FieldParams fp;
    const std::vector<double> cK = field_constants(m, d, coeffs, r, q_coeffs, &fp);
    fp.full = 1;
    fp.rows = N / dims[d - 1];
    fp.pitch = dims[d - 1];
    fp.fstride = N;
    fp.ws = ws;
    fp.cK = (const double*)ctx.upload(st, 61, cK.data(), sizeof(double) * cK.size());
    fp.qK = q_coeffs ? fp.cK + (size_t)m * m * (1 + fp.nof) : nullptr;
    SymParams sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.d = d;
    sp.r = r;
    sp.T = T;
    sp.scale = 1.0 / (double)N;
    for (int a = 0; a < 3; ++a) {
        sp.n[a] = a < d ? dims[a] : 1;
        sp.sdim[a] = sp.n[a];
    }
    sp.hcount = dims[d - 1];
    for (int a = 0; a < d; ++a) sp.eph[a] = ctx.phase_table(dims[a]);

    const int64_t esz = f64 ? 8 : 4;
    timed(st, "widen", f64, m * N * (esz + (int64_t)csz), [&] { return launch_widen(grid, ws, m * N, f64, st); });
    for (int a = 0; a < d; ++a) {
        int64_t outer = m, inner = 1;
        for (int b = 0; b < a; ++b) outer *= dims[b];
        for (int b = a + 1; b < d; ++b) inner *= dims[b];
        axis_transform(ws, tmp, outer, dims[a], inner, f64, false, &sp, a, st);
    }
    timed(st, "fields_symbol_full", f64, 2 * m * N * (int64_t)csz,
          [&] { return launch_fields_symbol(fp, sp, f64, st); });
    for (int a = d - 1; a >= 0; --a) {
        int64_t outer = m, inner = 1;
        for (int b = 0; b < a; ++b) outer *= dims[b];
        for (int b = a + 1; b < d; ++b) inner *= dims[b];
        axis_transform(ws, tmp, outer, dims[a], inner, f64, true, nullptr, a, st);
    }
    timed(st, "narrow", f64, m * N * (esz + (int64_t)csz), [&] { return launch_narrow(ws, grid, m * N, f64, st); });
}

}  // namespace sfft
