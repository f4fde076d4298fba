// C ABI entry points (declared in include/stencil_fft.h).
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/stencil_fft.h"
#include "sfft_fields.h"
#include "sfft_general.h"
#include "sfft_kernels.h"
#include "sfft_runtime.h"
#include "sfft_solvers.h"
#include "sfft_verify.h"

namespace sfft {
const char* last_error_cstr();
void profile_enable(bool on);
std::string profile_json();
void solve_aperiodic_cached(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r, int64_t T,
                            int bc, hipStream_t st);
void solve_periodic_noalloc(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r,
                            int64_t T, hipStream_t st);
}  // namespace sfft

using namespace sfft;

namespace {

template <typename F>
int guarded(F&& f) {
    clear_last_error();
    try {
        f();
        return SFFT_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return SFFT_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return SFFT_EINVAL;
    }
}

void validate(const void* ptr, int dtype, int ndim, const int64_t* dims, const double* coeffs, int radius,
              int64_t T, int max_radius = kMaxR) {
    if (!ptr) throw Error(SFFT_EINVAL, "grid pointer is null");
    if (dtype != SFFT_F32 && dtype != SFFT_F64) throw Error(SFFT_EINVAL, "unknown dtype");
    if (ndim < 1 || ndim > 3) throw Error(SFFT_EINVAL, "ndim must be 1, 2 or 3");
    if (!dims) throw Error(SFFT_EINVAL, "dims pointer is null");
    for (int a = 0; a < ndim; ++a)
        if (dims[a] < 1) throw Error(SFFT_EINVAL, "extents must be >= 1");
    if (radius < 0) throw Error(SFFT_EINVAL, "radius must be >= 0");
    if (radius > max_radius)
        throw Error(SFFT_EUNSUPPORTED, "radius above " + std::to_string(max_radius) + " is not supported here");
    if (T < 0) throw Error(SFFT_EINVAL, "T must be >= 0");
    if (!coeffs) throw Error(SFFT_EINVAL, "coeffs pointer is null");
    int nc = 1;
    for (int a = 0; a < ndim; ++a) nc *= 2 * radius + 1;
    for (int i = 0; i < nc; ++i)
        if (!std::isfinite(coeffs[i])) throw Error(SFFT_EINVAL, "coefficient " + std::to_string(i) + " is not finite");
}

}  // namespace

namespace sfft {

bool all_7smooth(int ndim, const int64_t* dims) {
    for (int a = 0; a < ndim; ++a)
        if (!is_7smooth(dims[a])) return false;
    return true;
}

void validate_bc(int bc, int ndim, const int64_t* dims, int radius) {
    if (bc != SFFT_BC_FIXED && bc != SFFT_BC_REFLECT) throw Error(SFFT_EINVAL, "unknown boundary condition");
    if (bc == SFFT_BC_REFLECT)
        for (int a = 0; a < ndim; ++a)
            if (dims[a] < radius)
                throw Error(SFFT_EINVAL, "a reflecting boundary needs interior extents >= radius");
}

int guarded_call(const std::function<void()>& f) { return guarded(f); }

// Periodic solve of B dense grids of `dims` stored back to back.
void solve_periodic_dense(void* grid, bool f64, int d, const int64_t* dims, int64_t B, const double* coeffs, int r,
                          int64_t T, hipStream_t st) {
    DevCtx& ctx = device_ctx();
    auto plan = ctx.plan(d, dims, B, f64);
    void* ws = ctx.workspace(st, (size_t)plan->s.spec_elems * (f64 ? 16 : 8));
    SymParams sp = plan->s.sym;
    double N = 1.0;
    for (int a = 0; a < d; ++a) N *= (double)dims[a];
    fill_symbol(sp, coeffs, r, d, T, 1.0 / N);
    RealView v = dense_view(grid, d, dims);
    KeepRule keep;
    std::memset(&keep, 0, sizeof(keep));
    run_plan(*plan, ws, v, v, keep, sp, st);
}

// Periodic solve of a stencil of any radius up to kMaxGeneralR (7-smooth extents;
// a 1-D extent must fit one row): forward passes, the general symbol kernel on
// the half spectrum, inverse passes.
// With `pool`, the workspace and the coefficients live at pool (at least
// periodic_general_footprint bytes) instead of the context's per-stream buffers.
size_t periodic_general_footprint(bool f64, int d, const int64_t* dims, int r) {
    Schedule s;
    std::string why;
    const int rc = build_schedule(d, dims, 1, f64, &s, &why, true);
    if (rc) throw Error(rc == -1 ? SFFT_EINVAL : SFFT_EUNSUPPORTED, why);
    int nc = 1;
    for (int a = 0; a < d; ++a) nc *= 2 * r + 1;
    return ((size_t)s.spec_elems * (f64 ? 16 : 8) + 255) / 256 * 256 + sizeof(double) * (size_t)nc;
}

void solve_periodic_general(void* grid, bool f64, int d, const int64_t* dims, const double* coeffs, int r,
                            int64_t T, hipStream_t st, void* pool) {
    DevCtx& ctx = device_ctx();
    auto plan = ctx.plan(d, dims, 1, f64, true);
    const size_t wsb = (size_t)plan->s.spec_elems * (f64 ? 16 : 8);
    void* ws = pool ? pool : ctx.workspace(st, wsb);
    SymParams sp = plan->s.sym;
    double N = 1.0;
    int nc = 1;
    for (int a = 0; a < d; ++a) {
        N *= (double)dims[a];
        nc *= 2 * r + 1;
    }
    std::vector<double> cn((size_t)nc);
    fill_symbol(sp, coeffs, r, d, T, 1.0 / N, cn.data());
    sp.d = d;
    GeneralParams gp;
    gp.ws = ws;
    gp.pitch = plan->s.sym.sdim[d - 1];
    gp.rows = plan->s.spec_elems / gp.pitch;
    if (pool) {
        void* cdev = (char*)pool + (wsb + 255) / 256 * 256;
        ctx.upload_to(st, cdev, cn.data(), sizeof(double) * cn.size());
        gp.c = (const double*)cdev;
    } else {
        gp.c = (const double*)ctx.upload(st, 61, cn.data(), sizeof(double) * cn.size());
    }
    gp.r = r;
    RealView v = dense_view(grid, d, dims);
    KeepRule keep;
    std::memset(&keep, 0, sizeof(keep));
    const int at = plan->s.sym_at;
    run_plan(*plan, ws, v, v, keep, sp, st, 0, (size_t)at);
    hipEvent_t ev = nullptr;
    const bool prof = profiling();
    if (prof) profile_launch_begin(st, &ev);
    check_hip(launch_symbol_general(gp, sp, f64, st), "general symbol launch");
    if (prof)
        profile_launch_end(st, ev, f64 ? "general_symbol_f64" : "general_symbol_f32",
                           2 * gp.rows * sp.hcount * (f64 ? 16 : 8));
    run_plan(*plan, ws, v, v, keep, sp, st, (size_t)at);
}

// m coupled periodic fields (field-major grid): forward transforms of all fields
// as one batch, the symbol-matrix power per mode, inverse transforms.
// q_coeffs (m = 1 only): the implicit part Q of Q a_{t+1} = S a_t, S = coeffs.
// The symbol-matrix constants of m coupled fields (and of an implicit stencil's Q):
// K_ij = delta_ij - sum_o c_ij[o] (compensated sum), then the coefficients, then
// (implicit) 1 - sum q and q.  Sets fp.m, nof, real_sym, implicit, qzero.
std::vector<double> field_constants(int m, int d, const double* coeffs, int r, const double* q_coeffs,
                                    FieldParams* fp) {
    int nof = 1;
    for (int a = 0; a < d; ++a) nof *= 2 * r + 1;
    // K_ij = delta_ij - sum_o c_ij[o] (compensated sum), then the coefficients
    std::vector<double> cK((size_t)m * m * (1 + nof));
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            const double* c = coeffs + ((size_t)i * m + j) * nof;
            double sum = i == j ? 1.0 : 0.0, comp = 0.0;
            for (int o = 0; o < nof; ++o) {
                const double x = -c[o], t = sum + x;
                comp += std::fabs(sum) >= std::fabs(x) ? (sum - t) + x : (x - t) + sum;
                sum = t;
            }
            cK[(size_t)i * m + j] = sum + comp;
        }
    std::memcpy(cK.data() + (size_t)m * m, coeffs, sizeof(double) * (size_t)m * m * nof);
    double qabs = 0.0;
    if (q_coeffs) {
        // 1 - sum q (compensated) and q, after S's block
        double sum = 1.0, comp = 0.0;
        for (int o = 0; o < nof; ++o) {
            const double x = -q_coeffs[o], t = sum + x;
            comp += std::fabs(sum) >= std::fabs(x) ? (sum - t) + x : (x - t) + sum;
            sum = t;
            qabs += std::fabs(q_coeffs[o]);
        }
        cK.push_back(sum + comp);
        cK.insert(cK.end(), q_coeffs, q_coeffs + nof);
    }
    std::memset(fp, 0, sizeof(*fp));
    fp->m = m;
    fp->nof = nof;
    fp->real_sym = q_coeffs ? 0 : 1;
    for (int b = 0; b < m * m; ++b)
        for (int o = 0; o < nof; ++o)
            if (coeffs[(size_t)b * nof + o] != coeffs[(size_t)b * nof + (nof - 1 - o)]) fp->real_sym = 0;
    fp->implicit = q_coeffs ? 1 : 0;
    // lambda_Q counts as zero below the rounding bound of its evaluation
    fp->qzero = 16.0 * 2.220446049250313e-16 * qabs;
    return cK;
}

void solve_periodic_fields(void* grid, bool f64, int m, int d, const int64_t* dims, const double* coeffs, int r,
                           int64_t T, hipStream_t st, const double* q_coeffs = nullptr) {
    DevCtx& ctx = device_ctx();
    auto plan = ctx.plan(d, dims, m, f64, true);
    void* ws = ctx.workspace(st, (size_t)plan->s.spec_elems * (f64 ? 16 : 8));
    FieldParams fp;
    const std::vector<double> cK = field_constants(m, d, coeffs, r, q_coeffs, &fp);
    const int nof = fp.nof;
    fp.fstride = plan->s.spec_elems / m;
    fp.pitch = plan->s.sym.sdim[d - 1];
    fp.rows = fp.fstride / fp.pitch;
    fp.ws = ws;
    fp.cK = (const double*)ctx.upload(st, 60, cK.data(), sizeof(double) * cK.size());
    fp.qK = q_coeffs ? fp.cK + (size_t)m * m * (1 + nof) : nullptr;
    SymParams sp = plan->s.sym;
    sp.d = d;
    sp.r = r;
    sp.T = T;
    double N = 1.0;
    for (int a = 0; a < d; ++a) N *= (double)dims[a];
    sp.scale = 1.0 / N;
    int64_t cells = 1;
    for (int a = 0; a < d; ++a) cells *= dims[a];
    RealView v = dense_view(grid, d, dims);
    v.boff = cells;
    KeepRule keep;
    std::memset(&keep, 0, sizeof(keep));
    const int at = plan->s.sym_at;
    run_plan(*plan, ws, v, v, keep, sp, st, 0, (size_t)at);
    hipEvent_t ev = nullptr;
    const bool prof = profiling();
    if (prof) profile_launch_begin(st, &ev);
    check_hip(launch_fields_symbol(fp, sp, f64, st), "fields symbol launch");
    if (prof)
        profile_launch_end(st, ev, f64 ? "fields_symbol_f64" : "fields_symbol_f32",
                           2 * (int64_t)m * fp.rows * plan->s.sym.hcount * (f64 ? 16 : 8));
    run_plan(*plan, ws, v, v, keep, sp, st, (size_t)at);
}

}  // namespace sfft

extern "C" {

const char* stencil_fft_version(void) { return "stencil_fft 0.1 (gfx950)"; }

const char* stencil_fft_last_error(void) { return last_error_cstr(); }

int stencil_fft_periodic(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims, const double* coeffs,
                         int radius, int64_t T, void* stream) {
    return guarded([&] {
        validate(grid, dtype, ndim, dims, coeffs, radius, T, kMaxGeneralR);
        bool smooth = true;
        for (int a = 0; a < ndim; ++a) {
            if (dims[a] > ((int64_t)1 << 30)) throw Error(SFFT_EUNSUPPORTED, "extents above 2^30 are not supported");
            smooth = smooth && is_7smooth(dims[a]);
        }
        if (radius > kMaxR && !smooth)
            throw Error(SFFT_EUNSUPPORTED, "radius above 2 needs 7-smooth extents");
        if (T == 0) return;
        if (radius > kMaxR)
            solve_periodic_general(grid, dtype == SFFT_F64, ndim, dims, coeffs, radius, T, (hipStream_t)stream,
                                   nullptr);
        else if (smooth)
            solve_periodic_dense(grid, dtype == SFFT_F64, ndim, dims, 1, coeffs, radius, T, (hipStream_t)stream);
        else
            solve_periodic_any(grid, dtype == SFFT_F64, ndim, dims, coeffs, radius, T, (hipStream_t)stream);
    });
}

int stencil_fft_periodic_noalloc(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims, const double* coeffs,
                                 int radius, int64_t T, void* stream) {
    return guarded([&] {
        validate(grid, dtype, ndim, dims, coeffs, radius, T);
        for (int a = 0; a < ndim; ++a)
            if (!is_7smooth(dims[a]))
                throw Error(SFFT_EUNSUPPORTED, "extent " + std::to_string(dims[a]) +
                                                   " has a prime factor above 7 (the no-allocation entry point "
                                                   "takes 7-smooth extents only)");
        if (T == 0) return;
        solve_periodic_noalloc(grid, dtype == SFFT_F64, ndim, dims, coeffs, radius, T, (hipStream_t)stream);
    });
}

int stencil_fft_periodic_fields(void* grid, sfft_dtype dtype, int nfields, int ndim, const int64_t* dims,
                                const double* coeffs, int radius, int64_t T, void* stream) {
    return guarded([&] {
        if (nfields < 1) throw Error(SFFT_EINVAL, "nfields must be >= 1");
        if (nfields > kMaxFields) throw Error(SFFT_EUNSUPPORTED, "more than 4 fields are not supported");
        validate(grid, dtype, ndim, dims, coeffs, radius, T);
        int nof = 1;
        for (int a = 0; a < ndim; ++a) nof *= 2 * radius + 1;
        for (int i = 0; i < nfields * nfields * nof; ++i)
            if (!std::isfinite(coeffs[i])) throw Error(SFFT_EINVAL, "coefficient " + std::to_string(i) + " is not finite");
        if (T == 0) return;
        if (!all_7smooth(ndim, dims))
            solve_fields_any(grid, dtype == SFFT_F64, nfields, ndim, dims, coeffs, radius, T, (hipStream_t)stream);
        else
            solve_periodic_fields(grid, dtype == SFFT_F64, nfields, ndim, dims, coeffs, radius, T, (hipStream_t)stream);
    });
}

int stencil_fft_periodic_implicit(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims,
                                  const double* q_coeffs, const double* s_coeffs, int radius, int64_t T,
                                  void* stream) {
    return guarded([&] {
        validate(grid, dtype, ndim, dims, s_coeffs, radius, T);
        validate(grid, dtype, ndim, dims, q_coeffs, radius, T);
        if (T == 0) return;
        if (!all_7smooth(ndim, dims))
            solve_fields_any(grid, dtype == SFFT_F64, 1, ndim, dims, s_coeffs, radius, T, (hipStream_t)stream,
                             q_coeffs);
        else
            solve_periodic_fields(grid, dtype == SFFT_F64, 1, ndim, dims, s_coeffs, radius, T, (hipStream_t)stream,
                                  q_coeffs);
    });
}

int stencil_fft_aperiodic(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims, const double* coeffs,
                          int radius, int64_t T, void* stream) {
    return stencil_fft_aperiodic_bc(grid, dtype, ndim, dims, coeffs, radius, T, SFFT_BC_FIXED, stream);
}

int stencil_fft_aperiodic_bc(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims, const double* coeffs,
                             int radius, int64_t T, int bc, void* stream) {
    return guarded([&] {
        validate(grid, dtype, ndim, dims, coeffs, radius, T);
        validate_bc(bc, ndim, dims, radius);
        if (T == 0) return;
        solve_aperiodic_cached(grid, dtype == SFFT_F64, ndim, dims, coeffs, radius, T, bc, (hipStream_t)stream);
    });
}

int stencil_fft_verify(sfft_dtype dtype, int ndim, const int64_t* dims, const double* coeffs, int radius, int64_t T,
                       int kind, char* report, int64_t cap) {
    Verifier v;
    const int rc = guarded([&] {
        void* const fake = (void*)((uintptr_t)1 << 44);
        if (kind < 0 || kind > 2) throw Error(SFFT_EINVAL, "kind must be 0, 1 or 2");
        validate(fake, dtype, ndim, dims, coeffs, radius, T, kind ? kMaxR : kMaxGeneralR);
        const bool f64 = dtype == SFFT_F64;
        if (kind) {
            validate_bc(kind - 1, ndim, dims, radius);
            verify_aperiodic(f64, ndim, dims, coeffs, radius, T, kind - 1, &v);
            return;
        }
        for (int a = 0; a < ndim; ++a)
            if (!is_7smooth(dims[a]))
                throw Error(SFFT_EUNSUPPORTED, "verification covers 7-smooth periodic extents");
        Schedule s;
        std::string why;
        const int brc = build_schedule(ndim, dims, 1, f64, &s, &why, radius > kMaxR);
        if (brc) throw Error(brc == -1 ? SFFT_EINVAL : SFFT_EUNSUPPORTED, why);
        int64_t cells = 1, ncol = 1;
        for (int a = 0; a < ndim; ++a) cells *= dims[a];
        for (int a = 1; a < ndim; ++a) ncol *= s.sym.sdim[a];
        void* ws = (void*)((uintptr_t)1 << 40);
        void* coltab = (void*)((uintptr_t)1 << 42);
        v.add(fake, (size_t)cells * (f64 ? 8 : 4), "grid");
        v.add(ws, (size_t)s.spec_elems * (f64 ? 16 : 8), "spectrum");
        v.add(coltab, (size_t)ncol * symbol_column_bytes(), "symbol columns");
        const RealView view = dense_view(fake, ndim, dims);
        v.schedule(s, ws, view, view, ndim >= 2 ? coltab : nullptr, ncol, "periodic");
    });
    if (rc != SFFT_OK) return rc;
    std::string js = "{\"checked\": " + std::to_string(v.checked) + ", \"failures\": " + std::to_string(v.nerr) +
                     ", \"errors\": [";
    for (size_t i = 0; i < v.errors.size(); ++i) {
        std::string e;
        for (char c : v.errors[i]) e += (c == '"' || c == '\\') ? ' ' : c;
        js += (i ? ", \"" : "\"") + e + "\"";
    }
    js += "]}";
    if (report && cap > 0) {
        const size_t n = std::min<size_t>((size_t)cap - 1, js.size());
        std::memcpy(report, js.data(), n);
        report[n] = 0;
    }
    return (int)std::min<int64_t>(v.nerr, 1 << 30);
}

int stencil_fft_symbol_power(double* out, int ndim, const int64_t* dims, const double* coeffs, int radius,
                             int64_t T, void* stream) {
    return guarded([&] {
        validate(out, SFFT_F64, ndim, dims, coeffs, radius, T);
        DevCtx& ctx = device_ctx();
        SymParams sp;
        std::memset(&sp, 0, sizeof(sp));
        sp.d = ndim;
        int64_t total = 1;
        for (int a = 0; a < 3; ++a) {
            sp.n[a] = a < ndim ? dims[a] : 1;
            sp.nlev[a] = 1;
            sp.sub[a][0] = sp.n[a];
            sp.sdim[a] = sp.n[a];
        }
        for (int a = 0; a < ndim; ++a) {
            total *= dims[a];
            sp.eph[a] = ctx.phase_table(dims[a]);
        }
        fill_symbol(sp, coeffs, radius, ndim, T, 1.0);
        check_hip(launch_symbol_power((double2*)out, sp, total, (hipStream_t)stream), "symbol power launch");
    });
}

int stencil_fft_set_option(const char* name, int64_t value) {
    return guarded([&] {
        if (!name) throw Error(SFFT_EINVAL, "option name is null");
        const std::string n(name);
        if (n == "col_max") {
            if (value != 0 && (value < 16 || value > 1024 || (value & (value - 1))))
                throw Error(SFFT_EINVAL, "col_max must be 0 or a power of two in 16..1024");
            tunables().col_max = (int)value;
        } else if (n == "generic_kernels") {
            if (value != 0 && value != 1) throw Error(SFFT_EINVAL, "generic_kernels must be 0 or 1");
            tunables().no_fast = (int)value;
        } else if (n == "aperiodic_graphs") {
            if (value != 0 && value != 1) throw Error(SFFT_EINVAL, "aperiodic_graphs must be 0 or 1");
            tunables().aperiodic_graphs = (int)value;
        } else if (n == "mixed_row_q" || n == "mixed_col_q") {
            if (value != 0 && value != 5 && value != 10 && value != 12 && value != 20 && value != 25)
                throw Error(SFFT_EINVAL, n + " must be 0, 5, 10, 12, 20 or 25");
            (n == "mixed_row_q" ? tunables().mixed_row_q : tunables().mixed_col_q) = (int)value;
        } else if (n == "aperiodic_cutoff") {
            if (value < 0 || value > (1 << 20)) throw Error(SFFT_EINVAL, "aperiodic_cutoff out of range");
            tunables().aperiodic_cutoff = (int)value;
        } else {
            throw Error(SFFT_EINVAL, "unknown option '" + n + "'");
        }
    });
}

int stencil_fft_profile(int enable) {
    return guarded([&] { profile_enable(enable != 0); });
}

int stencil_fft_profile_read(char* buf, int64_t cap) {
    std::string s;
    const int rc = guarded([&] {
        if (!buf || cap < 1) throw Error(SFFT_EINVAL, "buffer is null or empty");
        s = profile_json();
    });
    if (rc) return rc;
    const int64_t n = std::min<int64_t>((int64_t)s.size(), cap - 1);
    std::memcpy(buf, s.data(), (size_t)n);
    buf[n] = 0;
    return (int)n;
}

int stencil_fft_plan_describe(int ndim, const int64_t* dims, sfft_dtype dtype, char* buf, int64_t cap) {
    std::string s;
    const int rc = guarded([&] {
        if (!buf || cap < 1 || !dims) throw Error(SFFT_EINVAL, "null argument");
        if (dtype != SFFT_F32 && dtype != SFFT_F64) throw Error(SFFT_EINVAL, "unknown dtype");
        Schedule sch;
        std::string why;
        const int r = build_schedule(ndim, dims, 1, dtype == SFFT_F64, &sch, &why);
        if (r) throw Error(r == -1 ? SFFT_EINVAL : SFFT_EUNSUPPORTED, why);
        s = describe_schedule(sch);
    });
    if (rc) return rc;
    if ((int64_t)s.size() >= cap) {
        set_last_error("buffer too small");
        return SFFT_EINVAL;
    }
    std::memcpy(buf, s.data(), s.size() + 1);
    return (int)s.size();
}

}  // extern "C"
