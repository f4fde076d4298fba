// Per-device runtime: twiddle / phase tables, plan cache, per-stream workspace,
// error strings and optional per-kernel HIP-event timing.
#include "sfft_runtime.h"

#include <cmath>
#include <cstring>
#include <sstream>

#include "sfft_kernels.h"

namespace sfft {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }
const char* last_error_cstr() { return g_last_error.c_str(); }

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error(-4, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- context ----

DevCtx& device_ctx() {
    static std::mutex m;
    static std::map<int, std::unique_ptr<DevCtx>> ctxs;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> g(m);
    auto& p = ctxs[dev];
    if (!p) {
        p.reset(new DevCtx());
        p->device = dev;
        int lds = 0;
        check_hip(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                  "hipDeviceGetAttribute(max shared memory)");
        p->lds_max = (size_t)lds;
        // tables are generated on a private stream and waited for on the host, so
        // building a plan never synchronises the whole device
        check_hip(hipStreamCreateWithFlags(&p->tstream, hipStreamNonBlocking), "hipStreamCreate(tables)");
        // Opt the FFT kernels in to the device's full LDS; the kernels with static
        // LDS leave room for it.  Not every runtime requires the opt-in, so a
        // refusal is not fatal: launches that exceed the limit fail loudly.
        if (set_kernel_lds_limits(p->lds_max - 8192) != hipSuccess) (void)hipGetLastError();
    }
    return *p;
}

std::pair<double2*, float2*> DevCtx::table(const TwiddleReq& r) {
    auto it = tw.find(r);
    if (it != tw.end()) return it->second;
    double2* d64 = nullptr;
    float2* d32 = nullptr;
    check_hip(hipMalloc(&d64, sizeof(double2) * r.count), "hipMalloc(twiddles)");
    check_hip(hipMalloc(&d32, sizeof(float2) * r.count), "hipMalloc(twiddles)");
    check_hip(launch_twiddle_table(d64, d32, r.N, r.count, r.mult, tstream), "twiddle table");
    check_hip(hipStreamSynchronize(tstream), "twiddle table");
    tw[r] = {d64, d32};
    return {d64, d32};
}

const double2* DevCtx::phase_table(int64_t n) {
    std::lock_guard<std::mutex> g(mu);
    auto it = eph.find(n);
    if (it != eph.end()) return it->second;
    double2* E = nullptr;
    check_hip(hipMalloc(&E, sizeof(double2) * n), "hipMalloc(phase table)");
    check_hip(launch_phase_table(E, n, tstream), "phase table");
    check_hip(hipStreamSynchronize(tstream), "phase table");
    eph[n] = E;
    return E;
}

std::shared_ptr<Plan> DevCtx::plan(int d, const int64_t* dims, int64_t B, bool f64, bool unfused) {
    std::ostringstream key;
    key << d << ":" << B << ":" << f64 << ":" << tunables().col_max << ":" << tunables().no_fast << ":" << tunables().mixed_row_q << ":" << tunables().mixed_col_q << ":" << unfused
        << ":" << tune_db().gen.load();
    for (int a = 0; a < d; ++a) key << ":" << dims[a];
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = plans.find(key.str());
        if (it != plans.end()) return it->second;
    }
    auto p = std::make_shared<Plan>();
    std::string why;
    const int rc = build_schedule(d, dims, B, f64, &p->s, &why, unfused);
    if (rc) throw Error(rc == -1 ? -1 : -2, why);
    for (auto& pp : p->s.passes) {
        if (pp.lds_bytes > lds_max)
            throw Error(-2, "pass needs " + std::to_string(pp.lds_bytes) + " bytes of LDS");
    }
    for (int a = 0; a < d; ++a) p->s.sym.eph[a] = phase_table(dims[a]);
    {
        std::lock_guard<std::mutex> g(mu);
        bind_passes(*p, f64);
        plans[key.str()] = p;
    }
    return p;
}

std::shared_ptr<Plan> DevCtx::axis_plan(int64_t outer, int64_t n, int64_t inner, bool f64, bool inverse) {
    std::ostringstream key;
    key << "axis:" << outer << ":" << n << ":" << inner << ":" << f64 << ":" << inverse << ":"
        << tunables().col_max << ":" << tunables().no_fast << ":" << tunables().mixed_row_q << ":" << tunables().mixed_col_q << ":" << tune_db().gen.load();
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = plans.find(key.str());
        if (it != plans.end()) return it->second;
    }
    auto p = std::make_shared<Plan>();
    std::string why;
    std::vector<int64_t> levels;
    const int rc = axis_schedule(outer, n, inner, f64, inverse, &p->s.passes, &levels, &why);
    if (rc) throw Error(rc == -1 ? -1 : -2, why);
    for (auto& pp : p->s.passes) {
        if (pp.lds_bytes > lds_max)
            throw Error(-2, "pass needs " + std::to_string(pp.lds_bytes) + " bytes of LDS");
    }
    p->s.f64 = f64;
    p->s.fused = false;
    p->s.sym.nlev[0] = (int)levels.size();
    for (size_t i = 0; i < levels.size() && i < 3; ++i) p->s.sym.sub[0][i] = levels[i];
    p->s.spec_elems = outer * n * inner;
    {
        std::lock_guard<std::mutex> g(mu);
        bind_passes(*p, f64);
        plans[key.str()] = p;
    }
    return p;
}

// Bind the table pointers of every pass (caller holds mu).
void DevCtx::bind_passes(Plan& plan, bool f64) {
    auto* p = &plan;
    {
        for (auto& pp : p->s.passes) {
            PassDesc pd = pp.pd;
            auto st = table(pp.stage_tab);
            pd.st_tab = f64 ? (const void*)st.first : (const void*)st.second;
            if (pp.has_fast) {
                auto lo = table(pp.f_lo);
                auto hi = table(pp.f_hi);
                pd.f_lo = f64 ? (const void*)lo.first : (const void*)lo.second;
                pd.f_hi = f64 ? (const void*)hi.first : (const void*)hi.second;
            }
            if (pp.has_half) {
                auto lo = table(pp.h_lo);
                auto hi = table(pp.h_hi);
                pd.h_lo = f64 ? (const void*)lo.first : (const void*)lo.second;
                pd.h_hi = f64 ? (const void*)hi.first : (const void*)hi.second;
            }
            if (pp.has_tw) {
                auto lo = table(pp.tw_lo);
                auto hi = table(pp.tw_hi);
                pd.tw_lo = f64 ? (const void*)lo.first : (const void*)lo.second;
                pd.tw_hi = f64 ? (const void*)hi.first : (const void*)hi.second;
            }
            p->pd.push_back(pd);
            p->lds.push_back(pp.lds_bytes);
        }
    }
}

void* DevCtx::workspace(hipStream_t st, size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    auto& w = ws[st];
    if (bytes == 0) return w.first;
    if (w.second < bytes) {
        if (w.first) {
            check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize(workspace growth)");
            check_hip(hipFree(w.first), "hipFree(workspace)");
            ++epoch;
            w.first = nullptr;
            w.second = 0;
        }
        hipError_t e = hipMalloc(&w.first, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            w.first = nullptr;
            throw Error(-3, "workspace of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
        }
        w.second = bytes;
    }
    return w.first;
}

void* DevCtx::upload(hipStream_t st, int slot, const void* host, size_t bytes) {
    void* dev = scratch(st, slot, bytes);
    upload_to(st, dev, host, bytes);
    return dev;
}

void DevCtx::upload_to(hipStream_t st, void* dev, const void* host, size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    auto& sg = staging[st];
    if (!sg.second) check_hip(hipEventCreateWithFlags(&sg.second, hipEventDisableTiming), "hipEventCreate(staging)");
    // the previous upload through this buffer must have been read by the device
    check_hip(hipEventSynchronize(sg.second), "hipEventSynchronize(staging)");
    if (sg.first.second < bytes) {
        if (sg.first.first) check_hip(hipHostFree(sg.first.first), "hipHostFree(staging)");
        sg.first.first = nullptr;
        sg.first.second = 0;
        check_hip(hipHostMalloc(&sg.first.first, bytes), "hipHostMalloc(staging)");
        sg.first.second = bytes;
    }
    std::memcpy(sg.first.first, host, bytes);
    check_hip(hipMemcpyAsync(dev, sg.first.first, bytes, hipMemcpyHostToDevice, st), "upload");
    check_hip(hipEventRecord(sg.second, st), "hipEventRecord(staging)");
}

hipStream_t DevCtx::side_stream(hipStream_t st, int i) {
    std::lock_guard<std::mutex> g(mu);
    auto& s = sides[{st, i}];
    if (!s) check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags(side)");
    return s;
}

hipEvent_t DevCtx::side_event(hipStream_t st, int i) {
    std::lock_guard<std::mutex> g(mu);
    auto& e = side_events[{st, i}];
    if (!e) check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags(side)");
    return e;
}

void* DevCtx::scratch(hipStream_t st, int slot, size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    auto& w = extra[{st, slot}];
    if (w.second < bytes) {
        if (w.first) {
            check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize(scratch growth)");
            check_hip(hipFree(w.first), "hipFree(scratch)");
            ++epoch;
            w.first = nullptr;
            w.second = 0;
        }
        hipError_t e = hipMalloc(&w.first, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            w.first = nullptr;
            throw Error(-3, "scratch of " + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
        }
        w.second = bytes;
    }
    return w.first;
}

// ---------------------------------------------------------------- symbol -----

void fill_symbol(SymParams& sp, const double* coeffs, int r, int d, int64_t T, double scale, double* cout) {
    int nc = 1;
    for (int a = 0; a < d; ++a) nc *= 2 * r + 1;
    if (!cout) {
        if (nc > kMaxCoef) throw Error(-2, "stencil has more coefficients than the fused passes hold");
        cout = sp.c;
    }
    sp.r = r;
    sp.ncoef = nc;
    sp.T = T;
    // sum(c) carried as s + comp (Neumaier's compensated sum): lambda(0) exactly
    // to double-double precision.
    double s = 0.0, comp = 0.0;
    bool nonneg = true, nonpos = true;
    for (int i = 0; i < nc; ++i) {
        const double t = s + coeffs[i];
        if (std::fabs(s) >= std::fabs(coeffs[i])) comp += (s - t) + coeffs[i];
        else comp += (coeffs[i] - t) + s;
        s = t;
        nonneg = nonneg && coeffs[i] >= 0.0;
        nonpos = nonpos && coeffs[i] <= 0.0;
    }
    // point symmetric coefficients (c[o] == c[-o]) give a real symbol
    int sym = 1;
    for (int i = 0; i < nc; ++i)
        if (coeffs[i] != coeffs[nc - 1 - i]) { sym = 0; break; }
    sp.real_sym = sym;
    if ((nonneg || nonpos) && s != 0.0) {
        // One sign: |lambda(k)| <= |sum c| = |lambda(0)| for every k.  Solve with
        // c / lambda(0), whose symbol is exactly 1 at k = 0 (so 1 - sum = 0), and
        // multiply the result by lambda(0)^T, formed here in extended precision as
        // exp(T log|lambda(0)|) with log(s + comp) = log s + log1p(comp / s).
        const long double rho = (long double)s + (long double)comp;
        for (int i = 0; i < nc; ++i) cout[i] = (double)((long double)coeffs[i] / rho);
        sp.one_minus_sum = 0.0;
        const long double as = std::fabs((long double)s);
        const long double lg = std::log(as) + std::log1p((long double)comp / (long double)s);
        long double p = std::exp((long double)T * lg);
        if (s < 0.0 && (T & 1)) p = -p;
        sp.scale = (double)((long double)scale * p);
        sp.switching = 0;
    } else {
        // Mixed signs (or sum 0): no bound on |lambda| from lambda(0); every mode
        // takes the switching power.  1 - sum(c): when the sum is close to 1,
        // 1 - s is exact and only the final subtraction rounds.
        for (int i = 0; i < nc; ++i) cout[i] = coeffs[i];
        sp.one_minus_sum = (1.0 - s) - comp;
        sp.scale = scale;
        sp.switching = 1;
    }
}

RealView dense_view(void* ptr, int d, const int64_t* dims) {
    RealView v;
    std::memset(&v, 0, sizeof(v));
    v.ptr = ptr;
    int64_t s = 1;
    for (int a = d - 1; a >= 0; --a) {
        v.stride[a] = s;
        v.ext[a] = dims[a];
        s *= dims[a];
    }
    v.boff = s;
    return v;
}

void build_symbol_columns(SymParams& sym, void* tab, bool f64, hipStream_t st) {
    int64_t ncol = 1;
    for (int a = 1; a < sym.d; ++a) ncol *= sym.sdim[a];
    sym.coltab = tab;
    sym.ncol = ncol;
    hipEvent_t ev = nullptr;
    const bool prof = profiling();
    if (prof) profile_launch_begin(st, &ev);
    check_hip(launch_symbol_columns(tab, sym, ncol, st), "symbol column launch");
    if (prof) profile_launch_end(st, ev, f64 ? "symbol_columns_f64" : "symbol_columns_f32", 0);
}

void run_plan(const Plan& p, void* ws, const RealView& in, const RealView& out, const KeepRule& keep,
              const SymParams& sym_in, hipStream_t st, size_t pass_begin, size_t pass_end) {
    const bool f64 = p.s.f64;
    SymParams sym = sym_in;
    if (p.s.fused && sym.d >= 2 && !sym.coltab) {
        // per-column part of the symbol (axes 1..d-1), once per solve
        int64_t ncol = 1;
        for (int a = 1; a < sym.d; ++a) ncol *= sym.sdim[a];
        build_symbol_columns(sym, device_ctx().scratch(st, 50, (size_t)ncol * symbol_column_bytes()), f64, st);
    }
    pass_end = std::min(pass_end, p.pd.size());
    for (size_t i = pass_begin; i < pass_end; ++i) {
        PassDesc pd = p.pd[i];
        pd.buf = ws;
        if (pd.in_real) pd.rv = in;
        if (pd.out_real) {
            pd.rvo = out;
            pd.keep = keep;
        }
        hipEvent_t ev = nullptr;
        const bool prof = profiling();
        if (prof) profile_launch_begin(st, &ev);
        check_hip(launch_pass(pd, sym, f64, p.lds[i], st), "FFT pass launch");
        if (prof) profile_launch_end(st, ev, p.s.passes[i].name + (f64 ? "_f64" : "_f32"), p.s.passes[i].model_bytes);
    }
}

// ---------------------------------------------------------------- profiling --

namespace {
struct ProfRec {
    hipEvent_t a, b;
    std::string name;
    int64_t bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
}  // namespace

bool g_prof_paused = false;
bool profiling() { return g_prof_on && !g_prof_paused; }
void profile_pause(bool p) { g_prof_paused = p; }

void profile_launch_begin(hipStream_t st, hipEvent_t* ev) {
    check_hip(hipEventCreate(ev), "hipEventCreate");
    check_hip(hipEventRecord(*ev, st), "hipEventRecord");
}

void profile_launch_end(hipStream_t st, hipEvent_t ev0, const std::string& name, int64_t bytes) {
    hipEvent_t ev1;
    check_hip(hipEventCreate(&ev1), "hipEventCreate");
    check_hip(hipEventRecord(ev1, st), "hipEventRecord");
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back({ev0, ev1, name, bytes});
}

void profile_enable(bool on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto& r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    g_prof_on = on;
}

std::string profile_json() {
    std::lock_guard<std::mutex> g(g_prof_mu);
    struct Acc {
        int64_t n = 0;
        double ms = 0;
        int64_t bytes = 0;
    };
    std::map<std::string, Acc> acc;
    for (auto& r : g_prof) {
        check_hip(hipEventSynchronize(r.b), "hipEventSynchronize");
        float ms = 0.f;
        check_hip(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
        auto& a = acc[r.name];
        a.n += 1;
        a.ms += ms;
        a.bytes += r.bytes;
    }
    std::ostringstream o;
    o.precision(9);
    o << "{\"kernels\": {";
    bool first = true;
    for (auto& kv : acc) {
        o << (first ? "" : ", ") << "\"" << kv.first << "\": {\"launches\": " << kv.second.n
          << ", \"ms\": " << kv.second.ms << ", \"bytes\": " << kv.second.bytes << "}";
        first = false;
    }
    o << "}}";
    return o.str();
}

}  // namespace sfft
