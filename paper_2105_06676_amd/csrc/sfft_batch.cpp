// Batched periodic solves: every problem of a batch keeps its own pass
// schedule, workspace and symbol; pass k of all problems runs in one launch per
// kernel variant (the problems' tiles are concatenated into a work list that the
// kernel searches by workgroup index), so a batch of same-shape problems costs
// as many launches as one problem, and uneven batches a few more.  Pass k + 1
// of a problem starts after pass k of every problem (stream order).  The whole
// program can be captured into a hipGraph and replayed.
#include "sfft_batch.h"

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "sfft_general.h"
#include "sfft_kernels.h"
#include "sfft_mixed.h"
#include "sfft_solvers.h"

namespace sfft {

namespace {
size_t align256(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

void validate_problem(const sfft_problem& p) {
    if (!p.grid) throw Error(SFFT_EINVAL, "grid pointer is null");
    if (p.dtype != SFFT_F32 && p.dtype != SFFT_F64) throw Error(SFFT_EINVAL, "unknown dtype");
    if (p.ndim < 1 || p.ndim > 3) throw Error(SFFT_EINVAL, "ndim must be 1, 2 or 3");
    for (int a = 0; a < p.ndim; ++a)
        if (p.dims[a] < 1) throw Error(SFFT_EINVAL, "extents must be >= 1");
    if (p.radius < 0) throw Error(SFFT_EINVAL, "radius must be >= 0");
    if (p.radius > (p.aperiodic ? kMaxR : kMaxGeneralR))
        throw Error(SFFT_EUNSUPPORTED, "radius " + std::to_string(p.radius) + " is not supported for this problem kind");
    if (p.T < 0) throw Error(SFFT_EINVAL, "T must be >= 0");
    if (p.aperiodic < 0 || p.aperiodic > 2) throw Error(SFFT_EINVAL, "aperiodic must be 0, 1 or 2");
    if (p.aperiodic) validate_bc(p.aperiodic - 1, p.ndim, p.dims, p.radius);
    if (!p.coeffs) throw Error(SFFT_EINVAL, "coeffs pointer is null");
    int nc = 1;
    for (int a = 0; a < p.ndim; ++a) nc *= 2 * p.radius + 1;
    for (int i = 0; i < nc; ++i)
        if (!std::isfinite(p.coeffs[i])) throw Error(SFFT_EINVAL, "coefficient " + std::to_string(i) + " is not finite");
    if (!p.aperiodic)
        for (int a = 0; a < p.ndim; ++a) {
            if (p.dims[a] > ((int64_t)1 << 30)) throw Error(SFFT_EUNSUPPORTED, "extents above 2^30 are not supported");
            if (p.radius > kMaxR && !is_7smooth(p.dims[a]))
                throw Error(SFFT_EUNSUPPORTED, "radius above 2 needs 7-smooth extents");
        }
}

bool batchable(const sfft_problem& p) {
    if (p.aperiodic || p.radius > kMaxR) return false;
    for (int a = 0; a < p.ndim; ++a)
        if (!is_7smooth(p.dims[a])) return false;
    return true;
}

static size_t col_table_bytes(const SymParams& sym) {
    if (sym.d < 2) return 0;
    int64_t ncol = 1;
    for (int a = 1; a < sym.d; ++a) ncol *= sym.sdim[a];
    return (size_t)ncol * symbol_column_bytes();
}

ProblemSize problem_size(const sfft_problem& p) {
    Schedule s;
    std::string why;
    const int rc = build_schedule(p.ndim, p.dims, 1, p.dtype == SFFT_F64, &s, &why);
    if (rc) throw Error(rc == -1 ? SFFT_EINVAL : SFFT_EUNSUPPORTED, why);
    ProblemSize ps;
    ps.ws_bytes = align256((size_t)s.spec_elems * (p.dtype == SFFT_F64 ? 16 : 8)) + align256(col_table_bytes(s.sym));
    ps.passes = s.passes.size();
    ps.model_bytes = s.model_bytes;
    return ps;
}

size_t problem_workspace_bytes(const sfft_problem& p) { return problem_size(p).ws_bytes; }

ProblemRun prepare_periodic(const sfft_problem& p) {
    ProblemRun r;
    const bool f64 = p.dtype == SFFT_F64;
    r.plan = device_ctx().plan(p.ndim, p.dims, 1, f64);
    r.view = dense_view(p.grid, p.ndim, p.dims);
    r.sp = r.plan->s.sym;
    double N = 1.0;
    for (int a = 0; a < p.ndim; ++a) N *= (double)p.dims[a];
    fill_symbol(r.sp, p.coeffs, p.radius, p.ndim, p.T, 1.0 / N);
    r.ws_bytes = align256((size_t)r.plan->s.spec_elems * (f64 ? 16 : 8));
    r.col_bytes = align256(col_table_bytes(r.sp));
    return r;
}

size_t batch_ws_bytes(const std::vector<ProblemRun>& runs) {
    size_t t = 0;
    for (auto& r : runs) t += r.ws_bytes + r.col_bytes;
    return std::max<size_t>(t, 256);
}

size_t batch_desc_bytes(const std::vector<ProblemRun>& runs) {
    size_t items = 0;
    for (auto& r : runs) items += r.plan->pd.size();
    return align256(sizeof(SymParams) * std::max<size_t>(1, runs.size())) + sizeof(BatchItem) * std::max<size_t>(1, items) + 256;
}

BatchProgram build_batch(std::vector<ProblemRun>& runs, const BatchMem& mem, const std::vector<char*>* bases) {
    BatchProgram prog;
    // workspace and column tables
    size_t off = 0;
    std::vector<void*> ws(runs.size(), nullptr);
    for (size_t i = 0; i < runs.size(); ++i) {
        char* base = bases ? (*bases)[i] : mem.ws + off;
        ws[i] = base;
        if (!bases) off += runs[i].ws_bytes + runs[i].col_bytes;
        if (runs[i].col_bytes) {
            void* tab = base + runs[i].ws_bytes;
            runs[i].sp.coltab = tab;
            int64_t ncol = 1;
            for (int a = 1; a < runs[i].sp.d; ++a) ncol *= runs[i].sp.sdim[a];
            runs[i].sp.ncol = ncol;
            prog.coltabs.push_back({(int)i, tab});
        }
    }
    if (!bases && off > mem.ws_cap) throw Error(SFFT_ENOMEM, "batch workspace too small");
    // descriptors: syms first, then the work lists
    const size_t sym_bytes = align256(sizeof(SymParams) * runs.size());
    prog.host_desc.assign(batch_desc_bytes(runs), 0);
    if (prog.host_desc.size() > mem.desc_cap) throw Error(SFFT_ENOMEM, "batch descriptor buffer too small");
    for (size_t i = 0; i < runs.size(); ++i)
        std::memcpy(prog.host_desc.data() + i * sizeof(SymParams), &runs[i].sp, sizeof(SymParams));
    prog.syms = (const SymParams*)mem.desc;
    size_t maxp = 0;
    for (auto& r : runs) maxp = std::max(maxp, r.plan->pd.size());
    size_t item_off = sym_bytes;
    for (size_t k = 0; k < maxp; ++k) {
        // group pass k of every problem by kernel variant
        std::map<std::tuple<int, int, int, int, int, int, int, int>, std::vector<int>> groups;
        for (size_t i = 0; i < runs.size(); ++i) {
            if (k >= runs[i].plan->pd.size()) continue;
            const PassDesc& pd = runs[i].plan->pd[k];
            const bool f64 = runs[i].plan->s.f64;
            // one launch per kernel variant (for the mixed-radix kernels: points per
            // thread and last-stage radix, and the workgroup size, since the tile
            // code assumes W * P threads)
            // (10-point rows with a radix-4 middle stage run a kernel variant of their own)
            int variant = mixed_radix_at(pd.mrad, pd.nst - 1);
            if (pd.mq == 10 && pd.kind == PASS_ROW)
                for (int s = 1; s + 1 < pd.nst; ++s)
                    if (mixed_radix_at(pd.mrad, s) == 4) variant += 100;
            auto key = pd.mq ? std::make_tuple(2, pd.kind, pd.mode, pd.fast_kind, pd.mq, variant, (int)f64, pd.mthreads)
                       : pd.fast ? std::make_tuple(1, pd.kind, pd.mode, pd.fast_kind, pd.logL, 0, (int)f64, 0)
                                 : std::make_tuple(0, pd.kind, 0, 0, 0, 0, (int)f64, 0);
            groups[key].push_back((int)i);
        }
        for (auto& g : groups) {
            BatchLaunch L;
            L.items = (const BatchItem*)(mem.desc + item_off);
            L.n = (int)g.second.size();
            L.tiles = 0;
            L.lds = 0;
            L.bytes = 0;
            for (int i : g.second) {
                const Plan& pl = *runs[i].plan;
                BatchItem it;
                std::memset(&it, 0, sizeof(it));
                it.pd = pl.pd[k];
                it.pd.buf = ws[i];
                if (it.pd.in_real) it.pd.rv = runs[i].view;
                if (it.pd.out_real) it.pd.rvo = runs[i].view;
                it.first = L.tiles;
                it.sym = i;
                std::memcpy(prog.host_desc.data() + item_off, &it, sizeof(it));
                item_off += sizeof(BatchItem);
                L.tiles += it.pd.ntiles;
                L.lds = std::max(L.lds, pl.lds[k]);
                L.bytes += pl.s.passes[k].model_bytes;
                L.proto = it.pd;
                L.f64 = pl.s.f64;
                L.name = "batch_" + pl.s.passes[k].name + (pl.s.f64 ? "_f64" : "_f32");
            }
            prog.launches.push_back(L);
        }
    }
    return prog;
}

namespace {
// Pinned host staging per stream for descriptor uploads; an event guards reuse.
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
};
std::mutex g_stage_mu;
std::map<hipStream_t, Staging> g_stage;
}  // namespace

void enqueue_batch(BatchProgram& prog, std::vector<ProblemRun>& runs, const BatchMem& mem, hipStream_t st,
                   bool upload) {
    if (upload) {
        std::lock_guard<std::mutex> g(g_stage_mu);
        Staging& s = g_stage[st];
        if (!s.ev) check_hip(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming), "hipEventCreate");
        check_hip(hipEventSynchronize(s.ev), "hipEventSynchronize(staging)");
        if (s.cap < prog.host_desc.size()) {
            if (s.host) check_hip(hipHostFree(s.host), "hipHostFree");
            s.host = nullptr;
            check_hip(hipHostMalloc(&s.host, prog.host_desc.size()), "hipHostMalloc(staging)");
            s.cap = prog.host_desc.size();
        }
        std::memcpy(s.host, prog.host_desc.data(), prog.host_desc.size());
        check_hip(hipMemcpyAsync(mem.desc, s.host, prog.host_desc.size(), hipMemcpyHostToDevice, st),
                  "descriptor upload");
        check_hip(hipEventRecord(s.ev, st), "hipEventRecord");
    }
    const bool prof = profiling();
    for (auto& ct : prog.coltabs) {
        const ProblemRun& r = runs[ct.first];
        check_hip(launch_symbol_columns(ct.second, r.sp, r.sp.ncol, st), "symbol column launch");
    }
    for (auto& L : prog.launches) {
        hipEvent_t ev = nullptr;
        if (prof) profile_launch_begin(st, &ev);
        check_hip(launch_pass_batch(L.proto, L.items, L.n, prog.syms, L.tiles, L.f64, L.lds, st), "batched pass launch");
        if (prof) profile_launch_end(st, ev, L.name, L.bytes);
    }
}

}  // namespace sfft

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace sfft;

namespace sfft {

int guarded_call(const std::function<void()>& f);
}  // namespace sfft

struct sfft_graph {
    int device = 0;
    std::vector<ProblemRun> runs;
    BatchMem mem;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int stencil_fft_batch(const sfft_problem* probs, int n, void* stream) {
    return guarded_call([&] {
        if (n < 0 || (n > 0 && !probs)) throw Error(SFFT_EINVAL, "invalid problem list");
        for (int i = 0; i < n; ++i) {
            try {
                validate_problem(probs[i]);
            } catch (const Error& e) {
                throw Error(e.code, "problem " + std::to_string(i) + ": " + e.what());
            }
        }
        hipStream_t st = (hipStream_t)stream;
        std::vector<ProblemRun> runs;
        for (int i = 0; i < n; ++i)
            if (batchable(probs[i]) && probs[i].T > 0) runs.push_back(prepare_periodic(probs[i]));
        if (!runs.empty()) {
            DevCtx& ctx = device_ctx();
            BatchMem mem;
            mem.ws_cap = batch_ws_bytes(runs);
            mem.ws = (char*)ctx.scratch(st, 60, mem.ws_cap);
            mem.desc_cap = batch_desc_bytes(runs);
            mem.desc = (char*)ctx.scratch(st, 62, mem.desc_cap);
            BatchProgram prog = build_batch(runs, mem);
            enqueue_batch(prog, runs, mem, st, true);
        }
        for (int i = 0; i < n; ++i) {
            const sfft_problem& p = probs[i];
            if (batchable(p) || p.T == 0) continue;
            const bool f64 = p.dtype == SFFT_F64;
            if (p.aperiodic)
                solve_aperiodic(p.grid, f64, p.ndim, p.dims, p.coeffs, p.radius, p.T, p.aperiodic - 1, st);
            else if (p.radius > kMaxR)
                solve_periodic_general(p.grid, f64, p.ndim, p.dims, p.coeffs, p.radius, p.T, st);
            else
                solve_periodic_any(p.grid, f64, p.ndim, p.dims, p.coeffs, p.radius, p.T, st);
        }
    });
}

int stencil_fft_graph_create(const sfft_problem* probs, int n, sfft_graph** out) {
    return guarded_call([&] {
        if (!out || n < 1 || !probs) throw Error(SFFT_EINVAL, "invalid arguments");
        *out = nullptr;
        for (int i = 0; i < n; ++i) {
            try {
                validate_problem(probs[i]);
            } catch (const Error& e) {
                throw Error(e.code, "problem " + std::to_string(i) + ": " + e.what());
            }
            if (!batchable(probs[i]))
                throw Error(SFFT_EUNSUPPORTED, "problem " + std::to_string(i) +
                                                   ": graphs hold periodic problems of 7-smooth extents and radius <= 2");
        }
        std::unique_ptr<sfft_graph> g(new sfft_graph());
        check_hip(hipGetDevice(&g->device), "hipGetDevice");
        for (int i = 0; i < n; ++i)
            if (probs[i].T > 0) g->runs.push_back(prepare_periodic(probs[i]));
        g->mem.ws_cap = batch_ws_bytes(g->runs);
        g->mem.desc_cap = batch_desc_bytes(g->runs);
        check_hip(hipMalloc(&g->mem.ws, g->mem.ws_cap), "hipMalloc(graph workspace)");
        check_hip(hipMalloc(&g->mem.desc, g->mem.desc_cap), "hipMalloc(graph descriptors)");
        BatchProgram prog = build_batch(g->runs, g->mem);
        check_hip(hipMemcpy(g->mem.desc, prog.host_desc.data(), prog.host_desc.size(), hipMemcpyHostToDevice),
                  "descriptor upload");
        hipStream_t cs;
        check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        const bool prof = profiling();
        if (prof) profile_pause(true);
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            try {
                enqueue_batch(prog, g->runs, g->mem, cs, false);
            } catch (...) {
                hipGraph_t tmp;
                (void)hipStreamEndCapture(cs, &tmp);
                if (tmp) (void)hipGraphDestroy(tmp);
                if (prof) profile_pause(false);
                (void)hipStreamDestroy(cs);
                throw;
            }
            e = hipStreamEndCapture(cs, &g->graph);
        }
        if (prof) profile_pause(false);
        (void)hipStreamDestroy(cs);
        check_hip(e, "stream capture");
        check_hip(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        *out = g.release();
    });
}

int stencil_fft_graph_launch(sfft_graph* g, void* stream) {
    return guarded_call([&] {
        if (!g || !g->exec) throw Error(SFFT_EINVAL, "invalid graph");
        check_hip(hipGraphLaunch(g->exec, (hipStream_t)stream), "hipGraphLaunch");
    });
}

void stencil_fft_graph_destroy(sfft_graph* g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->mem.ws) (void)hipFree(g->mem.ws);
    if (g->mem.desc) (void)hipFree(g->mem.desc);
    delete g;
}

}  // extern "C"
