// Per-device runtime shared by the entry points: tables, plans, workspace,
// error reporting and kernel timing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <functional>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "sfft_plan.h"
#include "sfft_types.h"

namespace sfft {

// Error carried to the C ABI boundary.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
void check_hip(hipError_t e, const char* what);
void set_last_error(const std::string& msg);
void clear_last_error();

struct Plan {
    Schedule s;
    std::vector<PassDesc> pd;      // with table pointers bound
    std::vector<size_t> lds;
};

struct DevCtx {
    int device = 0;
    std::mutex mu;
    std::map<TwiddleReq, std::pair<double2*, float2*>> tw;
    std::map<int64_t, double2*> eph;
    std::map<std::string, std::shared_ptr<Plan>> plans;
    std::map<hipStream_t, std::pair<void*, size_t>> ws;
    size_t lds_max = 0;
    hipStream_t tstream = nullptr;   // table generation

    std::shared_ptr<Plan> plan(int d, const int64_t* dims, int64_t B, bool f64, bool unfused = false);
    // Complex transform along the middle axis of [outer][n][inner] (sym.nlev[0] /
    // sym.sub[0] hold its factor levels).
    std::shared_ptr<Plan> axis_plan(int64_t outer, int64_t n, int64_t inner, bool f64, bool inverse);
    void bind_passes(Plan& p, bool f64);
    const double2* phase_table(int64_t n);
    void* workspace(hipStream_t st, size_t bytes);
    void* scratch(hipStream_t st, int slot, size_t bytes);  // extra per-stream buffers
    std::map<std::pair<hipStream_t, int>, std::pair<void*, size_t>> extra;
    // Helper streams and events owned by a caller stream, for solves that fork
    // independent work off it and join it back (created on first use, default
    // priority, non-blocking).
    // Copy `bytes` of host data into scratch slot `slot` of stream `st`, in stream
    // order, through a pinned staging buffer of that stream (the host data may be
    // released on return); returns the device pointer.
    void* upload(hipStream_t st, int slot, const void* host, size_t bytes);
    // The same into a device buffer the caller owns.
    void upload_to(hipStream_t st, void* dev, const void* host, size_t bytes);
    std::map<hipStream_t, std::pair<std::pair<void*, size_t>, hipEvent_t>> staging;
    hipStream_t side_stream(hipStream_t st, int i);
    hipEvent_t side_event(hipStream_t st, int i);
    std::map<std::pair<hipStream_t, int>, hipStream_t> sides;
    std::map<std::pair<hipStream_t, int>, hipEvent_t> side_events;
    // Count of workspace / scratch buffers released so far; enqueued work (or a
    // captured graph) that baked in buffer addresses is stale once it changes.
    std::atomic<uint64_t> epoch{0};

   private:
    std::pair<double2*, float2*> table(const TwiddleReq& r);
};

DevCtx& device_ctx();  // context of the current HIP device (created on first use)

// Coefficient-dependent part of the symbol parameters (Sec. 3 Steps 1(i), 2).
// The (possibly normalised) coefficients go to sp.c, or to `cout` when given
// (stencils with more than kMaxCoef coefficients).
void fill_symbol(SymParams& sp, const double* coeffs, int radius, int d, int64_t T, double scale,
                 double* cout = nullptr);

// Fill `tab` with the per-column symbol parts of `sym` (d >= 2) and point
// sym.coltab / sym.ncol at it.
void build_symbol_columns(SymParams& sym, void* tab, bool f64, hipStream_t st);

// Enqueue passes [pass_begin, pass_end) of a plan (all by default; builds the
// column table first unless sym.coltab is set).  in/out: real views of the first / last pass.
void run_plan(const Plan& p, void* ws, const RealView& in, const RealView& out, const KeepRule& keep,
              const SymParams& sym, hipStream_t st, size_t pass_begin = 0, size_t pass_end = SIZE_MAX);

// Natural row-major view of a dense array of `dims` (batch stride = element count).
RealView dense_view(void* ptr, int d, const int64_t* dims);

// Kernel timing (HIP events on the launch stream).
bool profiling();
void profile_pause(bool paused);  // no events while a graph is being captured
void profile_launch_begin(hipStream_t st, hipEvent_t* ev);
void profile_launch_end(hipStream_t st, hipEvent_t ev0, const std::string& name, int64_t bytes);

}  // namespace sfft
