// Batched execution of many periodic problems (uneven shapes, dtypes and T).
#pragma once

#include <memory>
#include <vector>

#include "../../include/stencil_fft.h"
#include "sfft_runtime.h"

namespace sfft {

// One validated periodic problem bound to its plan and symbol parameters.
struct ProblemRun {
    std::shared_ptr<Plan> plan;
    RealView view;
    SymParams sp;
    size_t ws_bytes = 0;    // spectrum workspace
    size_t col_bytes = 0;   // per-column symbol table
};

// Validation shared by every entry point; throws Error.  Periodic problems may
// have any extent and radius up to kMaxGeneralR; aperiodic ones radius <= 2.
void validate_problem(const sfft_problem& p);
// Boundary condition of an aperiodic problem (SFFT_BC_*), checked against its extents.
void validate_bc(int bc, int ndim, const int64_t* dims, int radius);
// Periodic problems that run in batched launches (7-smooth extents, radius <= 2);
// the others are solved one after another on the batch's stream.
bool batchable(const sfft_problem& p);

// Plan a periodic problem (creates plans and tables on the current device).
ProblemRun prepare_periodic(const sfft_problem& p);
// Host-only estimate of a problem's device workspace (no GPU needed).
size_t problem_workspace_bytes(const sfft_problem& p);
// Host-only sizes of a periodic problem: workspace + column table bytes, number
// of passes, algorithmic HBM bytes of all passes.
struct ProblemSize {
    size_t ws_bytes = 0;
    size_t passes = 0;
    int64_t model_bytes = 0;
};
ProblemSize problem_size(const sfft_problem& p);

// Device buffers a batch runs in: workspaces and column tables sub-allocated from
// `ws`, descriptors in `desc`.
struct BatchMem {
    char* ws = nullptr;
    size_t ws_cap = 0;
    char* desc = nullptr;
    size_t desc_cap = 0;
};
size_t batch_ws_bytes(const std::vector<ProblemRun>& runs);
size_t batch_desc_bytes(const std::vector<ProblemRun>& runs);

// Build the work lists of a batch (one list per pass index and kernel variant)
// and upload them to mem.desc.  Returns the launches to make.
struct BatchLaunch {
    PassDesc proto;
    const BatchItem* items;   // device
    int n;
    int64_t tiles;
    size_t lds;
    bool f64;
    std::string name;
    int64_t bytes;
};
struct BatchProgram {
    std::vector<std::pair<int, void*>> coltabs;  // (run index, device table) to fill before the passes
    const SymParams* syms = nullptr;              // device
    std::vector<BatchLaunch> launches;
    std::vector<char> host_desc;                  // image of mem.desc
};
// With `bases`, run i's workspace (and then its column table) lives at bases[i]
// instead of being sub-allocated from mem.ws.
BatchProgram build_batch(std::vector<ProblemRun>& runs, const BatchMem& mem,
                         const std::vector<char*>* bases = nullptr);

// Upload the descriptors (through per-stream pinned staging) and enqueue the
// program on `st`.  With upload = false the descriptors must already be there.
void enqueue_batch(BatchProgram& prog, std::vector<ProblemRun>& runs, const BatchMem& mem, hipStream_t st,
                   bool upload);

}  // namespace sfft
