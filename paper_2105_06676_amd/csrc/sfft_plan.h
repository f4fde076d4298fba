// Host-side pass schedule for one periodic problem shape (no GPU needed).
#pragma once

#include <stdint.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sfft_types.h"

namespace sfft {

// A device table the schedule needs: exp(-2 pi i (m * mult) / N) for m < count.
struct TwiddleReq {
    int64_t N, count, mult;
    bool operator<(const TwiddleReq& o) const {
        if (N != o.N) return N < o.N;
        if (count != o.count) return count < o.count;
        return mult < o.mult;
    }
};

struct PassPlan {
    PassDesc pd;              // table pointers, buffer and views unset
    TwiddleReq stage_tab;     // stage twiddles
    bool has_tw = false;
    TwiddleReq tw_lo, tw_hi;  // split twiddles
    bool has_fast = false;    // power-of-two kernels: two-level tables of exp(-2 pi i m / L)
    TwiddleReq f_lo, f_hi;
    bool has_half = false;    // ... and of exp(-2 pi i m / 2L) for real rows
    TwiddleReq h_lo, h_hi;
    size_t lds_bytes = 0;
    int64_t model_bytes = 0;  // algorithmic HBM bytes (read + write) of one launch
    std::string name;         // kernel family for profiling
};

struct Schedule {
    int d = 0;
    int64_t dims[3] = {1, 1, 1};
    int64_t B = 1;
    bool f64 = false;
    std::vector<PassPlan> passes;
    int64_t spec_elems = 0;   // complex elements of the spectrum workspace
    SymParams sym{};          // geometry part (n, nlev, sub, sdim, hcount)
    int64_t model_bytes = 0;  // sum over passes
    bool fused = true;        // the middle pass multiplies by the symbol
    int sym_at = -1;          // unfused: index of the first inverse pass (the whole
                              // forward spectrum is in the workspace before it)
};

// Passes of an unnormalised complex DFT of length n along the middle axis of a
// complex [outer][n][inner] array held in the workspace (any 7-smooth n).  Forward:
// every factor level, twiddles after each level but the last, output in
// digit-reversed order across levels; inverse: the mirror, natural order out.
// levels receives the factorisation (position -> frequency as in the solver).
int axis_schedule(int64_t outer, int64_t n, int64_t inner, bool f64, bool inverse, std::vector<PassPlan>* out,
                  std::vector<int64_t>* levels, std::string* why);

// Autotuned factorisations of strided axes: (extent, f64) -> factor levels in
// pass order (the last level of axis 0 is the fused middle pass).  `gen` counts
// changes, so cached plans built before a change are not reused.
constexpr int64_t kMaxTunedLevel = 1024;
struct TuneDB {
    std::mutex mu;
    std::map<std::pair<int64_t, int>, std::vector<int64_t>> split;
    std::atomic<uint64_t> gen{0};
};
TuneDB& tune_db();
bool valid_split(int64_t n, const std::vector<int64_t>& levels);

struct Tunables {
    int col_max = 0;          // 0: default
    int aperiodic_cutoff = 0; // 0: per-shape default
    int no_fast = 0;          // 1: generic kernels only (testing)
    int aperiodic_graphs = 1; // 1: replay repeated aperiodic solves from captured graphs
    int mixed_row_q = 0;      // most points per thread of mixed-radix row passes (0: default)
    int mixed_col_q = 0;      // ... and of strided-axis passes
};
Tunables& tunables();

bool is_7smooth(int64_t n);
// 0 on success; on failure a message in *why.
// unfused: forward transform, a gap for an elementwise spectral step, then the
// inverse transform (no fused middle pass; d = 1 needs a single row).
int build_schedule(int d, const int64_t* dims, int64_t B, bool f64, Schedule* out, std::string* why,
                   bool unfused = false);
std::string describe_schedule(const Schedule& s);

}  // namespace sfft
