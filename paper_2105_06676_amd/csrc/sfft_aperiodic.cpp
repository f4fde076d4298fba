// StencilFFT-A / RecursiveBoundary (Sec. 4) -- placeholder until the planner lands.
#include "sfft_runtime.h"

namespace sfft {

void solve_aperiodic(void*, bool, int, const int64_t*, const double*, int, int64_t, hipStream_t) {
    throw Error(-2, "aperiodic solver not built yet");
}

}  // namespace sfft
