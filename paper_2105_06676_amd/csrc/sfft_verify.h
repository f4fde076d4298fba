// Host-side verification of pass schedules against the buffers of a solve
// (sfft_verify.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "sfft_plan.h"

namespace sfft {

struct Verifier {
    struct Buf {
        uintptr_t base;
        size_t bytes;
        std::string name;
    };
    std::vector<Buf> bufs;
    std::vector<std::string> errors;  // the first 64 failures
    int64_t nerr = 0, checked = 0;

    void add(const void* base, size_t bytes, const std::string& name);
    void fail(const std::string& what);
    // elements [0, hi_elem] of size esz from p lie inside one registered buffer
    void range(const void* p, int64_t hi_elem, size_t esz, const std::string& what);
    // every pass of s with the solve's workspace, views and symbol column table
    void schedule(const Schedule& s, const void* ws, const RealView& in, const RealView& out, const void* coltab,
                  int64_t ncol, const std::string& tag);
};

}  // namespace sfft
