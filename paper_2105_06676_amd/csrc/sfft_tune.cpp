// Autotuner of the periodic pass schedule.
//
// For every distinct extent of a strided axis of a problem shape the tuner times
// the candidate factorisations of that axis into sub-transforms (the single
// transform when it fits, balanced and unbalanced two-level splits in both
// orders, the orders of a three-level split) with whole solves, keeps the
// fastest in the tuning database (which the planner consults before its
// balanced default) and reports what it measured.  A candidate is only eligible
// after its result on a step count that keeps every mode visible matched the
// default schedule's result to the dtype's tolerance.  The database persists
// as JSON (stencil_fft_tune_save / _load).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <vector>

#include "../../include/stencil_fft.h"
#include "sfft_plan.h"
#include "sfft_runtime.h"
#include "sfft_solvers.h"

namespace sfft {

int guarded_call(const std::function<void()>& f);

namespace {

std::vector<std::vector<int64_t>> candidates(int64_t n) {
    std::vector<std::vector<int64_t>> out;
    if (n <= kMaxTunedLevel) out.push_back({n});
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (int64_t s0 = 2; s0 <= kMaxTunedLevel && s0 < n; ++s0) {
        if (n % s0) continue;
        const int64_t s1 = n / s0;
        if (s1 > kMaxTunedLevel || s1 < 2 || s0 > s1) continue;
        pairs.push_back({s0, s1});
    }
    // the most balanced few, both orders
    std::sort(pairs.begin(), pairs.end(), [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
        return a.first > b.first;
    });
    for (size_t i = 0; i < pairs.size() && i < 3; ++i) {
        out.push_back({pairs[i].first, pairs[i].second});
        if (pairs[i].first != pairs[i].second) out.push_back({pairs[i].second, pairs[i].first});
    }
    if (out.empty()) {
        // three levels: the orders of the most balanced factorisation
        int64_t best = 0;
        std::vector<int64_t> f;
        for (int64_t a = 2; a <= kMaxTunedLevel && a < n; ++a) {
            if (n % a) continue;
            for (int64_t b = a; b <= kMaxTunedLevel && a * b < n; ++b) {
                if ((n / a) % b) continue;
                const int64_t c = n / a / b;
                if (c < b || c > kMaxTunedLevel) continue;
                if (a > best) { best = a; f = {a, b, c}; }
            }
        }
        if (!f.empty()) {
            std::sort(f.begin(), f.end());
            do out.push_back(f); while (std::next_permutation(f.begin(), f.end()));
        }
    }
    return out;
}

struct DevBuf {
    void* p = nullptr;
    explicit DevBuf(size_t bytes) { check_hip(hipMalloc(&p, bytes), "hipMalloc(tuning buffer)"); }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

std::string levels_json(const std::vector<int64_t>& l) {
    std::ostringstream o;
    o << "[";
    for (size_t i = 0; i < l.size(); ++i) o << (i ? ", " : "") << l[i];
    o << "]";
    return o.str();
}

// One tuning stream per device for the life of the process (the solves' per-stream
// workspace is keyed by it, so it is reused by every tuning call).
hipStream_t tuning_stream() {
    static std::mutex m;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> g(m);
    hipStream_t& s = streams[dev];
    if (!s) check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate(tuning)");
    return s;
}

void set_split(int64_t n, bool f64, const std::vector<int64_t>* lev) {
    TuneDB& db = tune_db();
    std::lock_guard<std::mutex> g(db.mu);
    if (lev) db.split[{n, f64 ? 1 : 0}] = *lev;
    else db.split.erase({n, f64 ? 1 : 0});
    db.gen++;
}

}  // namespace

std::string tune_shape(int d, const int64_t* dims, bool f64, int reps) {
    const size_t esz = f64 ? 8 : 4;
    int64_t N = 1;
    for (int a = 0; a < d; ++a) N *= dims[a];
    // input: a deterministic pattern; stencil: an asymmetric 3^d box of positive
    // weights (every mode visible after the few steps of the check)
    std::vector<double> h((size_t)N);
    uint64_t z = 0x9E3779B97F4A7C15ull;
    for (int64_t i = 0; i < N; ++i) {
        z ^= z >> 33;
        z *= 0xff51afd7ed558ccdull;
        z ^= z >> 29;
        h[(size_t)i] = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    }
    std::vector<float> hf;
    const void* src = h.data();
    if (!f64) {
        hf.assign(h.begin(), h.end());
        src = hf.data();
    }
    int nc = 1;
    for (int a = 0; a < d; ++a) nc *= 3;
    std::vector<double> c((size_t)nc);
    double sum = 0.0;
    for (int i = 0; i < nc; ++i) sum += (c[(size_t)i] = 1.0 + (double)((i * 37) % 11));
    for (auto& x : c) x /= sum;
    DevBuf x0((size_t)N * esz), x((size_t)N * esz);
    check_hip(hipMemcpy(x0.p, src, (size_t)N * esz, hipMemcpyHostToDevice), "tuning input");
    hipStream_t st = tuning_stream();
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    check_hip(hipEventCreate(&e1), "hipEventCreate");
    const int64_t Tcheck = 3, Ttime = 4096;
    auto solve = [&](int64_t T) {
        check_hip(hipMemcpyAsync(x.p, x0.p, (size_t)N * esz, hipMemcpyDeviceToDevice, st), "tuning copy");
        solve_periodic_dense(x.p, f64, d, dims, 1, c.data(), 1, T, st);
    };
    auto fetch = [&](std::vector<double>& out) {
        check_hip(hipStreamSynchronize(st), "hipStreamSynchronize(tuning)");
        out.resize((size_t)N);
        if (f64) {
            check_hip(hipMemcpy(out.data(), x.p, (size_t)N * 8, hipMemcpyDeviceToHost), "tuning result");
        } else {
            std::vector<float> t((size_t)N);
            check_hip(hipMemcpy(t.data(), x.p, (size_t)N * 4, hipMemcpyDeviceToHost), "tuning result");
            for (int64_t i = 0; i < N; ++i) out[(size_t)i] = t[(size_t)i];
        }
    };
    // back-to-back solves in place, as a serving loop or a benchmark runs them
    // (a copy before each solve would leave part of the input in the last-level
    // cache and favour some schedules); the median of three such runs
    auto time_us = [&]() {
        solve(Ttime);  // warm
        std::vector<float> ts;
        for (int k = 0; k < 3; ++k) {
            check_hip(hipEventRecord(e0, st), "hipEventRecord");
            for (int i = 0; i < reps; ++i) solve_periodic_dense(x.p, f64, d, dims, 1, c.data(), 1, Ttime, st);
            check_hip(hipEventRecord(e1, st), "hipEventRecord");
            check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            ts.push_back(ms * 1e3f / (float)reps);
        }
        std::sort(ts.begin(), ts.end());
        return (double)ts[1];
    };
    const double tol = f64 ? 1e-12 : 1e-5;
    std::ostringstream rep;
    rep.precision(6);
    rep << "{\"dims\": [";
    for (int a = 0; a < d; ++a) rep << (a ? ", " : "") << dims[a];
    rep << "], \"f64\": " << (f64 ? 1 : 0) << ", \"axes\": [";
    std::vector<int64_t> seen;
    bool first_axis = true;
    try {
        for (int a = 0; a + 1 < d; ++a) {
            const int64_t n = dims[a];
            if (n < 2 || std::find(seen.begin(), seen.end(), n) != seen.end()) continue;
            seen.push_back(n);
            // the default schedule (no database entry) is the reference and a candidate
            set_split(n, f64, nullptr);
            std::vector<int64_t> deflev;
            {
                Schedule s0;
                std::string why0;
                if (build_schedule(d, dims, 1, f64, &s0, &why0) == 0)
                    for (int l = 0; l < s0.sym.nlev[a]; ++l) deflev.push_back(s0.sym.sub[a][l]);
            }
            std::vector<double> ref, got;
            solve(Tcheck);
            fetch(ref);
            double rn = 0.0;
            for (double v : ref) rn += v * v;
            rn = std::sqrt(rn);
            double best_us = time_us();
            std::vector<int64_t> best;  // empty: the default
            rep << (first_axis ? "" : ", ") << "{\"n\": " << n << ", \"default_us\": " << best_us
                << ", \"candidates\": [";
            first_axis = false;
            bool first = true;
            const double default_us = best_us;
            for (const auto& cand : candidates(n)) {
                if (cand == deflev) continue;  // the default itself, timed above
                set_split(n, f64, &cand);
                std::string why;
                Schedule s;
                if (build_schedule(d, dims, 1, f64, &s, &why) != 0) continue;
                try {
                    solve(Tcheck);
                    fetch(got);
                } catch (const Error& err) {
                    // e.g. a level whose tile exceeds the LDS: not a candidate
                    rep << (first ? "" : ", ") << "{\"levels\": " << levels_json(cand) << ", \"error\": \"" << err.code
                        << "\", \"eligible\": false}";
                    first = false;
                    continue;
                }
                double en = 0.0, emax = 0.0, rmax = 0.0;
                for (size_t i = 0; i < got.size(); ++i) {
                    const double e = got[i] - ref[i];
                    en += e * e;
                    emax = std::max(emax, std::fabs(e));
                    rmax = std::max(rmax, std::fabs(ref[i]));
                }
                const double rel = rn > 0 ? std::sqrt(en) / rn : std::sqrt(en);
                const bool ok = rel <= tol && emax <= tol * std::max(rmax, 1e-300);
                const double us = ok ? time_us() : -1.0;
                rep << (first ? "" : ", ") << "{\"levels\": " << levels_json(cand) << ", \"rel_l2_vs_default\": " << rel
                    << ", \"eligible\": " << (ok ? "true" : "false") << ", \"us\": " << us << "}";
                first = false;
                // a different schedule must win by more than the run-to-run noise
                if (ok && us < best_us && us < 0.99 * default_us) {
                    best_us = us;
                    best = cand;
                }
            }
            set_split(n, f64, best.empty() ? nullptr : &best);
            rep << "], \"chosen\": " << (best.empty() ? std::string("\"default\"") : levels_json(best))
                << ", \"chosen_us\": " << best_us << "}";
        }
    } catch (...) {
        (void)hipStreamSynchronize(st);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    check_hip(hipStreamSynchronize(st), "hipStreamSynchronize(tuning)");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    rep << "]}";
    return rep.str();
}

std::string tune_db_json() {
    TuneDB& db = tune_db();
    std::lock_guard<std::mutex> g(db.mu);
    std::ostringstream o;
    o << "{\"version\": 1, \"splits\": [";
    bool first = true;
    for (auto& kv : db.split) {
        o << (first ? "" : ", ") << "{\"n\": " << kv.first.first << ", \"f64\": " << kv.first.second
          << ", \"levels\": " << levels_json(kv.second) << "}";
        first = false;
    }
    o << "]}";
    return o.str();
}

// Entries of the JSON written by tune_db_json: every {"n": .., "f64": .., "levels": [..]}.
void tune_db_parse(const std::string& text) {
    std::vector<std::pair<std::pair<int64_t, int>, std::vector<int64_t>>> entries;
    size_t pos = text.find("\"splits\"");
    if (pos == std::string::npos) throw Error(SFFT_EINVAL, "tuning file has no \"splits\" list");
    auto read_int = [&](const std::string& key, size_t from, size_t to, int64_t* v) {
        const size_t k = text.find("\"" + key + "\"", from);
        if (k == std::string::npos || k > to) return false;
        size_t c = text.find(':', k);
        if (c == std::string::npos || c > to) return false;
        *v = std::strtoll(text.c_str() + c + 1, nullptr, 10);
        return true;
    };
    for (;;) {
        const size_t b = text.find('{', pos + 1);
        if (b == std::string::npos) break;
        const size_t e = text.find('}', b);
        if (e == std::string::npos) throw Error(SFFT_EINVAL, "tuning file: unterminated entry");
        int64_t n = 0, f = 0;
        if (!read_int("n", b, e, &n) || !read_int("f64", b, e, &f)) throw Error(SFFT_EINVAL, "tuning file: bad entry");
        const size_t l0 = text.find('[', text.find("\"levels\"", b));
        const size_t l1 = text.find(']', l0);
        if (l0 == std::string::npos || l1 == std::string::npos || l1 > e) throw Error(SFFT_EINVAL, "tuning file: bad levels");
        std::vector<int64_t> lev;
        const char* p = text.c_str() + l0 + 1;
        const char* end = text.c_str() + l1;
        while (p < end) {
            char* q = nullptr;
            const long long v = std::strtoll(p, &q, 10);
            if (q == p) { ++p; continue; }
            lev.push_back(v);
            p = q;
        }
        if (!valid_split(n, lev)) throw Error(SFFT_EINVAL, "tuning file: levels do not multiply to n = " + std::to_string(n));
        entries.push_back({{n, f ? 1 : 0}, lev});
        pos = e;
    }
    TuneDB& db = tune_db();
    std::lock_guard<std::mutex> g(db.mu);
    for (auto& en : entries) db.split[en.first] = en.second;
    db.gen++;
}

}  // namespace sfft

using namespace sfft;

extern "C" {

int stencil_fft_tune(int ndim, const int64_t* dims, sfft_dtype dtype, int reps, char* report, int64_t cap) {
    std::string out;
    const int rc = guarded_call([&] {
        if (ndim < 1 || ndim > 3 || !dims) throw Error(SFFT_EINVAL, "ndim must be 1..3");
        if (dtype != SFFT_F32 && dtype != SFFT_F64) throw Error(SFFT_EINVAL, "unknown dtype");
        if (reps < 1 || reps > 1000) throw Error(SFFT_EINVAL, "reps must be in 1..1000");
        for (int a = 0; a < ndim; ++a) {
            if (dims[a] < 1) throw Error(SFFT_EINVAL, "extents must be >= 1");
            if (!is_7smooth(dims[a])) throw Error(SFFT_EUNSUPPORTED, "the tuner takes 7-smooth extents");
        }
        out = tune_shape(ndim, dims, dtype == SFFT_F64, reps);
    });
    if (rc) return rc;
    if (report && cap > 0) {
        const int64_t n = std::min<int64_t>((int64_t)out.size(), cap - 1);
        std::memcpy(report, out.data(), (size_t)n);
        report[n] = 0;
    }
    return (int)std::min<int64_t>((int64_t)out.size(), INT32_MAX);
}

int stencil_fft_tune_save(const char* path) {
    return guarded_call([&] {
        if (!path) throw Error(SFFT_EINVAL, "path is null");
        std::ofstream f(path);
        if (!f) throw Error(SFFT_EINVAL, std::string("cannot write ") + path);
        f << tune_db_json() << "\n";
    });
}

int stencil_fft_tune_load(const char* path) {
    return guarded_call([&] {
        if (!path) throw Error(SFFT_EINVAL, "path is null");
        std::ifstream f(path);
        if (!f) throw Error(SFFT_EINVAL, std::string("cannot read ") + path);
        std::stringstream ss;
        ss << f.rdbuf();
        tune_db_parse(ss.str());
    });
}

int stencil_fft_tune_clear(void) {
    return guarded_call([&] {
        TuneDB& db = tune_db();
        std::lock_guard<std::mutex> g(db.mu);
        db.split.clear();
        db.gen++;
    });
}

}  // extern "C"
