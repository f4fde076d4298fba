// Pass schedule of a periodic solve (Sec. 3, StencilFFT-P; d-D form in the
// appendix on d-D grids).
//
// d >= 2:  row R2C along the last (contiguous) axis, column passes along axes
//          d-2 .. 1, column passes along axis 0 whose last sub-transform is the
//          fused middle pass (forward, lambda^T / N, inverse), then the inverse
//          passes in reverse order and a row C2R.
// d == 1:  one fused row pass when the row fits in LDS; otherwise the axis is
//          split n = s_0 [* s_1] * s_row: column sub-passes over the leading
//          factors, a complex row middle pass over s_row, and back.
// A strided axis longer than col_max is split into up to three factors; the
// forward output stays in digit-reversed order (no transposes).
#include "sfft_plan.h"

#include "sfft_fast.h"
#include "sfft_mixed.h"

#include <algorithm>
#include <cstring>
#include <sstream>

namespace sfft {

Tunables& tunables() {
    static Tunables t;
    return t;
}

bool is_7smooth(int64_t n) {
    if (n < 1) return false;
    for (int64_t p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

static bool radix_list(int64_t L, int* out, int* nst) {
    std::vector<int> r;
    int64_t n = L;
    while (n % 8 == 0) { r.push_back(8); n /= 8; }
    if (n % 4 == 0) { r.push_back(4); n /= 4; }
    if (n % 2 == 0) { r.push_back(2); n /= 2; }
    for (int p : {7, 5, 3})
        while (n % p == 0) { r.push_back(p); n /= p; }
    if (n != 1 || (int)r.size() > kMaxStages) return false;
    *nst = (int)r.size();
    for (size_t i = 0; i < r.size(); ++i) out[i] = r[i];
    return true;
}

static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// Stage list of a length L with Q points per thread (Q | L): radix Q first; radix Q
// last when Q^2 | L, else the largest prime of Q that divides L / Q; the rest in
// between as the fewest radices, largest first, from the proper divisors of Q and
// (general: the families mixing 3, 5 and 7) the primes 2..7 with 4 — a middle
// radix that does not divide Q spreads its butterflies unevenly over the threads,
// and the kernels of those families carry the guarded stages for it.  When no
// prime of Q divides L / Q, `gather` allows a last radix that does not divide Q:
// the kernels then run it through LDS like a middle stage and read the outputs
// back in natural order.
static bool mixed_stages(int64_t L, int q, bool general, bool gather, std::vector<int>* out) {
    if (L % q) return false;
    int64_t rest = L / q;
    int last = 0;
    if (rest % q == 0 && rest > 1) {
        last = q;
    } else {
        for (int p : {7, 5, 3, 2})
            if (q % p == 0 && rest % p == 0) { last = p; break; }
    }
    if (last == 0 && !gather) return false;
    if (last != 0) {
        if (rest < last) return false;
        rest /= last;
    }
    std::vector<int> cand;
    for (int dv : {25, 21, 20, 15, 14, 12, 10, 6})
        if (dv < q && q % dv == 0) cand.push_back(dv);
    for (int dv : {7, 5, 4, 3, 2})
        if (general || q % dv == 0) cand.push_back(dv);
    // Q itself for the inner stages when it divides the rest
    std::vector<int> mid;
    while (rest % q == 0 && rest > 1) { mid.push_back(q); rest /= q; }
    for (int dv : cand)
        while (rest % dv == 0) { mid.push_back(dv); rest /= dv; }
    if (rest != 1) return false;
    std::vector<int> r{q};
    r.insert(r.end(), mid.begin(), mid.end());
    if (last != 0) r.push_back(last);
    *out = r;
    return true;
}

// Families whose kernels carry the gather form (a last radix not dividing Q).
static bool gather_family(int q, bool f64) {
    return q == 7 || q == 9 || q == 12 || q == 14 || q == 15 || (q == 21 && !f64);
}

bool mixed_family(int64_t L, bool column, bool f64, int* Q, int64_t* packed, int* nst) {
    if (tunables().no_fast || L < 2) return false;
    int64_t n = L;
    int e2 = 0, e3 = 0, e5 = 0, e7 = 0;
    while (n % 2 == 0) { n /= 2; ++e2; }
    while (n % 3 == 0) { n /= 3; ++e3; }
    while (n % 5 == 0) { n /= 5; ++e5; }
    while (n % 7 == 0) { n /= 7; ++e7; }
    if (n != 1) return false;
    // Points per thread, most preferred first.  Every stage is one LDS exchange and
    // the radix-Q stages cover most of the length, so more points per thread means
    // fewer stages; but a long row is one workgroup of L/Q threads, and at 20
    // points (about 200 VGPRs) only two rows fit a CU, as at 10 points (about 110
    // VGPRs, twice the threads), so even rows prefer 10 (measured equal on
    // 4000-point rows, faster on short rows where many rows share a workgroup).
    // FP64 points take twice the registers: 20, 21 or 25 of them would run one
    // wave per SIMD.  The 2^a 5^b, 2^a 3^b (a >= 2), 5^b, 7^b and 3^b (times at
    // most one 2) lengths keep their families; the others take the first of 12,
    // 14, 15, 21, 9, 7 that divides them and leaves a last radix, else the first
    // whose gather form fits.  An option caps the choice, rows and columns
    // separately.
    std::vector<int> pref;
    bool general = false;
    if (e3 == 0 && e7 == 0 && e5 >= 1) {
        if (e2 >= 2 && !f64 && column) pref.push_back(20);
        if (e2 >= 1) pref.push_back(10);
        if (e2 == 0 && !f64) pref.push_back(25);
        pref.push_back(5);
    } else if (e5 == 0 && e7 == 0 && e3 >= 1 && e2 >= 2) {
        pref.push_back(12);
    } else if (e2 == 0 && e3 == 0 && e5 == 0 && e7 >= 2) {
        pref.push_back(7);
    } else if (e5 == 0 && e7 == 0 && e3 >= 2 && e2 <= 1) {
        pref.push_back(9);
        general = true;
    } else {
        pref = {12, 14, 15};
        if (!f64) pref.push_back(21);
        pref.push_back(9);
        pref.push_back(7);
        general = true;
    }
    const int cap = column ? tunables().mixed_col_q : tunables().mixed_row_q;
    std::vector<int> r;
    int q = 0;
    for (int gather = 0; gather <= 1 && q == 0; ++gather) {
        for (int c : pref) {
            if (cap != 0 && c > cap && c != pref.back()) continue;
            if (gather && !gather_family(c, f64)) continue;
            if (mixed_stages(L, c, general || c == 12, gather != 0, &r)) { q = c; break; }
        }
    }
    if (q == 0) return false;
    const int64_t P = L / q;
    if (P < 1 || P > (column ? 64 : 512) || r.size() < 2 || (int)r.size() * kMRadBits > 64) return false;
    int64_t pk = 0, prod = 1;
    for (size_t i = 0; i < r.size(); ++i) {
        prod *= r[i];
        pk |= (int64_t)r[i] << (kMRadBits * i);
    }
    if (prod != L || (q % r.back() && !gather_family(q, f64))) return false;
    *Q = q;
    *packed = pk;
    *nst = (int)r.size();
    return true;
}

TuneDB& tune_db() {
    static TuneDB db;
    return db;
}

bool valid_split(int64_t n, const std::vector<int64_t>& lev) {
    if (lev.empty() || lev.size() > 3) return false;
    int64_t p = 1;
    for (int64_t s : lev) {
        if (s < 1 || s > kMaxTunedLevel) return false;
        if (lev.size() > 1 && s < 2) return false;
        p *= s;
    }
    return p == n;
}

// Register mixed-radix column tile of length L (a register family, at least
// four columns per workgroup, at most 128 KB of LDS); the tile geometry in *W,
// *bytes when given.
static bool mixed_col_fit(int64_t L, bool f64, int* mq, int64_t* mrad, int* mst, int64_t* W = nullptr,
                          size_t* bytes = nullptr) {
    if (!mixed_family(L, true, f64, mq, mrad, mst)) return false;
    const int64_t P = L / *mq;
    const int64_t Wm = std::min<int64_t>(64, 256 / P);
    const size_t b = (size_t)std::max<int64_t>(L * (Wm + 1), 256 * (int64_t)*mq) * (f64 ? 16 : 8);
    if (Wm < 4 || b > 128 * 1024) return false;
    if (W) *W = Wm;
    if (bytes) *bytes = b;
    return true;
}

// A strided level of L points runs on the register kernels (power-of-two or
// mixed-radix) rather than the generic ones.
static bool col_register(int64_t L, bool f64) {
    if (is_pow2(L)) return L >= kFastMinL && L <= kFastMaxColL && !tunables().no_fast;
    int mq = 0, mst = 0;
    int64_t mrad = 0;
    return mixed_col_fit(L, f64, &mq, &mrad, &mst);
}

// Split n (7-smooth) into 1..3 strided levels, unless the tuning database holds
// a factorisation for (n, f64).  Measured on one MI355X (strided axes of 600 to
// 8000 points, 2-D and 3-D, FP32 and FP64): every split moves the spectrum
// through HBM twice more, so one pass wins whenever a register kernel covers
// the whole axis (up to 1024 points with the default cap); otherwise a
// power-of-two level of at least 16 points with a register-kernel rest of at
// least 16 points (FP32: last, in the fused middle pass; FP64: first), else
// the most balanced split whose levels both run on register kernels, else the
// most balanced one.
static bool split_axis(int64_t n, int64_t cap, std::vector<int64_t>* out, bool f64) {
    out->clear();
    {
        TuneDB& db = tune_db();
        std::lock_guard<std::mutex> g(db.mu);
        auto it = db.split.find({n, f64 ? 1 : 0});
        if (it != db.split.end() && valid_split(n, it->second)) {
            *out = it->second;
            return true;
        }
    }
    if (n <= cap) { out->push_back(n); return true; }
    const bool dflt = tunables().col_max == 0;
    if (dflt && n <= kMaxTunedLevel && col_register(n, f64)) { out->push_back(n); return true; }
    const int64_t lmax = dflt ? kMaxTunedLevel : cap;
    auto level_ok = [&](int64_t s) { return s <= cap || (s <= lmax && col_register(s, f64)); };
    if (!is_pow2(n)) {
        int64_t p2 = 0;
        for (int64_t p = kFastMinL; p <= cap && n % p == 0; p *= 2) {
            const int64_t r = n / p;
            if (r >= kFastMinL && level_ok(r) && col_register(r, f64)) p2 = p;
        }
        if (p2) {
            out->push_back(f64 ? p2 : n / p2);
            out->push_back(f64 ? n / p2 : p2);
            return true;
        }
    }
    int64_t best = 0, b0 = 0;
    bool best_reg = false;
    for (int64_t s0 = 2; s0 <= lmax && s0 < n; ++s0) {
        if (n % s0) continue;
        const int64_t s1 = n / s0;
        if (!level_ok(s0) || !level_ok(s1)) continue;
        const bool reg = col_register(s0, f64) && col_register(s1, f64);
        const int64_t score = std::min(s0, s1);
        if ((reg && !best_reg) || (reg == best_reg && score > best)) { best = score; b0 = s0; best_reg = reg; }
    }
    if (b0) { out->push_back(b0); out->push_back(n / b0); return true; }
    int64_t bs = 0, c0 = 0, c1 = 0;
    for (int64_t s0 = 2; s0 <= cap && s0 < n; ++s0) {
        if (n % s0) continue;
        const int64_t rest = n / s0;
        for (int64_t s1 = 2; s1 <= cap && s1 < rest; ++s1) {
            if (rest % s1) continue;
            const int64_t s2 = rest / s1;
            if (s2 > cap) continue;
            const int64_t score = std::min(s0, std::min(s1, s2));
            if (score > bs) { bs = score; c0 = s0; c1 = s1; }
        }
    }
    if (!c0) return false;
    out->push_back(c0);
    out->push_back(c1);
    out->push_back(n / (c0 * c1));
    return true;
}


static int ilog2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

// Row length of a contiguous axis too long for one row pass: the largest divisor
// up to row_max, except that a power-of-two split keeps its strided cofactor at
// least kFastMinL long (shorter strided levels would run on the generic kernels,
// several times slower than a shorter register row pass).
static int64_t split_row(int64_t n, int64_t row_max) {
    int64_t first = 0;
    for (int64_t s = std::min(n, row_max); s >= 2; --s) {
        if (n % s) continue;
        if (!first) first = s;
        const int64_t co = n / s;
        if (is_pow2(s) && is_pow2(co) && co < kFastMinL) continue;
        return s;
    }
    return first;
}

static void two_level(int64_t N, TwiddleReq* lo, TwiddleReq* hi) {
    *lo = {N, 64, 1};
    *hi = {N, std::max<int64_t>(1, N / 64), 64};
}

static int64_t pow2_floor(int64_t x) {
    int64_t p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

struct Ctx {
    bool f64;
    int64_t esz;      // bytes per real
    int64_t csz;      // bytes per complex
    int64_t budget;   // complex elements per tile
};

static PassPlan make_row(const Ctx& c, int64_t rows, int L, int rowtrans, int mode, int nreal, int hcount,
                         int64_t ostride, bool allow_fast = true) {
    PassPlan p;
    PassDesc& pd = p.pd;
    std::memset(&pd, 0, sizeof(pd));
    pd.kind = PASS_ROW;
    pd.mode = mode;
    pd.rowtrans = rowtrans;
    pd.L = L;
    pd.nreal = nreal;
    pd.hcount = hcount;
    pd.outer = rows;
    pd.inner = 1;
    pd.ostride = ostride;
    pd.kstride = 1;
    pd.q_mod = 1;
    pd.lds_stride = rowtrans == RT_HALF ? L + 1 : L;
    int64_t W = std::max<int64_t>(1, c.budget / pd.lds_stride);
    W = std::min<int64_t>(W, rows);
    pd.W = (int)W;
    pd.ntiles = (rows + W - 1) / W;
    pd.tiles_inner = 1;
    radix_list(L, pd.radix, &pd.nst);
    if (rowtrans == RT_HALF) {
        p.stage_tab = {2 * (int64_t)L, 2 * (int64_t)L, 1};
        pd.st_mul = 2;
    } else {
        p.stage_tab = {L, L, 1};
        pd.st_mul = 1;
    }
    p.lds_bytes = (size_t)W * pd.lds_stride * c.csz;
    const bool fast_ok = allow_fast && (rowtrans == RT_HALF || rowtrans == RT_C2C) && is_pow2(L) &&
                         L >= kFastMinL && L <= kFastMaxRowL && !tunables().no_fast;
    if (fast_ok) {
        pd.fast = 1;
        pd.logL = ilog2(L);
        const int64_t ntr = kFastMaxRowL / L;
        pd.W = (int)ntr;
        pd.ntiles = (rows + ntr - 1) / ntr;
        pd.lds_stride = L + L / 16 + 2;
        p.lds_bytes = (size_t)ntr * pd.lds_stride * c.csz;
        p.has_fast = true;
        two_level(L, &p.f_lo, &p.f_hi);
        if (rowtrans == RT_HALF) {
            p.has_half = true;
            two_level(2 * (int64_t)L, &p.h_lo, &p.h_hi);
        }
        if (rowtrans == RT_C2C)
            pd.fast_kind = mode == MODE_FWD ? ROW_CFWD : mode == MODE_INV ? ROW_CINV : ROW_MIDC;
        else
            pd.fast_kind = mode == MODE_FWD ? ROW_R2C : mode == MODE_INV ? ROW_C2R : ROW_MIDR;
    }
    int mq = 0, mst = 0;
    int64_t mrad = 0;
    if (!fast_ok && allow_fast &&
        (rowtrans == RT_HALF || (rowtrans == RT_ODD && L % 2 == 1) || (rowtrans == RT_C2C && mode == MODE_MID)) &&
        mixed_family(L, false, c.f64, &mq, &mrad, &mst)) {
        // register mixed-radix rows: P = L / Q threads per row, NTR rows per workgroup
        const int64_t P = L / mq;
        const int64_t LS = L + L / 16 + 2;
        int64_t ntr = std::max<int64_t>(1, 512 / P);
        ntr = std::min<int64_t>(ntr, rows);
        auto bytes = [&](int64_t w) {
            return (size_t)std::max<int64_t>(w * LS, mode == MODE_MID ? 512 * (int64_t)mq : 0) * c.csz;
        };
        // at most ~48 KB of LDS per workgroup, so that three fit a compute unit
        while (ntr > 1 && bytes(ntr) > 48 * 1024) --ntr;
        if (bytes(ntr) <= 128 * 1024) {
            if (mq == 10 && mode == MODE_FWD && rowtrans == RT_HALF && mixed_radix_at(mrad, mst - 1) == 10) {
                // first-pass 10-point rows: two radix-2 middle stages become one guarded
                // radix-4 stage (one LDS exchange fewer; measured faster there, slower in
                // the last pass, whose variant keeps the radix-2 stages)
                std::vector<int> rs, keep;
                int twos = 0;
                for (int i = 1; i + 1 < mst; ++i) {
                    const int x = mixed_radix_at(mrad, i);
                    if (x == 2) ++twos;
                    else keep.push_back(x);
                }
                if (twos >= 2) {
                    rs.push_back(10);
                    rs.insert(rs.end(), keep.begin(), keep.end());
                    for (; twos >= 2; twos -= 2) rs.push_back(4);
                    if (twos) rs.push_back(2);
                    rs.push_back(10);
                    mrad = 0;
                    for (size_t i = 0; i < rs.size(); ++i) mrad |= (int64_t)rs[i] << (kMRadBits * i);
                    mst = (int)rs.size();
                }
            }
            pd.mq = mq;
            pd.mrad = mrad;
            pd.nst = mst;
            for (int i = 0; i < mst; ++i) pd.radix[i] = mixed_radix_at(mrad, i);
            pd.W = (int)ntr;
            pd.mthreads = (int)(ntr * P);
            pd.ntiles = (rows + ntr - 1) / ntr;
            if (rowtrans == RT_C2C)
                pd.fast_kind = ROW_MIDC;
            else if (rowtrans == RT_ODD)
                pd.fast_kind = mode == MODE_FWD ? ROW_R2C_ODD : mode == MODE_INV ? ROW_C2R_ODD : ROW_MIDR_ODD;
            else
                pd.fast_kind = mode == MODE_FWD ? ROW_R2C : mode == MODE_INV ? ROW_C2R : ROW_MIDR;
            p.lds_bytes = bytes(ntr);
        }
    }
    return p;
}

static PassPlan make_col(const Ctx& c, int64_t outer, int L, int64_t inner, int mode, int64_t tw_n, int64_t tw_div,
                         int64_t Wcap) {
    PassPlan p;
    PassDesc& pd = p.pd;
    std::memset(&pd, 0, sizeof(pd));
    pd.kind = PASS_COL;
    pd.mode = mode;
    pd.L = L;
    pd.outer = outer;
    pd.inner = inner;
    pd.kstride = inner;
    pd.ostride = (int64_t)L * inner;
    pd.q_mod = 1;
    int64_t W = pow2_floor(std::max<int64_t>(1, c.budget / L));
    if (Wcap > 0) W = std::min(W, Wcap);
    if (W > inner) W = inner;
    pd.W = (int)W;
    pd.tiles_inner = (inner + W - 1) / W;
    pd.ntiles = outer * pd.tiles_inner;
    radix_list(L, pd.radix, &pd.nst);
    p.stage_tab = {L, L, 1};
    pd.st_mul = 1;
    if (tw_n > 0) {
        pd.tw = 1;
        pd.tw_n = tw_n;
        pd.tw_div = tw_div;
        pd.tw_B = kTwSplit;
        p.has_tw = true;
        p.tw_lo = {tw_n, kTwSplit, 1};
        p.tw_hi = {tw_n, (tw_n + kTwSplit - 1) / kTwSplit, kTwSplit};
    }
    p.lds_bytes = (size_t)L * W * c.csz;
    if (is_pow2(L) && L >= kFastMinL && L <= kFastMaxColL && !tunables().no_fast) {
        pd.fast = 1;
        pd.logL = ilog2(L);
        const int64_t Wf = (col_half(c.f64, ilog2(L)) ? kFastMaxRowL / 2 : kFastMaxRowL) / L;
        pd.W = (int)Wf;
        pd.tiles_inner = (inner + Wf - 1) / Wf;
        pd.ntiles = outer * pd.tiles_inner;
        pd.xcd_remap = 1;
        p.lds_bytes = (size_t)L * (Wf + 1) * c.csz;
        p.has_fast = true;
        two_level(L, &p.f_lo, &p.f_hi);
    } else {
        int mq = 0, mst = 0;
        int64_t mrad = 0, Wm = 0;
        size_t bytes = 0;
        // register mixed-radix columns: P = L / Q threads per column, W columns
        if (mixed_col_fit(L, c.f64, &mq, &mrad, &mst, &Wm, &bytes)) {
            pd.mq = mq;
            pd.mrad = mrad;
            pd.nst = mst;
            for (int i = 0; i < mst; ++i) pd.radix[i] = mixed_radix_at(mrad, i);
            pd.W = (int)Wm;
            pd.mthreads = (int)(Wm * (L / mq));
            pd.tiles_inner = (inner + Wm - 1) / Wm;
            pd.ntiles = outer * pd.tiles_inner;
            pd.xcd_remap = 1;
            p.lds_bytes = bytes;
        }
    }
    return p;
}

static void col_bytes(const Ctx& c, PassPlan& p, int64_t hcount) {
    const PassDesc& pd = p.pd;
    int64_t valid = pd.inner;
    if (pd.cpitch > 0) valid = pd.inner / pd.cpitch * hcount;
    const int64_t elems = pd.outer * pd.L * valid;
    p.model_bytes = elems * ((pd.in_real ? c.esz : c.csz) + (pd.out_real ? c.esz : c.csz));
}

int build_schedule(int d, const int64_t* dims, int64_t B, bool f64, Schedule* S, std::string* why, bool unfused) {
    *S = Schedule();
    S->fused = !unfused;
    S->d = d;
    S->B = B;
    S->f64 = f64;
    if (d < 1 || d > 3 || B < 1) { *why = "ndim must be 1..3"; return -1; }
    for (int a = 0; a < d; ++a) {
        S->dims[a] = dims[a];
        if (dims[a] < 1) { *why = "extents must be >= 1"; return -1; }
        if (!is_7smooth(dims[a])) {
            *why = "extent " + std::to_string(dims[a]) + " has a prime factor above 7";
            return -2;
        }
    }
    Ctx c{f64, f64 ? 8 : 4, f64 ? 16 : 8, f64 ? 4096 : 8192};
    const int64_t col_max = tunables().col_max ? tunables().col_max : 512;
    const int64_t row_max = 4096;                // complex points of a row middle pass
    const int64_t row_single = 8192;             // complex points of one LDS row (any pass)
    SymParams& sp = S->sym;
    std::memset(&sp, 0, sizeof(sp));
    sp.d = d;
    for (int a = 0; a < 3; ++a) sp.n[a] = a < d ? dims[a] : 1;

    if (d == 1 && unfused) {
        // one row: R2C into the workspace, the spectral step, C2R back
        const int64_t n = dims[0];
        const bool half = (n % 2) == 0;
        const int64_t L = half ? n / 2 : n;
        if (L > row_single) {
            *why = "1-D extent " + std::to_string(n) + " exceeds one LDS row";
            return -2;
        }
        const int64_t h = n / 2 + 1;
        const int64_t P = (h + 15) / 16 * 16;
        sp.sdim[0] = P;
        sp.hcount = h;
        sp.nlev[0] = 1;
        sp.sub[0][0] = n;
        S->spec_elems = B * P;
        PassPlan r0 = make_row(c, B, (int)L, half ? RT_HALF : RT_ODD, MODE_FWD, (int)n, (int)h, P);
        r0.pd.in_real = 1;
        r0.model_bytes = B * (n * c.esz + h * c.csz);
        r0.name = "row_fwd_r2c";
        S->passes.push_back(r0);
        S->sym_at = 1;
        PassPlan r1 = make_row(c, B, (int)L, half ? RT_HALF : RT_ODD, MODE_INV, (int)n, (int)h, P);
        r1.pd.out_real = 1;
        r1.model_bytes = B * (n * c.esz + h * c.csz);
        r1.name = "row_inv_c2r";
        S->passes.push_back(r1);
    } else if (d == 1) {
        const int64_t n = dims[0];
        const bool half = (n % 2) == 0;
        const int64_t L = half ? n / 2 : n;
        if (L <= row_single) {
            PassPlan p = make_row(c, B, (int)L, half ? RT_HALF : RT_ODD, MODE_MID, (int)n, (int)(n / 2 + 1), 0);
            p.pd.in_real = p.pd.out_real = 1;
            p.model_bytes = B * 2 * n * c.esz;
            p.name = "row_mid_real";
            S->passes.push_back(p);
            sp.nlev[0] = 1;
            sp.sub[0][0] = n;
            sp.sdim[0] = n;
            S->spec_elems = 0;
        } else {
            const int64_t nr = split_row(n, row_max);
            std::vector<int64_t> lev;
            if (!nr || !split_axis(n / nr, col_max, &lev, f64) || lev.size() > 2) {
                *why = "1-D extent " + std::to_string(n) + " cannot be split into supported factors";
                return -2;
            }
            lev.push_back(nr);
            const int nl = (int)lev.size();
            sp.nlev[0] = nl;
            for (int i = 0; i < nl; ++i) sp.sub[0][i] = lev[i];
            sp.sdim[0] = n;
            S->spec_elems = B * n;
            int64_t pre = 1;
            for (int l = 0; l < nl - 1; ++l) {
                int64_t post = 1;
                for (int i = l + 1; i < nl; ++i) post *= lev[i];
                PassPlan p = make_col(c, B * pre, (int)lev[l], post, MODE_FWD, lev[l] * post, 1, 0);
                if (l == 0) p.pd.in_real = 1;
                col_bytes(c, p, 0);
                p.name = l == 0 ? "col_fwd_real" : "col_fwd";
                S->passes.push_back(p);
                pre *= lev[l];
            }
            PassPlan m = make_row(c, B * pre, (int)nr, RT_C2C, MODE_MID, 0, 0, nr);
            m.pd.q_mod = pre;
            m.model_bytes = B * n * 2 * c.csz;
            m.name = "row_mid_c2c";
            S->passes.push_back(m);
            for (int l = nl - 2; l >= 0; --l) {
                pre /= lev[l];
                int64_t post = 1;
                for (int i = l + 1; i < nl; ++i) post *= lev[i];
                PassPlan p = make_col(c, B * pre, (int)lev[l], post, MODE_INV, lev[l] * post, 1, 0);
                if (l == 0) p.pd.out_real = 1;
                col_bytes(c, p, 0);
                p.name = l == 0 ? "col_inv_real" : "col_inv";
                S->passes.push_back(p);
            }
        }
    } else {
        const int64_t nl = dims[d - 1];
        const bool half = (nl % 2) == 0;
        const int64_t L = half ? nl / 2 : nl;
        if (L > row_single) {
            *why = "last extent " + std::to_string(nl) + " exceeds one LDS row";
            return -2;
        }
        const int64_t h = nl / 2 + 1;
        const int64_t P = (h + 15) / 16 * 16;
        for (int a = 0; a < d - 1; ++a) sp.sdim[a] = dims[a];
        sp.sdim[d - 1] = P;
        sp.hcount = h;
        sp.nlev[d - 1] = 1;
        sp.sub[d - 1][0] = nl;
        int64_t rows = B;
        for (int a = 0; a < d - 1; ++a) rows *= dims[a];
        S->spec_elems = rows * P;

        std::vector<std::vector<int64_t>> lev(d);
        for (int a = 0; a < d - 1; ++a) {
            if (!split_axis(dims[a], col_max, &lev[a], f64)) {
                *why = "extent " + std::to_string(dims[a]) + " cannot be split into supported factors";
                return -2;
            }
            sp.nlev[a] = (int)lev[a].size();
            for (size_t i = 0; i < lev[a].size(); ++i) sp.sub[a][i] = lev[a][i];
        }

        PassPlan r0 = make_row(c, rows, (int)L, half ? RT_HALF : RT_ODD, MODE_FWD, (int)nl, (int)h, P);
        r0.pd.in_real = 1;
        r0.model_bytes = rows * (nl * c.esz + h * c.csz);
        r0.name = "row_fwd_r2c";
        S->passes.push_back(r0);

        auto outer_of = [&](int a) {
            int64_t o = B;
            for (int b = 0; b < a; ++b) o *= sp.sdim[b];
            return o;
        };
        auto inner_of = [&](int a) {
            int64_t i = 1;
            for (int b = a + 1; b < d; ++b) i *= sp.sdim[b];
            return i;
        };
        auto level_pass = [&](int a, int l, int mode) {
            const auto& s = lev[a];
            const int nlv = (int)s.size();
            int64_t pre = 1, post = 1;
            for (int i = 0; i < l; ++i) pre *= s[i];
            for (int i = l + 1; i < nlv; ++i) post *= s[i];
            const bool tw = (mode != MODE_MID) && (l < nlv - 1);
            PassPlan p = make_col(c, outer_of(a) * pre, (int)s[l], post * inner_of(a), mode,
                                  tw ? s[l] * post : 0, inner_of(a), mode == MODE_MID ? 64 : 0);
            p.pd.cpitch = P;
            p.pd.hcount = (int)h;
            if (mode == MODE_MID) p.pd.q_mod = pre;
            col_bytes(c, p, h);
            p.name = mode == MODE_MID ? "col_mid" : (mode == MODE_FWD ? "col_fwd" : "col_inv");
            return p;
        };
        for (int a = d - 2; a >= 1; --a) {
            if (dims[a] == 1) continue;
            for (int l = 0; l < (int)lev[a].size(); ++l) S->passes.push_back(level_pass(a, l, MODE_FWD));
        }
        const int n0 = (int)lev[0].size();
        if (unfused) {
            if (dims[0] > 1)
                for (int l = 0; l < n0; ++l) S->passes.push_back(level_pass(0, l, MODE_FWD));
            S->sym_at = (int)S->passes.size();
            if (dims[0] > 1)
                for (int l = n0 - 1; l >= 0; --l) S->passes.push_back(level_pass(0, l, MODE_INV));
        } else {
            for (int l = 0; l < n0 - 1; ++l) S->passes.push_back(level_pass(0, l, MODE_FWD));
            S->passes.push_back(level_pass(0, n0 - 1, MODE_MID));
            for (int l = n0 - 2; l >= 0; --l) S->passes.push_back(level_pass(0, l, MODE_INV));
        }
        for (int a = 1; a <= d - 2; ++a) {
            if (dims[a] == 1) continue;
            for (int l = (int)lev[a].size() - 1; l >= 0; --l) S->passes.push_back(level_pass(a, l, MODE_INV));
        }
        PassPlan r1 = make_row(c, rows, (int)L, half ? RT_HALF : RT_ODD, MODE_INV, (int)nl, (int)h, P);
        r1.pd.out_real = 1;
        r1.model_bytes = rows * (nl * c.esz + h * c.csz);
        r1.name = "row_inv_c2r";
        S->passes.push_back(r1);
    }
    for (auto& p : S->passes) {
        p.pd.d = d;
        p.pd.B = B;
        for (int a = 0; a < 3; ++a) p.pd.rdims[a] = a < d ? dims[a] : 1;
        S->model_bytes += p.model_bytes;
    }
    return 0;
}

int axis_schedule(int64_t outer, int64_t n, int64_t inner, bool f64, bool inverse, std::vector<PassPlan>* out,
                  std::vector<int64_t>* levels, std::string* why) {
    out->clear();
    levels->clear();
    if (outer < 1 || n < 1 || inner < 1) { *why = "extents must be >= 1"; return -1; }
    if (!is_7smooth(n)) { *why = "transform length " + std::to_string(n) + " is not 7-smooth"; return -2; }
    Ctx c{f64, f64 ? 8 : 4, f64 ? 16 : 8, f64 ? 4096 : 8192};
    const int64_t col_max = tunables().col_max ? tunables().col_max : 512;
    const int64_t row_max = 4096, row_single = 8192;
    std::vector<int64_t> lev;
    bool last_row = false;  // the last level runs as a row pass (contiguous axis)
    if (n == 1) {
        lev.push_back(1);
    } else if (inner == 1 && n <= row_single && !(is_pow2(n) && n > kFastMaxRowL)) {
        lev.push_back(n);
        last_row = true;
    } else if (inner == 1) {
        // (a power of two above the register row kernels' limit splits off
        // strided levels so that its row level stays on them)
        const int64_t nr = split_row(n, row_max);
        if (!nr || !split_axis(n / nr, col_max, &lev, f64) || lev.size() > 2) {
            *why = "length " + std::to_string(n) + " cannot be split into supported factors";
            return -2;
        }
        lev.push_back(nr);
        last_row = true;
    } else if (!split_axis(n, col_max, &lev, f64)) {
        *why = "length " + std::to_string(n) + " cannot be split into supported factors";
        return -2;
    }
    *levels = lev;
    if (n == 1) return 0;  // identity
    const int nl = (int)lev.size();
    auto level = [&](int l) {
        int64_t pre = 1, post = 1;
        for (int i = 0; i < l; ++i) pre *= lev[i];
        for (int i = l + 1; i < nl; ++i) post *= lev[i];
        const int mode = inverse ? MODE_INV : MODE_FWD;
        if (l == nl - 1 && last_row) {
            PassPlan p = make_row(c, outer * pre, (int)lev[l], RT_C2C, mode, (int)lev[l], (int)lev[l], lev[l]);
            p.model_bytes = outer * n * 2 * c.csz;
            p.name = inverse ? "axis_inv_row" : "axis_fwd_row";
            return p;
        }
        const bool tw = l < nl - 1;
        PassPlan p = make_col(c, outer * pre, (int)lev[l], post * inner, mode, tw ? lev[l] * post : 0, inner, 0);
        col_bytes(c, p, 0);
        p.name = inverse ? "axis_inv" : "axis_fwd";
        return p;
    };
    if (!inverse)
        for (int l = 0; l < nl; ++l) out->push_back(level(l));
    else
        for (int l = nl - 1; l >= 0; --l) out->push_back(level(l));
    for (auto& p : *out) {
        p.pd.d = 1;
        p.pd.B = 1;
        for (int a = 0; a < 3; ++a) p.pd.rdims[a] = 1;
    }
    return 0;
}

std::string describe_schedule(const Schedule& s) {
    std::ostringstream o;
    o << "{\"ndim\": " << s.d << ", \"dims\": [";
    for (int a = 0; a < s.d; ++a) o << (a ? ", " : "") << s.dims[a];
    o << "], \"batch\": " << s.B << ", \"dtype\": \"" << (s.f64 ? "f64" : "f32") << "\""
      << ", \"spectrum_elems\": " << s.spec_elems << ", \"model_bytes\": " << s.model_bytes << ", \"passes\": [";
    for (size_t i = 0; i < s.passes.size(); ++i) {
        const PassPlan& p = s.passes[i];
        const PassDesc& pd = p.pd;
        o << (i ? ", " : "") << "{\"name\": \"" << p.name << "\", \"kind\": \""
          << (pd.kind == PASS_ROW ? "row" : "col") << "\", \"mode\": \""
          << (pd.mode == MODE_FWD ? "fwd" : pd.mode == MODE_INV ? "inv" : "mid") << "\", \"L\": " << pd.L
          << ", \"fast\": " << pd.fast << ", \"mixed_q\": " << pd.mq << ", \"W\": " << pd.W << ", \"outer\": " << pd.outer << ", \"inner\": " << pd.inner
          << ", \"tiles\": " << pd.ntiles << ", \"twiddle\": " << pd.tw << ", \"lds_bytes\": " << p.lds_bytes
          << ", \"model_bytes\": " << p.model_bytes << ", \"radices\": [";
        for (int k = 0; k < pd.nst; ++k) o << (k ? ", " : "") << pd.radix[k];
        o << "]}";
    }
    o << "], \"levels\": [";
    for (int a = 0; a < s.d; ++a) {
        o << (a ? ", " : "") << "[";
        for (int l = 0; l < s.sym.nlev[a]; ++l) o << (l ? ", " : "") << s.sym.sub[a][l];
        o << "]";
    }
    o << "]}";
    return o.str();
}

}  // namespace sfft
