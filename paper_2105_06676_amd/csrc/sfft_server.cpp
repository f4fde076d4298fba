// Serving loop: continuous batching of stencil solves on one GPU.
//
// submit() copies a request into a FIFO and returns a ticket.  A worker thread
// admits requests in arrival order while a slot is free and the request's
// workspace fits what is left of the HBM budget (one device arena allocated
// at creation, first-fit), packs the admitted requests into one batched
// program on a free stream, and retires a batch when its completion event has
// fired: tickets become done, slots and arena space return.  Requests that
// arrive while batches run therefore join the next batch, and batches on
// different streams overlap on the device.
//
// Device memory: the whole budget is one arena allocated at creation.  It holds
// each stream's descriptor buffer (reserved at creation) and, per admitted
// request, one block with everything the request's solve needs: the spectrum
// workspace and column table of a periodic request, every buffer of an
// aperiodic one (its size found on the host at submit by the solver's own
// bookkeeping with nothing enqueued).  Serving therefore allocates nothing and
// never synchronises the device after creation.
#include <algorithm>
#include <functional>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <sstream>
#include <thread>

#include "sfft_batch.h"
#include "sfft_solvers.h"

namespace sfft {
int guarded_call(const std::function<void()>& f);
}  // namespace sfft

using namespace sfft;

namespace {

using Clock = std::chrono::steady_clock;

// passes per request the descriptor reserve is sized for (the deepest
// schedules have 9); a request with more is rejected at submit
constexpr size_t kDescPasses = 12;

struct Req {
    uint64_t ticket;
    sfft_problem p;
    std::vector<double> coeffs;
    size_t bytes;          // arena block: the request's device buffers
    size_t desc_bytes;     // its share of a batch's descriptor buffer
    int64_t model_bytes;   // algorithmic HBM bytes of its passes (batched requests)
    bool batched;          // runs in the batched launches (else solved on its own)
};

// first-fit allocator over [0, cap)
struct Arena {
    size_t cap = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void init(size_t c) {
        cap = c;
        free_.clear();
        free_[0] = c;
    }
    bool alloc(size_t n, size_t* off) {
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t o2 = it->first + n;
                free_.erase(it);
                if (rest) free_[o2] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) / 256 * 256;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Flight {
    int stream;
    hipEvent_t start = nullptr, done = nullptr;  // timing events around the batch's work
    std::vector<uint64_t> tickets;
    std::vector<std::pair<size_t, size_t>> allocs;
    int64_t model_bytes = 0;
    bool all_periodic = true;
};

// Device-time span of one retired batch (ms since the server's base event).
struct Span {
    double t0, t1;
    int64_t bytes;
    bool periodic;
};

struct TicketInfo {
    int status = 1;  // 1 pending, 0 done, < 0 error
    double t_submit = 0, t_done = 0;
};

}  // namespace

struct sfft_server {
    int device = 0;
    uint64_t budget = 0;
    int max_slots = 64;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> queue;
    std::map<uint64_t, TicketInfo> tickets;
    uint64_t next_ticket = 1;
    std::vector<hipStream_t> streams;
    std::vector<char*> desc;   // per stream, inside the arena
    size_t desc_cap = 0;
    hipEvent_t base_ev = nullptr;
    std::vector<Span> spans;
    std::vector<int> stream_busy;
    std::vector<Flight> flights;
    char* arena_base = nullptr;
    Arena arena;
    size_t in_use = 0, peak_use = 0;
    int inflight_reqs = 0;
    uint64_t n_admitted = 0, n_completed = 0, n_batches = 0, max_batch = 0;
    bool stop = false;
    std::thread worker;
    Clock::time_point t0 = Clock::now();

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    size_t reserved() const { return streams.size() * ((desc_cap + 255) / 256 * 256); }
    void run();
    void launch(int si, std::vector<Req>& reqs, std::vector<size_t>& offs);
};

void sfft_server::launch(int si, std::vector<Req>& reqs, std::vector<size_t>& offs) {
    hipStream_t st = streams[si];
    std::vector<ProblemRun> runs;
    std::vector<int> which;
    for (size_t i = 0; i < reqs.size(); ++i)
        if (reqs[i].batched && reqs[i].p.T > 0) {
            runs.push_back(prepare_periodic(reqs[i].p));
            which.push_back((int)i);
        }
    if (!runs.empty()) {
        // every admitted request owns an arena block holding its workspace and
        // column table; admission kept the batch's descriptors within the
        // stream's reserved buffer
        BatchMem mem;
        mem.desc = desc[si];
        mem.desc_cap = desc_cap;
        std::vector<char*> bases;
        for (int k : which) bases.push_back(arena_base + offs[k]);
        BatchProgram prog = build_batch(runs, mem, &bases);
        enqueue_batch(prog, runs, mem, st, true);
    }
    // the others, each in its own arena block
    for (size_t i = 0; i < reqs.size(); ++i) {
        const Req& r = reqs[i];
        if (r.batched || r.p.T == 0) continue;
        const bool f64 = r.p.dtype == SFFT_F64;
        void* pool = arena_base + offs[i];
        if (r.p.aperiodic)
            solve_aperiodic_pooled(r.p.grid, f64, r.p.ndim, r.p.dims, r.coeffs.data(), r.p.radius, r.p.T,
                                   r.p.aperiodic - 1, st, pool, r.bytes);
        else if (r.p.radius > kMaxR)
            solve_periodic_general(r.p.grid, f64, r.p.ndim, r.p.dims, r.coeffs.data(), r.p.radius, r.p.T, st, pool);
        else
            solve_periodic_any(r.p.grid, f64, r.p.ndim, r.p.dims, r.coeffs.data(), r.p.radius, r.p.T, st, pool);
    }
}

// Bytes of the descriptor buffer a batch of requests with these shares needs
// (the layout of batch_desc_bytes: symbol parameters, then the work lists).
static size_t desc_need(size_t nreq, size_t items) {
    return (sizeof(SymParams) * std::max<size_t>(1, nreq) + 255) / 256 * 256 +
           sizeof(BatchItem) * std::max<size_t>(1, items) + 256;
}

void sfft_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // retire finished batches
        for (size_t i = 0; i < flights.size();) {
            Flight& f = flights[i];
            const hipError_t q = hipEventQuery(f.done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            const int status = q == hipSuccess ? 0 : SFFT_EHIP;
            const double t = now();
            if (status == 0) {
                float a = 0.f, b = 0.f;
                if (hipEventElapsedTime(&a, base_ev, f.start) == hipSuccess &&
                    hipEventElapsedTime(&b, base_ev, f.done) == hipSuccess)
                    spans.push_back({a, b, f.model_bytes, f.all_periodic});
                else
                    (void)hipGetLastError();
            }
            for (uint64_t tk : f.tickets) {
                auto& ti = tickets[tk];
                ti.status = status;
                ti.t_done = t;
            }
            for (auto& a : f.allocs) {
                arena.release(a.first, a.second);
                in_use -= (a.second + 255) / 256 * 256;
            }
            inflight_reqs -= (int)f.tickets.size();
            n_completed += f.tickets.size();
            stream_busy[f.stream] = 0;
            (void)hipEventDestroy(f.start);
            (void)hipEventDestroy(f.done);
            flights.erase(flights.begin() + i);
            cv_done.notify_all();
        }
        // admit and launch
        int si = -1;
        for (size_t k = 0; k < streams.size(); ++k)
            if (!stream_busy[k]) { si = (int)k; break; }
        if (si >= 0 && !queue.empty()) {
            std::vector<Req> adm;
            std::vector<size_t> offs;
            std::vector<std::pair<size_t, size_t>> allocs;
            size_t nper = 0, items = 0;
            while (!queue.empty() && inflight_reqs + (int)adm.size() < max_slots) {
                Req& r = queue.front();
                const size_t add_items = r.batched ? r.desc_bytes / sizeof(BatchItem) : 0;
                if (r.batched && desc_need(nper + 1, items + add_items) > desc_cap) break;
                size_t off = 0;
                if (!arena.alloc(std::max<size_t>(r.bytes, 256), &off)) break;
                if (r.batched) {
                    nper += 1;
                    items += add_items;
                }
                in_use += (std::max<size_t>(r.bytes, 256) + 255) / 256 * 256;
                peak_use = std::max(peak_use, in_use);
                allocs.push_back({off, std::max<size_t>(r.bytes, 256)});
                offs.push_back(off);
                adm.push_back(std::move(r));
                queue.pop_front();
            }
            if (!adm.empty()) {
                Flight f;
                f.stream = si;
                f.allocs = allocs;
                for (auto& r : adm) {
                    f.tickets.push_back(r.ticket);
                    // requests point at their own coefficient copies
                    r.p.coeffs = r.coeffs.data();
                    f.model_bytes += r.model_bytes;
                    f.all_periodic = f.all_periodic && r.batched;
                }
                stream_busy[si] = 1;
                inflight_reqs += (int)adm.size();
                n_admitted += adm.size();
                n_batches += 1;
                max_batch = std::max<uint64_t>(max_batch, adm.size());
                lk.unlock();
                int status = 0;
                hipEvent_t ev0 = nullptr;
                (void)hipEventCreate(&ev0);
                (void)hipEventRecord(ev0, streams[si]);
                try {
                    launch(si, adm, offs);
                } catch (const Error& e) {
                    status = e.code;
                } catch (...) {
                    status = SFFT_EHIP;
                }
                hipEvent_t ev;
                (void)hipEventCreate(&ev);
                (void)hipEventRecord(ev, streams[si]);
                lk.lock();
                f.start = ev0;
                f.done = ev;
                if (status) {
                    // failed to enqueue: finish these tickets with the error at once
                    (void)hipStreamSynchronize(streams[si]);
                    for (uint64_t tk : f.tickets) {
                        tickets[tk].status = status;
                        tickets[tk].t_done = now();
                    }
                    for (auto& a : f.allocs) {
                        arena.release(a.first, a.second);
                        in_use -= (a.second + 255) / 256 * 256;
                    }
                    inflight_reqs -= (int)f.tickets.size();
                    stream_busy[si] = 0;
                    (void)hipEventDestroy(ev0);
                    (void)hipEventDestroy(ev);
                    cv_done.notify_all();
                } else {
                    flights.push_back(std::move(f));
                }
                continue;
            }
        }
        if (stop && queue.empty() && flights.empty()) break;
        cv_work.wait_for(lk, std::chrono::microseconds(flights.empty() ? 2000 : 50));
    }
}

namespace {

// Device-time statistics of the retired batches: the union of their spans (GPU
// busy time), their sum (> union when batches on different streams overlapped),
// the most batches in flight at once on the device, and each periodic batch's
// algorithmic HBM bytes over its own span against 8 TB/s.
std::string span_stats(const std::vector<Span>& sp) {
    std::vector<std::pair<double, int>> ev;
    double sum = 0.0;
    int64_t bytes = 0;
    std::vector<double> frac;
    for (auto& x : sp) {
        ev.push_back({x.t0, 1});
        ev.push_back({x.t1, -1});
        sum += x.t1 - x.t0;
        if (x.periodic && x.t1 > x.t0) {
            frac.push_back((double)x.bytes / ((x.t1 - x.t0) * 1e-3) / 8e12);
            bytes += x.bytes;
        }
    }
    std::sort(ev.begin(), ev.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        return a.first != b.first ? a.first < b.first : a.second < b.second;
    });
    int cur = 0, mx = 0;
    double uni = 0.0, last = 0.0;
    for (auto& e : ev) {
        if (cur > 0) uni += e.first - last;
        cur += e.second;
        mx = std::max(mx, cur);
        last = e.first;
    }
    std::sort(frac.begin(), frac.end());
    auto pct = [&](double q) { return frac.empty() ? 0.0 : frac[(size_t)std::min<double>(frac.size() - 1, q * frac.size())]; };
    std::ostringstream o;
    o.precision(6);
    o << "\"device\": {\"batches_timed\": " << sp.size() << ", \"busy_ms\": " << uni << ", \"sum_batch_ms\": " << sum
      << ", \"max_concurrent_batches\": " << mx << ", \"periodic_model_bytes\": " << bytes
      << ", \"hbm_frac_of_busy\": " << (uni > 0 ? (double)bytes / (uni * 1e-3) / 8e12 : 0.0)
      << ", \"batch_hbm_frac_p10\": " << pct(0.1) << ", \"batch_hbm_frac_p50\": " << pct(0.5)
      << ", \"batch_hbm_frac_p90\": " << pct(0.9) << "}";
    return o.str();
}

}  // namespace

extern "C" {

int sfft_server_create(sfft_server** out, int device, uint64_t hbm_budget_bytes, int max_slots) {
    return guarded_call([&] {
        if (!out) throw Error(SFFT_EINVAL, "out is null");
        *out = nullptr;
        int ndev = 0;
        check_hip(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (device < 0 || device >= ndev) throw Error(SFFT_EINVAL, "no such device");
        std::unique_ptr<sfft_server> s(new sfft_server());
        s->device = device;
        s->budget = hbm_budget_bytes ? hbm_budget_bytes : (32ull << 30);
        s->max_slots = max_slots > 0 ? max_slots : 64;
        int prev = 0;
        check_hip(hipGetDevice(&prev), "hipGetDevice");
        check_hip(hipSetDevice(device), "hipSetDevice");
        hipError_t e = hipMalloc(&s->arena_base, s->budget);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipSetDevice(prev);
            throw Error(SFFT_ENOMEM, "HBM budget of " + std::to_string(s->budget) + " bytes: " + hipGetErrorString(e));
        }
        s->arena.init(s->budget);
        const int nst = 4;
        // descriptor buffers, reserved from the budget: room for a full batch of
        // requests of up to kDescPasses passes each (admission keeps every batch
        // within it)
        s->desc_cap = desc_need((size_t)s->max_slots, (size_t)s->max_slots * kDescPasses);
        for (int i = 0; i < nst; ++i) {
            hipStream_t st;
            check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
            s->streams.push_back(st);
            size_t off = 0;
            if (!s->arena.alloc(s->desc_cap, &off)) {
                (void)hipSetDevice(prev);
                throw Error(SFFT_ENOMEM, "HBM budget of " + std::to_string(s->budget) +
                                             " bytes is smaller than the descriptor reserve of " +
                                             std::to_string(nst * s->desc_cap) + " bytes");
            }
            s->in_use += (s->desc_cap + 255) / 256 * 256;
            s->desc.push_back(s->arena_base + off);
            s->stream_busy.push_back(0);
        }
        s->peak_use = s->in_use;
        check_hip(hipEventCreate(&s->base_ev), "hipEventCreate");
        check_hip(hipEventRecord(s->base_ev, s->streams[0]), "hipEventRecord");
        check_hip(hipEventSynchronize(s->base_ev), "hipEventSynchronize");
        (void)hipSetDevice(prev);
        sfft_server* raw = s.get();
        s->worker = std::thread([raw] { raw->run(); });
        *out = s.release();
    });
}

int sfft_server_submit(sfft_server* s, const sfft_problem* p, uint64_t* ticket) {
    return guarded_call([&] {
        if (!s || !p || !ticket) throw Error(SFFT_EINVAL, "null argument");
        validate_problem(*p);
        Req r;
        r.p = *p;
        int nc = 1;
        for (int a = 0; a < p->ndim; ++a) nc *= 2 * p->radius + 1;
        r.coeffs.assign(p->coeffs, p->coeffs + nc);
        r.p.coeffs = r.coeffs.data();
        r.model_bytes = 0;
        r.desc_bytes = 0;
        r.batched = batchable(*p);
        const bool f64 = p->dtype == SFFT_F64;
        if (p->aperiodic) {
            // every buffer of the solve, sized by its own bookkeeping on the host
            r.bytes = aperiodic_footprint(f64, p->ndim, p->dims, r.coeffs.data(), p->radius, p->T, p->aperiodic - 1);
        } else if (!r.batched) {
            r.bytes = p->radius > kMaxR ? periodic_general_footprint(f64, p->ndim, p->dims, p->radius)
                                        : periodic_any_footprint(f64, p->ndim, p->dims);
        } else {
            const ProblemSize ps = problem_size(*p);
            r.bytes = ps.ws_bytes;
            r.model_bytes = ps.model_bytes;
            r.desc_bytes = ps.passes * sizeof(BatchItem);
            if (desc_need(1, ps.passes) > s->desc_cap)
                throw Error(SFFT_EUNSUPPORTED, "request has more passes than a server batch holds");
        }
        if (r.bytes > s->budget - s->reserved())
            throw Error(SFFT_ENOMEM, "request workspace exceeds the server's HBM budget");
        std::lock_guard<std::mutex> g(s->mu);
        r.ticket = s->next_ticket++;
        TicketInfo ti;
        ti.t_submit = s->now();
        s->tickets[r.ticket] = ti;
        *ticket = r.ticket;
        s->queue.push_back(std::move(r));
        s->cv_work.notify_one();
    });
}

int sfft_server_poll(sfft_server* s, uint64_t ticket, int* done) {
    if (!s || !done) return SFFT_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return SFFT_ENOTFOUND;
    if (it->second.status < 0) return it->second.status;
    *done = it->second.status == 0 ? 1 : 0;
    return SFFT_OK;
}

int sfft_server_wait(sfft_server* s, uint64_t ticket) {
    if (!s) return SFFT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return SFFT_ENOTFOUND;
    s->cv_done.wait(lk, [&] { return s->tickets[ticket].status != 1; });
    return s->tickets[ticket].status;
}

int sfft_server_ticket_times(sfft_server* s, uint64_t ticket, double* submit_s, double* done_s) {
    if (!s || !submit_s || !done_s) return SFFT_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return SFFT_ENOTFOUND;
    *submit_s = it->second.t_submit;
    *done_s = it->second.status == 1 ? -1.0 : it->second.t_done;
    return SFFT_OK;
}

int sfft_server_stats(sfft_server* s, char* buf, int64_t cap) {
    if (!s || !buf || cap < 1) return SFFT_EINVAL;
    std::ostringstream o;
    {
        std::lock_guard<std::mutex> g(s->mu);
        o << "{\"admitted\": " << s->n_admitted << ", \"completed\": " << s->n_completed << ", \"batches\": "
          << s->n_batches << ", \"max_batch\": " << s->max_batch << ", \"queued\": " << s->queue.size()
          << ", \"in_flight\": " << s->inflight_reqs << ", \"budget_bytes\": " << s->budget
          << ", \"reserved_bytes\": " << s->reserved()
          << ", \"peak_bytes\": " << s->peak_use << ", \"streams\": " << s->streams.size()
          << ", \"max_slots\": " << s->max_slots << ", " << span_stats(s->spans) << "}";
    }
    const std::string str = o.str();
    if ((int64_t)str.size() >= cap) return SFFT_EINVAL;
    std::memcpy(buf, str.c_str(), str.size() + 1);
    return (int)str.size();
}

void sfft_server_destroy(sfft_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (s->base_ev) (void)hipEventDestroy(s->base_ev);
    if (s->arena_base) (void)hipFree(s->arena_base);
    (void)hipSetDevice(prev);
    delete s;
}

}  // extern "C"
