// Serving loop: continuous batching of DCT / IDCT / Poisson requests of uneven
// sizes on one GPU.
//
// A scheduler thread owns a private library handle, `nstreams` HIP streams
// (default priority) and one device pool of `hbm_budget` bytes, from which it
// carves each batch's workspace (first fit, coalescing free list).  Requests
// carry an arrival time; once arrived they wait in FIFO order and are admitted
// while (a) fewer than max_inflight requests are on the GPU and (b) their
// workspace fits in the pool.  Every scheduler pass turns the admitted requests
// into one batch (the persistent per-pass launches of the batched submit) on
// the next stream, so requests arriving while earlier batches run are admitted
// as soon as slots and memory free up, and batches on different streams
// overlap on the device.  Completion is observed through one event per batch;
// latency = completion observed - arrival, on the host's steady clock.
// Inside a batch, requests of one kind and shape run each pass as one launch
// of the compile-time kernels with a grid layer per request (the launches of
// the plain call, so a result is bitwise the same alone and in a batch), and
// small requests of any shape share the persistent batch passes.  While
// batches are on the GPU a new one starts only once min_batch requests wait
// (or the GPU has gone idle, or the oldest waiting request has waited
// max_wait_us), so arrivals during a busy period are gathered into batches
// instead of being launched one by one, and a lone request at low load is not
// held back for long.  In plain mode the same
// loop launches every request by itself with its plain entry point, in
// arrival order, on one stream (the per-request baseline).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "dctx.h"

namespace dctx {
dctx_status rt_check_desc(const dctx_desc &d);
size_t rt_footprint(const dctx_desc &d);
dctx_status rt_run_batch(dctx_context *h, const dctx_desc *d, int count, hipStream_t s, void *ws, size_t ws_cap);
dctx_status rt_run_plain(dctx_context *h, const dctx_desc &d, hipStream_t s, void *ws);
}  // namespace dctx

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device range, offsets aligned to 256 bytes.
class Pool {
  public:
    void reset(size_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
        cap_ = bytes;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, o = it->first + bytes;
                free_.erase(it);
                if (rest) free_[o] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
    size_t capacity() const { return cap_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Req {
    dctx_desc d;
    size_t footprint = 0;
    double arrival = 0.0, launch = -1.0, done = -1.0;
    int batch = 0;
    dctx_status status = DCTX_ERR_BUSY;
};

struct Flight {
    hipEvent_t ev = nullptr;
    std::vector<uint64_t> reqs;
    size_t off = 0, bytes = 0;
};

}  // namespace

struct dctx_server_s {
    dctx_server_config cfg{};
    dctx_handle h = nullptr;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    void *pool_mem = nullptr;
    Pool pool;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<Req> reqs;                         // by ticket
    std::vector<std::pair<double, uint64_t>> future;   // (arrival, ticket) not yet arrived, min-heap
    std::deque<uint64_t> ready;                    // arrived, FIFO
    std::vector<Flight> flights;
    int inflight = 0;
    uint64_t outstanding = 0;                      // submitted, not done
    int64_t batches = 0, batched_reqs = 0;
    int inject_fail = 0;                           // batches still to fail (failure injection)
    dctx_status fatal = DCTX_OK;
    std::atomic<bool> stop{false};
    std::thread th;
    std::vector<hipEvent_t> ev_pool;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

hipEvent_t take_ev(dctx_server_s *s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// One scheduler pass (called with the lock held; releases it around GPU calls
// that may block).  Returns true if it made progress.
bool step(dctx_server_s *s, std::unique_lock<std::mutex> &lk) {
    bool progress = false;
    const double t = s->now();
    // completions
    for (size_t i = 0; i < s->flights.size();) {
        Flight &f = s->flights[i];
        const hipError_t q = hipEventQuery(f.ev);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        const dctx_status st = q == hipSuccess ? DCTX_OK : DCTX_ERR_DEVICE;
        for (uint64_t tk : f.reqs) {
            Req &r = s->reqs[tk];
            r.done = t;
            r.status = st;
            s->outstanding--;
        }
        s->inflight -= (int)f.reqs.size();
        if (f.bytes) s->pool.release(f.off, f.bytes);
        s->ev_pool.push_back(f.ev);
        s->flights.erase(s->flights.begin() + i);
        progress = true;
        s->cv_done.notify_all();
    }
    // arrivals
    while (!s->future.empty() && s->future.front().first <= t) {
        std::pop_heap(s->future.begin(), s->future.end(), std::greater<std::pair<double, uint64_t>>());
        s->ready.push_back(s->future.back().second);
        s->future.pop_back();
        progress = true;
    }
    // admission: one batch (or one plain request) per stream while slots and
    // memory allow; while batches run, a new one waits for min_batch requests
    // or until the oldest waiting request has waited max_wait_us
    const int max_batch = s->cfg.plain ? 1 : std::max(1, s->cfg.max_batch);
    while (!s->ready.empty() && s->inflight < s->cfg.max_inflight &&
           (int)s->flights.size() < (s->cfg.plain ? s->cfg.max_inflight : 2 * (int)s->streams.size())) {
        if (!s->cfg.plain && !s->flights.empty() && (int)s->ready.size() < std::min(s->cfg.min_batch, max_batch)) {
            const double waited = t - s->reqs[s->ready.front()].arrival;
            if (s->cfg.max_wait_us < 0 || waited * 1e6 < s->cfg.max_wait_us) break;
        }
        std::vector<uint64_t> take;
        size_t bytes = 0;
        while (!s->ready.empty() && (int)take.size() < max_batch &&
               s->inflight + (int)take.size() < s->cfg.max_inflight) {
            const Req &r = s->reqs[s->ready.front()];
            const size_t need = s->cfg.plain ? 0 : r.footprint;
            if (need && s->pool.largest_free() < bytes + need) break;
            bytes += need;
            take.push_back(s->ready.front());
            s->ready.pop_front();
        }
        if (take.empty()) break;   // the FIFO head does not fit yet
        Flight f;
        f.reqs = take;
        f.bytes = bytes;
        if (bytes && !s->pool.alloc(bytes, &f.off)) {
            for (auto it = take.rbegin(); it != take.rend(); ++it) s->ready.push_front(*it);
            break;
        }
        std::vector<dctx_desc> ds;
        ds.reserve(take.size());
        const double tl = s->now();
        for (uint64_t tk : take) {
            s->reqs[tk].launch = tl;
            s->reqs[tk].batch = (int)take.size();
            ds.push_back(s->reqs[tk].d);
        }
        hipStream_t st = s->streams[s->next_stream];
        s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
        f.ev = take_ev(s);
        s->inflight += (int)take.size();
        s->batches += 1;
        s->batched_reqs += (int64_t)take.size();
        void *ws = static_cast<char *>(s->pool_mem) + f.off;
        const bool fail_now = s->inject_fail > 0;
        if (fail_now) s->inject_fail--;
        lk.unlock();
        dctx_status rs = DCTX_OK;
        if (fail_now)
            rs = DCTX_ERR_NOMEM;   // injected: nothing enqueued
        else if (s->cfg.plain)
            rs = dctx::rt_run_plain(s->h, ds[0], st, nullptr);
        else
            rs = dctx::rt_run_batch(s->h, ds.data(), (int)ds.size(), st, ws, bytes);
        hipError_t e = f.ev ? hipEventRecord(f.ev, st) : hipErrorOutOfMemory;
        lk.lock();
        if (rs != DCTX_OK || e != hipSuccess) {
            // the work may be partly enqueued: wait for the stream, then fail the requests
            lk.unlock();
            (void)hipStreamSynchronize(st);
            lk.lock();
            for (uint64_t tk : take) {
                s->reqs[tk].status = rs != DCTX_OK ? rs : DCTX_ERR_DEVICE;
                s->reqs[tk].done = s->now();
                s->outstanding--;
            }
            s->inflight -= (int)take.size();
            if (f.bytes) s->pool.release(f.off, f.bytes);
            if (f.ev) s->ev_pool.push_back(f.ev);
            s->cv_done.notify_all();
        } else {
            s->flights.push_back(f);
        }
        progress = true;
    }
    return progress;
}

void loop(dctx_server_s *s) {
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop.load()) {
        const bool progress = step(s, lk);
        if (progress) continue;
        if (s->flights.empty()) {
            // nothing on the GPU: sleep until the next arrival or a submit
            if (s->future.empty() && s->ready.empty()) {
                s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
            } else if (!s->future.empty() && s->ready.empty()) {
                const double dt = s->future.front().first - s->now();
                if (dt > 0) s->cv_work.wait_for(lk, std::chrono::duration<double>(std::min(dt, 0.05)));
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(10));
            lk.lock();
        }
    }
}

void server_free(dctx_server_s *s) {
    if (s->th.joinable()) {
        s->stop.store(true);
        s->cv_work.notify_all();
        s->th.join();
    }
    for (auto &f : s->flights) (void)hipEventSynchronize(f.ev);
    for (auto &f : s->flights) (void)hipEventDestroy(f.ev);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (s->pool_mem) (void)hipFree(s->pool_mem);
    if (s->h) (void)dctx_destroy(s->h);
    delete s;
}

}  // namespace

extern "C" {

dctx_status dctx_server_create(const dctx_server_config *cfg, dctx_server *out) {
    if (!cfg || !out) return DCTX_ERR_INVALID;
    *out = nullptr;
    if (cfg->max_inflight < 1 || cfg->nstreams < 1 || cfg->nstreams > 16 || cfg->max_batch < 0 ||
        cfg->min_batch < 0 || (cfg->plain != 0 && cfg->plain != 1))
        return DCTX_ERR_INVALID;
    dctx_server_s *s = new (std::nothrow) dctx_server_s();
    if (!s) return DCTX_ERR_NOMEM;
    s->cfg = *cfg;
    if (s->cfg.max_batch == 0) s->cfg.max_batch = 1024;
    if (s->cfg.min_batch == 0) s->cfg.min_batch = 4;
    if (s->cfg.max_wait_us == 0) s->cfg.max_wait_us = 1;
    if (s->cfg.plain) s->cfg.nstreams = 1;
    dctx_status st = dctx_create(cfg->device, &s->h);
    if (st != DCTX_OK) {
        delete s;
        return st;
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < s->cfg.nstreams && e == hipSuccess; ++i) {
        hipStream_t hs = nullptr;
        e = hipStreamCreateWithFlags(&hs, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(hs);
    }
    const size_t pool = s->cfg.plain ? 0 : s->cfg.hbm_budget;
    if (e == hipSuccess && pool) e = hipMalloc(&s->pool_mem, pool);
    if (e != hipSuccess) {
        server_free(s);
        return e == hipErrorOutOfMemory ? DCTX_ERR_NOMEM : DCTX_ERR_DEVICE;
    }
    s->pool.reset(pool);
    s->t0 = Clock::now();
    try {
        s->th = std::thread(loop, s);
    } catch (...) {
        server_free(s);
        return DCTX_ERR_NOMEM;
    }
    *out = s;
    return DCTX_OK;
}

dctx_status dctx_server_now(dctx_server s, double *t) {
    if (!s || !t) return DCTX_ERR_INVALID;
    *t = s->now();
    return DCTX_OK;
}

dctx_status dctx_server_submit(dctx_server s, const dctx_desc *d, double arrival_s, uint64_t *ticket) {
    if (!s || !d || !ticket) return DCTX_ERR_INVALID;
    const dctx_status st = dctx::rt_check_desc(*d);
    if (st != DCTX_OK) return st;
    Req r;
    r.d = *d;
    r.footprint = dctx::rt_footprint(*d);
    if (!s->cfg.plain && r.footprint > s->pool.capacity()) return DCTX_ERR_NOMEM;   // can never be admitted
    try {
        std::lock_guard<std::mutex> g(s->mu);
        r.arrival = arrival_s >= 0.0 ? arrival_s : s->now();
        *ticket = s->reqs.size();
        s->reqs.push_back(r);
        s->future.emplace_back(r.arrival, *ticket);
        std::push_heap(s->future.begin(), s->future.end(), std::greater<std::pair<double, uint64_t>>());
        s->outstanding++;
    } catch (const std::bad_alloc &) {
        return DCTX_ERR_NOMEM;
    }
    s->cv_work.notify_all();
    return DCTX_OK;
}

dctx_status dctx_server_poll(dctx_server s, uint64_t ticket, dctx_req_stats *out) {
    if (!s) return DCTX_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    if (ticket >= s->reqs.size()) return DCTX_ERR_INVALID;
    const Req &r = s->reqs[ticket];
    if (r.done < 0.0) return DCTX_ERR_BUSY;
    if (out) {
        out->status = r.status;
        out->arrival_s = r.arrival;
        out->launch_s = r.launch;
        out->done_s = r.done;
        out->latency_ms = (r.done - r.arrival) * 1e3;
        out->batch_size = r.batch;
    }
    return DCTX_OK;
}

dctx_status dctx_server_drain(dctx_server s) {
    if (!s) return DCTX_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_work.notify_all();
    while (s->outstanding > 0) s->cv_done.wait_for(lk, std::chrono::milliseconds(10));
    return DCTX_OK;
}

dctx_status dctx_server_summary_get(dctx_server s, uint64_t first_ticket, dctx_server_summary *out) {
    if (!s || !out) return DCTX_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof(*out));
    std::vector<double> lat;
    double t_first = 1e300, t_last = -1e300;
    for (uint64_t i = first_ticket; i < s->reqs.size(); ++i) {
        const Req &r = s->reqs[i];
        if (r.done < 0.0 || r.status != DCTX_OK) continue;
        lat.push_back((r.done - r.arrival) * 1e3);
        t_first = std::min(t_first, r.arrival);
        t_last = std::max(t_last, r.done);
    }
    out->completed = (int64_t)lat.size();
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            const size_t k = (size_t)std::min<double>((double)lat.size() - 1, std::ceil(p * lat.size()) - 1);
            return lat[k];
        };
        double sum = 0.0;
        for (double v : lat) sum += v;
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->mean_ms = sum / lat.size();
        out->max_ms = lat.back();
        out->span_s = t_last - t_first;
        out->req_per_s = out->span_s > 0 ? lat.size() / out->span_s : 0.0;
    }
    out->batches = s->batches;
    out->mean_batch = s->batches ? (double)s->batched_reqs / s->batches : 0.0;
    out->peak_pool_bytes = s->pool.peak();
    return DCTX_OK;
}

dctx_status dctx_server_cancel(dctx_server s, uint64_t ticket) {
    if (!s) return DCTX_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    if (ticket >= s->reqs.size()) return DCTX_ERR_INVALID;
    Req &r = s->reqs[ticket];
    if (r.launch >= 0.0 || r.done >= 0.0) return DCTX_ERR_BUSY;
    bool found = false;
    auto fit = std::find_if(s->future.begin(), s->future.end(),
                            [ticket](const std::pair<double, uint64_t> &e) { return e.second == ticket; });
    if (fit != s->future.end()) {
        s->future.erase(fit);
        std::make_heap(s->future.begin(), s->future.end(), std::greater<std::pair<double, uint64_t>>());
        found = true;
    } else {
        auto rit = std::find(s->ready.begin(), s->ready.end(), ticket);
        if (rit != s->ready.end()) {
            s->ready.erase(rit);
            found = true;
        }
    }
    if (!found) return DCTX_ERR_BUSY;   // taken by a batch being formed
    r.status = DCTX_ERR_CANCELLED;
    r.batch = 0;
    r.done = s->now();
    s->outstanding--;
    s->cv_done.notify_all();
    return DCTX_OK;
}

dctx_status dctx_server_inject_alloc_failures(dctx_server s, int count) {
    if (!s || count < 0) return DCTX_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    s->inject_fail = count;
    return DCTX_OK;
}

dctx_status dctx_server_destroy(dctx_server s) {
    if (!s) return DCTX_ERR_INVALID;
    (void)dctx_server_drain(s);
    server_free(s);
    return DCTX_OK;
}

}  // extern "C"
