// rd_server.hip -- served form: a request loop with continuous batching under an HBM budget.
//
// Requests (a grid and host events) queue up as they are submitted.  Each of `max_inflight` worker
// threads owns a HIP stream; whenever a worker is free it admits every waiting request that fits
// (first come, first served, up to max_batch) into one pass: the requests' events and the pass's
// workspace are carved out of the caller's device arena -- the budget -- and the pass is one
// rd_check_many over workspace-less member traces, reported with one rd_races_many.  Passes of
// different workers overlap on the device; a request that does not fit waits until memory is
// returned.  The arena is the only device memory used, reused from pass to pass.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rd.h"

namespace rd {
int ctx_device(rd_ctx c);
}

namespace {

using clk = std::chrono::steady_clock;

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
  public:
    explicit Arena(uint64_t size) { if (size >= 256) free_[0] = size / 256 * 256; }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
        }
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

struct Request {
    uint64_t ticket;
    rd_grid grid;
    const rd_event *events;
    uint64_t n;
    double t_submit = 0, t_start = 0, t_done = 0;
    bool done = false;
    rd_status status = RD_OK;
    uint64_t bad_index = UINT64_MAX;
    std::vector<rd_pair> pairs;
};

}  // namespace

struct rd_server_s {
    rd_ctx ctx;
    std::vector<rd_ctx> wctx;  // one context per worker: error details stay per thread
    char *arena_base;
    Arena arena;
    uint32_t max_batch, max_inflight;
    clk::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    uint64_t passes = 0, requests_done = 0;
    uint32_t inflight = 0;
    rd_server_s(rd_ctx c, void *base, uint64_t bytes) : ctx(c), arena_base((char *)base), arena(bytes) {}
    double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
};

namespace {

struct Admitted {
    Request *r;
    uint64_t ev_off;
    rd_trace trace;
};

static void answer_now(rd_server s, Request *r, rd_status st) {
    s->pending.pop_front();
    r->status = st;
    r->t_start = r->t_done = s->now();
    r->done = true;
    s->cv_done.notify_all();
}

// Takes waiting requests, in order, while their events and the pass's workspace fit the arena and
// they can share one pass.  Called with s->mu held.
static bool admit(rd_server s, rd_ctx ctx, std::vector<Admitted> &batch, uint64_t *ws_off, uint64_t *ws_bytes) {
    batch.clear();
    std::vector<rd_trace> traces;
    while (!s->pending.empty() && batch.size() < s->max_batch) {
        Request *r = s->pending.front();
        uint64_t off = 0;
        if (r->n && !s->arena.alloc(16 * r->n, &off)) {
            if (batch.empty() && s->inflight == 0) { answer_now(s, r, RD_ENOMEM); continue; }  // never fits
            break;
        }
        rd_trace t = nullptr;
        // bound to where its events will be; the events are copied in by the worker
        if (rd_trace_upload(ctx, &r->grid, r->n ? (const rd_event *)(s->arena_base + off) : nullptr, r->n, 1,
                            nullptr, 0, nullptr, nullptr, &t) != RD_OK) {
            if (r->n) s->arena.release(off, 16 * r->n);
            answer_now(s, r, RD_EINVAL);  // an unusable request (bad grid or size)
            continue;
        }
        traces.push_back(t);
        uint64_t need = 0, woff = 0;
        rd_batch_workspace_bytes(ctx, traces.data(), (uint32_t)traces.size(), nullptr, &need);
        if (!need || !s->arena.alloc(need, &woff)) {  // cannot share the pass, or no room
            traces.pop_back();
            rd_trace_free(ctx, t);
            if (r->n) s->arena.release(off, 16 * r->n);
            if (batch.empty() && s->inflight == 0) { answer_now(s, r, RD_ENOMEM); continue; }  // never fits
            break;
        }
        s->arena.release(woff, need);  // only a probe: the pass's workspace is taken once below
        s->pending.pop_front();
        batch.push_back({r, off, t});
    }
    if (batch.empty()) return false;
    uint64_t need = 0;
    rd_batch_workspace_bytes(ctx, traces.data(), (uint32_t)traces.size(), nullptr, &need);
    if (!s->arena.alloc(need, ws_off)) {  // cannot happen: probed above under the same lock
        for (auto it = batch.rbegin(); it != batch.rend(); ++it) {
            rd_trace_free(ctx, it->trace);
            if (it->r->n) s->arena.release(it->ev_off, 16 * it->r->n);
            s->pending.push_front(it->r);
        }
        batch.clear();
        return false;
    }
    *ws_bytes = need;
    s->inflight++;
    return true;
}

static void worker(rd_server s, uint32_t k, int dev) {
    hipStream_t st = s->streams[k];
    rd_ctx ctx = s->wctx[k];
    (void)hipSetDevice(dev);
    std::vector<Admitted> batch;
    std::vector<rd_trace> traces;
    std::vector<rd_pair> out;
    for (;;) {
        uint64_t ws_off = 0, ws_bytes = 0;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_work.wait(g, [&] { return s->stop || (!s->pending.empty() && admit(s, ctx, batch, &ws_off, &ws_bytes)); });
            if (s->stop && batch.empty()) return;
            const double t = s->now();
            for (auto &a : batch) a.r->t_start = t;
        }
        traces.clear();
        bool ok = true;
        for (auto &a : batch) {
            traces.push_back(a.trace);
            if (a.r->n && hipMemcpyAsync(s->arena_base + a.ev_off, a.r->events, 16 * a.r->n, hipMemcpyHostToDevice,
                                         st) != hipSuccess)
                ok = false;
        }
        rd_status rs = ok ? rd_check_many(ctx, traces.data(), (uint32_t)traces.size(), s->arena_base + ws_off,
                                          ws_bytes, nullptr, st)
                          : RD_EHIP;
        std::vector<uint64_t> counts(batch.size());
        std::vector<rd_status> sts(batch.size(), rs);
        if (rs == RD_OK) {
            rd_races_many(ctx, traces.data(), (uint32_t)traces.size(), nullptr, 0, counts.data(), sts.data());
            uint64_t total = 0;
            for (size_t j = 0; j < batch.size(); j++)
                if (sts[j] == RD_OK || sts[j] == RD_ETRUNC) total += counts[j];
            out.resize(total ? total : 1);
            rd_races_many(ctx, traces.data(), (uint32_t)traces.size(), out.data(), total, counts.data(),
                          sts.data());
        }
        // results; members whose status is an error are asked once more alone for the error details
        uint64_t used = 0;
        std::vector<rd_status> final_st(batch.size());
        std::vector<uint64_t> final_bad(batch.size(), UINT64_MAX);
        std::vector<std::vector<rd_pair>> final_pairs(batch.size());
        for (size_t j = 0; j < batch.size(); j++) {
            if (rs == RD_OK && sts[j] == RD_OK) {
                final_pairs[j].assign(out.begin() + used, out.begin() + used + counts[j]);
                used += counts[j];
                final_st[j] = RD_OK;
            } else if (rs == RD_OK) {
                uint64_t n = 0;
                final_st[j] = rd_races(ctx, traces[j], nullptr, 0, &n);
                if (final_st[j] == RD_ETRACE) rd_last_error(ctx, &final_bad[j], nullptr, 0);
            } else {
                final_st[j] = rs;
            }
        }
        (void)hipStreamSynchronize(st);
        {
            std::lock_guard<std::mutex> g(s->mu);
            const double t = s->now();
            for (size_t j = 0; j < batch.size(); j++) {
                Request *r = batch[j].r;
                r->status = final_st[j];
                r->bad_index = final_bad[j];
                r->pairs.swap(final_pairs[j]);
                r->t_done = t;
                r->done = true;
                rd_trace_free(ctx, batch[j].trace);
                if (r->n) s->arena.release(batch[j].ev_off, 16 * r->n);
            }
            s->arena.release(ws_off, ws_bytes);
            s->inflight--;
            s->passes++;
            s->requests_done += batch.size();
            batch.clear();
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();  // memory came back: another worker may admit now
    }
}

}  // namespace

extern "C" {

rd_status rd_server_open(rd_ctx ctx, void *device_arena, const rd_server_config *cfg, rd_server *out) {
    if (!ctx || !cfg || !out || !device_arena || ((uintptr_t)device_arena & 255) || cfg->device_bytes < 4096)
        return RD_EINVAL;
    *out = nullptr;
    rd_server s = new (std::nothrow) rd_server_s(ctx, device_arena, cfg->device_bytes);
    if (!s) return RD_ENOMEM;
    s->max_batch = cfg->max_batch ? cfg->max_batch : 256;
    s->max_inflight = cfg->max_inflight ? cfg->max_inflight : 2;
    s->t0 = clk::now();
    const int dev = rd::ctx_device(ctx);
    if (hipSetDevice(dev) != hipSuccess) { delete s; return RD_EHIP; }
    for (uint32_t k = 0; k < s->max_inflight; k++) {
        hipStream_t st;
        rd_ctx c = nullptr;
        if (hipStreamCreate(&st) != hipSuccess || rd_init(dev, &c) != RD_OK) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            for (rd_ctx x : s->wctx) rd_shutdown(x);
            delete s;
            return RD_EHIP;
        }
        uint32_t tuning = 0;
        rd_get_tuning(ctx, &tuning);
        rd_set_tuning(c, tuning);  // the workers sort with the caller's chosen variant
        s->streams.push_back(st);
        s->wctx.push_back(c);
    }
    for (uint32_t k = 0; k < s->max_inflight; k++) s->workers.emplace_back(worker, s, k, dev);
    *out = s;
    return RD_OK;
}

rd_status rd_server_submit(rd_server s, const rd_grid *grid, const rd_event *events, uint64_t n_events,
                           uint64_t *ticket) {
    if (!s || !grid || !ticket || (n_events && !events)) return RD_EINVAL;
    Request *r = new (std::nothrow) Request;
    if (!r) return RD_ENOMEM;
    r->grid = *grid;
    r->events = events;
    r->n = n_events;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) { delete r; return RD_ESTATE; }
        r->ticket = s->next_ticket++;
        r->t_submit = s->now();
        s->pending.push_back(r);
        s->all[r->ticket] = r;
    }
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return RD_OK;
}

rd_status rd_server_wait(rd_server s, uint64_t ticket, rd_pair *out, uint64_t capacity, rd_request_info *info) {
    if (!s) return RD_EINVAL;
    Request *r;
    {
        std::unique_lock<std::mutex> g(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return RD_EINVAL;
        r = it->second;
        s->cv_done.wait(g, [&] { return r->done; });
        s->all.erase(it);
    }
    const uint64_t m = r->pairs.size();
    const uint64_t k = out ? (capacity < m ? capacity : m) : 0;
    if (k) memcpy(out, r->pairs.data(), k * sizeof(rd_pair));
    if (info) {
        info->n_races = r->status == RD_OK ? m : 0;
        info->bad_index = r->bad_index;
        info->submit_s = r->t_submit;
        info->start_s = r->t_start;
        info->done_s = r->t_done;
    }
    rd_status st = r->status;
    if (st == RD_OK && capacity < m) st = RD_ETRUNC;
    delete r;
    return st;
}

rd_status rd_server_stats(rd_server s, uint64_t *passes, uint64_t *requests_done) {
    if (!s) return RD_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    if (passes) *passes = s->passes;
    if (requests_done) *requests_done = s->requests_done;
    return RD_OK;
}

rd_status rd_server_close(rd_server s) {
    if (!s) return RD_EINVAL;
    {
        std::unique_lock<std::mutex> g(s->mu);
        s->cv_done.wait(g, [&] {
            for (auto &kv : s->all)
                if (!kv.second->done) return false;
            return true;
        });
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &w : s->workers) w.join();
    for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    for (rd_ctx x : s->wctx) rd_shutdown(x);
    for (auto &kv : s->all) delete kv.second;
    delete s;
    return RD_OK;
}

}  // extern "C"
