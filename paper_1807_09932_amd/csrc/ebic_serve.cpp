// ebic_serve.cpp -- the serving engine: population evaluations submitted by
// many concurrent evolutionary runs, batched continuously onto one GPU.
//
// Each run submits one population per generation (host CSR, host outputs)
// and waits for its counts. The engine owns:
//
//   * a device arena of exactly the HBM budget, carved by a first-fit
//     allocator with coalescing: a batch holds one contiguous region (its
//     requests' CSR inputs, then their outputs) from launch to completion,
//     so the admitted bytes never exceed the budget;
//   * stream slots, each with a pinned host buffer laid out like its device
//     region, an event and a thread of its own;
//   * a scheduler thread. Whenever a slot is idle and requests are waiting,
//     it assigns the slot the longest FIFO prefix (up to max_batch requests,
//     and up to an equal share of the waiting requests per idle slot) whose
//     bytes fit the largest free block, with its region of the arena.
//
// The slot's thread packs the batch's CSR into its pinned buffer and
// enqueues on its stream one host-to-device copy, one ebic_eval_batch (a
// replayed graph; capturing a new one takes milliseconds, which then hold
// up this slot alone), one device-to-host copy of all outputs and an event.
// Batches on different slots overlap on the device. It then waits for the
// event, copies each request's counts (and masks) to the caller's buffers,
// records the latency, frees the region and hands the tags to
// ebic_server_poll.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_internal.h"
#include "ebic_runtime_internal.h"

namespace ebic {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device bytes of one request: its CSR inputs, then its outputs.
struct Sizes {
    size_t in = 0, out = 0;
    size_t total() const { return in + out; }
};

Sizes request_sizes(int64_t rows, int32_t n, int64_t ncols, bool negative, bool mmask, bool nmask)
{
    const int64_t words = (rows + 63) / 64;
    Sizes s;
    s.in = align_up(sizeof(int32_t) * ((size_t)n + 1)) + align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(1, ncols));
    s.out = align_up(sizeof(int32_t) * (size_t)n);
    if (negative) s.out += align_up(sizeof(int32_t) * (size_t)n);
    if (mmask) s.out += align_up(sizeof(uint64_t) * (size_t)n * (size_t)words);
    if (nmask) s.out += align_up(sizeof(uint64_t) * (size_t)n * (size_t)words);
    return s;
}

struct Req {
    // The matrix reference taken at submission (dropped with the request).
    ebic_ctx *held_ctx = nullptr;
    ~Req()
    {
        if (held_ctx) matrix_unref(held_ctx, matrix);
    }
    uint64_t tag = 0;
    int32_t matrix = 0, n = 0;
    uint32_t flags = 0;
    int64_t rows = 0, ncols = 0;
    std::vector<int32_t> offsets, cols;
    int32_t *matched = nullptr, *negative = nullptr;
    uint64_t *mmask = nullptr, *nmask = nullptr;
    Sizes sz;
    double t_submit = 0, t_launched = 0;
    int64_t checks = 0;
    // placement inside the batch region
    size_t in_off = 0, out_off = 0;
};

// First-fit allocator over [0, cap) in kAlign units, with coalescing.
class FreeList {
  public:
    explicit FreeList(size_t cap) { blocks_[0] = cap; }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = blocks_.begin(); it != blocks_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                blocks_.erase(it);
                if (rest) blocks_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = blocks_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != blocks_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            blocks_.erase(next);
        }
        if (it != blocks_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                blocks_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &b : blocks_) m = std::max(m, b.second);
        return m;
    }

  private:
    std::map<size_t, size_t> blocks_;  // offset -> size
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char *h_buf = nullptr;
    size_t h_cap = 0;
    std::vector<std::unique_ptr<Req>> batch;
    size_t dev_off = 0, dev_bytes = 0, in_bytes = 0;
    bool busy = false;      // owns a batch (from assignment to completion)
    bool assigned = false;  // a batch waits for this slot's thread to launch it
    std::thread completer;  // launches the slot's batches and completes them
};

}  // namespace
}  // namespace ebic

using namespace ebic;

struct ebic_server {
    ebic_ctx *ctx = nullptr;
    int64_t budget = 0;
    int32_t max_batch = 256;
    char *d_arena = nullptr;
    std::unique_ptr<FreeList> free_list;
    std::vector<std::unique_ptr<Slot>> slots;
    std::mutex mu;
    std::condition_variable cv_sched;  // scheduler: new requests, an idle slot, freed memory
    std::condition_variable cv_slot;   // slot threads: a batch was assigned
    std::condition_variable cv_done;   // pollers: tags completed
    std::deque<std::unique_ptr<Req>> pending;
    std::deque<std::pair<uint64_t, ebic_status>> done;
    bool stop = false;
    bool paused = false;      // launch no new batch
    bool sched_done = false;  // the scheduler has drained every request and exited
    std::thread scheduler;
    // statistics
    int64_t submitted = 0, completed = 0, cancelled = 0, batches = 0, batched_requests = 0;
    int64_t reserved = 0, high_water = 0, checks = 0, staging_grows = 0;
    std::vector<double> latencies_ms;
    std::vector<double> queue_ms;  // submission to the batch's enqueue on its slot
};

namespace ebic {
namespace {

void complete_locked(ebic_server *srv, std::unique_ptr<Req> r, ebic_status st, double t_done)
{
    if (st == EBIC_ECANCELED) {
        ++srv->cancelled;
    } else {
        srv->latencies_ms.push_back((t_done - r->t_submit) * 1e3);
        srv->queue_ms.push_back(((r->t_launched > 0 ? r->t_launched : t_done) - r->t_submit) * 1e3);
        ++srv->completed;
        srv->checks += r->checks;
    }
    srv->done.emplace_back(r->tag, st);
}

// Pack the slot's batch into its pinned buffer and enqueue the copies and
// the evaluation. Called without the server lock.
ebic_status launch_batch_on(ebic_server *srv, Slot &sl)
{
    return guarded([&] {
        DeviceGuard dg(srv->ctx->device);
        size_t in_total = 0, out_total = 0;
        for (auto &r : sl.batch) {
            r->in_off = in_total;
            in_total += r->sz.in;
        }
        for (auto &r : sl.batch) {
            r->out_off = in_total + out_total;
            out_total += r->sz.out;
        }
        const size_t total = in_total + out_total;
        if (sl.h_cap < total) {
            const size_t cap = std::max<size_t>(total, 2 * sl.h_cap);
            if (sl.h_buf) hip_check(hipHostFree(sl.h_buf), "hipHostFree");
            sl.h_buf = nullptr;
            sl.h_cap = 0;
            {
                std::lock_guard<std::mutex> lk(srv->mu);
                ++srv->staging_grows;
            }
            hip_check(hipHostMalloc(reinterpret_cast<void **>(&sl.h_buf), cap, hipHostMallocDefault),
                      "hipHostMalloc");
            sl.h_cap = cap;
        }
        char *h = sl.h_buf;
        char *d = srv->d_arena + sl.dev_off;
        std::vector<ebic_request> reqs;
        reqs.reserve(sl.batch.size());
        for (auto &r : sl.batch) {
            char *hi = h + r->in_off;
            std::memcpy(hi, r->offsets.data(), sizeof(int32_t) * r->offsets.size());
            const size_t cols_at = align_up(sizeof(int32_t) * r->offsets.size());
            if (!r->cols.empty()) std::memcpy(hi + cols_at, r->cols.data(), sizeof(int32_t) * r->cols.size());
            else std::memset(hi + cols_at, 0, sizeof(int32_t));
            char *dout = d + r->out_off;
            const int64_t words = (r->rows + 63) / 64;
            ebic_request q{};
            q.matrix = r->matrix;
            q.n_ind = r->n;
            q.d_offsets = reinterpret_cast<const int32_t *>(d + r->in_off);
            q.d_cols = reinterpret_cast<const int32_t *>(d + r->in_off + cols_at);
            q.flags = r->flags;
            size_t o = 0;
            q.d_matched = reinterpret_cast<int32_t *>(dout + o);
            o += align_up(sizeof(int32_t) * (size_t)r->n);
            if (r->negative) {
                q.d_negative = reinterpret_cast<int32_t *>(dout + o);
                o += align_up(sizeof(int32_t) * (size_t)r->n);
            }
            if (r->mmask) {
                q.d_matched_mask = reinterpret_cast<uint64_t *>(dout + o);
                o += align_up(sizeof(uint64_t) * (size_t)r->n * (size_t)words);
            }
            if (r->nmask) q.d_negative_mask = reinterpret_cast<uint64_t *>(dout + o);
            reqs.push_back(q);
        }
        hip_check(hipMemcpyAsync(d, h, in_total, hipMemcpyHostToDevice, sl.stream), "hipMemcpyAsync");
        const ebic_status st = ebic_eval_batch(srv->ctx, reqs.data(), (int32_t)reqs.size(), sl.stream);
        if (st != EBIC_OK) fail(st, ebic_last_error());
        hip_check(hipMemcpyAsync(h + in_total, d + in_total, out_total, hipMemcpyDeviceToHost, sl.stream),
                  "hipMemcpyAsync");
        hip_check(hipEventRecord(sl.done, sl.stream), "hipEventRecord");
    });
}

void scheduler_main(ebic_server *srv)
{
    (void)hipSetDevice(srv->ctx->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    while (true) {
        Slot *idle = nullptr;
        for (auto &s : srv->slots)
            if (!s->busy) {
                idle = s.get();
                break;
            }
        bool all_idle = true;
        for (auto &s : srv->slots) all_idle = all_idle && !s->busy;
        if (srv->stop && srv->pending.empty() && all_idle) {
            srv->sched_done = true;
            srv->cv_slot.notify_all();
            break;
        }
        if (!idle || srv->pending.empty() || (srv->paused && !srv->stop)) {
            srv->cv_sched.wait(lk);
            continue;
        }
        // The longest FIFO prefix that fits the largest free block, and at
        // most an equal share (rounded up) of the waiting requests for each
        // idle slot: when several slots are idle, a backlog is spread over
        // them, whose batches run side by side, instead of going whole to
        // the first one as one long batch that every request in it waits
        // for.
        const size_t room = srv->free_list->largest();
        size_t n_idle = 0;
        for (auto &sl : srv->slots) n_idle += sl->busy ? 0 : 1;
        const size_t share = (srv->pending.size() + n_idle - 1) / std::max<size_t>(1, n_idle);
        size_t bytes = 0;
        size_t take = 0;
        while (take < srv->pending.size() && (int32_t)take < srv->max_batch && take < share &&
               bytes + srv->pending[take]->sz.total() <= room) {
            bytes += srv->pending[take]->sz.total();
            ++take;
        }
        if (take == 0) {  // wait for a batch to free memory
            srv->cv_sched.wait(lk);
            continue;
        }
        size_t off = 0;
        if (!srv->free_list->alloc(bytes, &off)) {  // cannot happen: bytes <= largest block
            srv->cv_sched.wait(lk);
            continue;
        }
        srv->reserved += (int64_t)bytes;
        srv->high_water = std::max(srv->high_water, srv->reserved);
        Slot &sl = *idle;
        sl.busy = true;
        sl.dev_off = off;
        sl.dev_bytes = bytes;
        sl.batch.clear();
        for (size_t i = 0; i < take; ++i) {
            sl.batch.push_back(std::move(srv->pending.front()));
            srv->pending.pop_front();
        }
        ++srv->batches;
        srv->batched_requests += (int64_t)take;
        // The slot's own thread packs and launches the batch: a launch that
        // captures a new graph (milliseconds) then holds up that slot alone,
        // not the scheduler and every other slot.
        sl.assigned = true;
        srv->cv_slot.notify_all();
    }
}

void completer_main(ebic_server *srv, Slot *sl)
{
    (void)hipSetDevice(srv->ctx->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    while (true) {
        srv->cv_slot.wait(lk, [&] { return sl->assigned || srv->sched_done; });
        if (!sl->assigned) break;  // every request has completed
        sl->assigned = false;
        lk.unlock();
        ebic_status st = launch_batch_on(srv, *sl);
        const double t_l = now_s();
        for (auto &r : sl->batch) r->t_launched = t_l;
        if (st == EBIC_OK && hipEventSynchronize(sl->done) != hipSuccess) st = EBIC_EHIP;
        // After a failed launch, let whatever was enqueued drain before the
        // pinned buffer is reused.
        if (st != EBIC_OK) (void)hipStreamSynchronize(sl->stream);
        if (st == EBIC_OK) {
            // Scatter the outputs to the callers' buffers.
            for (auto &r : sl->batch) {
                const char *src = sl->h_buf + r->out_off;
                const int64_t words = (r->rows + 63) / 64;
                size_t o = 0;
                std::memcpy(r->matched, src + o, sizeof(int32_t) * (size_t)r->n);
                o += align_up(sizeof(int32_t) * (size_t)r->n);
                if (r->negative) {
                    std::memcpy(r->negative, src + o, sizeof(int32_t) * (size_t)r->n);
                    o += align_up(sizeof(int32_t) * (size_t)r->n);
                }
                if (r->mmask) {
                    std::memcpy(r->mmask, src + o, sizeof(uint64_t) * (size_t)r->n * (size_t)words);
                    o += align_up(sizeof(uint64_t) * (size_t)r->n * (size_t)words);
                }
                if (r->nmask) std::memcpy(r->nmask, src + o, sizeof(uint64_t) * (size_t)r->n * (size_t)words);
            }
        }
        const double t = now_s();
        lk.lock();
        for (auto &r : sl->batch) complete_locked(srv, std::move(r), st, t);
        sl->batch.clear();
        srv->free_list->release(sl->dev_off, sl->dev_bytes);
        srv->reserved -= (int64_t)sl->dev_bytes;
        sl->busy = false;
        srv->cv_sched.notify_all();
        srv->cv_done.notify_all();
    }
}

void shutdown(ebic_server *srv)
{
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_sched.notify_all();
    if (srv->scheduler.joinable()) srv->scheduler.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->sched_done = true;  // also when the scheduler never started
    }
    srv->cv_slot.notify_all();
    for (auto &s : srv->slots)
        if (s->completer.joinable()) s->completer.join();
    (void)hipSetDevice(srv->ctx->device);
    for (auto &s : srv->slots) {
        if (s->stream) (void)hipStreamSynchronize(s->stream);
        if (s->done) (void)hipEventDestroy(s->done);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->h_buf) (void)hipHostFree(s->h_buf);
    }
    srv->slots.clear();
    if (srv->d_arena) ctx_free(srv->ctx, srv->d_arena);
    srv->d_arena = nullptr;
}

}  // namespace
}  // namespace ebic

extern "C" {

ebic_status ebic_server_request_bytes(ebic_ctx *ctx, int32_t matrix, int32_t n_ind, int64_t nnz,
                                      uint32_t flags, int32_t masks, int64_t *out_bytes)
{
    return guarded([&] {
        if (!ctx || !out_bytes) fail(EBIC_EINVAL, "ctx and out_bytes are required");
        if (n_ind < 0 || nnz < 0) fail(EBIC_EINVAL, "n_ind and nnz must be >= 0");
        int64_t rows;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            rows = ctx_matrix(ctx, matrix).dev.rows;
        }
        const bool neg = (flags & EBIC_NEG_TRENDS) != 0;
        *out_bytes = (int64_t)request_sizes(rows, n_ind, nnz, neg, masks != 0, masks != 0 && neg).total();
    });
}

ebic_status ebic_server_create(ebic_ctx *ctx, int64_t hbm_budget_bytes, int32_t slots, int32_t max_batch,
                               ebic_server **out)
{
    return guarded([&] {
        if (!ctx || !out) fail(EBIC_EINVAL, "ctx and out are required");
        *out = nullptr;
        if (hbm_budget_bytes < (int64_t)kAlign) fail(EBIC_EINVAL, "HBM budget below 256 bytes");
        if (slots < 1 || slots > 16) fail(EBIC_EINVAL, "slots must be in 1..16");
        if (max_batch < 1) fail(EBIC_EINVAL, "max_batch must be >= 1");
        DeviceGuard dg(ctx->device);
        auto srv = std::make_unique<ebic_server>();
        srv->ctx = ctx;
        srv->budget = (int64_t)(hbm_budget_bytes & ~(int64_t)(kAlign - 1));
        srv->max_batch = max_batch;
        srv->d_arena = static_cast<char *>(ctx_alloc(ctx, (size_t)srv->budget));
        srv->free_list = std::make_unique<FreeList>((size_t)srv->budget);
        try {
            // Pinned staging per slot, sized for a full batch of typical
            // requests up front (grown by doubling if a batch needs more).
            const size_t stage0 = (size_t)std::min<int64_t>(srv->budget, (int64_t)16 << 20);
            for (int32_t i = 0; i < slots; ++i) {
                auto s = std::make_unique<Slot>();
                hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
                hip_check(hipEventCreateWithFlags(&s->done, hipEventDisableTiming), "hipEventCreate");
                hip_check(hipHostMalloc(reinterpret_cast<void **>(&s->h_buf), stage0, hipHostMallocDefault),
                          "hipHostMalloc");
                s->h_cap = stage0;
                srv->slots.push_back(std::move(s));
            }
            srv->scheduler = std::thread(scheduler_main, srv.get());
            for (auto &s : srv->slots) s->completer = std::thread(completer_main, srv.get(), s.get());
        } catch (...) {
            shutdown(srv.get());
            throw;
        }
        *out = srv.release();
    });
}

ebic_status ebic_server_destroy(ebic_server *srv)
{
    return guarded([&] {
        if (!srv) return;
        shutdown(srv);
        delete srv;
    });
}

ebic_status ebic_server_submit(ebic_server *srv, int32_t matrix, int32_t n_ind, const int32_t *offsets,
                               const int32_t *cols, uint32_t flags, int32_t *matched, int32_t *negative,
                               uint64_t *matched_mask, uint64_t *negative_mask, uint64_t tag)
{
    return guarded([&] {
        if (!srv) fail(EBIC_EINVAL, "server is NULL");
        if (n_ind < 0) fail(EBIC_EINVAL, "n_ind < 0");
        if (flags & ~(EBIC_NAN_INCLUDE | EBIC_NEG_TRENDS)) fail(EBIC_EINVAL, "unknown flags");
        if (n_ind > 0 && (!offsets || !matched)) fail(EBIC_EINVAL, "offsets and matched are required");
        if (negative_mask && !negative) fail(EBIC_EINVAL, "negative_mask needs negative");
        auto r = std::make_unique<Req>();
        r->tag = tag;
        r->matrix = matrix;
        r->n = n_ind;
        r->flags = flags;
        {
            std::lock_guard<std::mutex> lk(srv->ctx->mu);
            r->rows = ctx_matrix(srv->ctx, matrix).dev.rows;
            matrix_ref_locked(srv->ctx, matrix);
            r->held_ctx = srv->ctx;
        }
        // The column array's length: the largest offset (decreasing offsets
        // mark invalid individuals, which the kernels report as -1).
        int64_t ncols = 0;
        for (int32_t i = 0; i <= n_ind && n_ind > 0; ++i) {
            if (offsets[i] < 0) fail(EBIC_EINVAL, "negative offset");
            ncols = std::max<int64_t>(ncols, offsets[i]);
        }
        if (ncols > 0 && !cols) fail(EBIC_EINVAL, "cols is required");
        r->ncols = ncols;
        r->matched = matched;
        r->negative = negative;
        r->mmask = matched_mask;
        r->nmask = negative_mask;
        r->sz = request_sizes(r->rows, n_ind, ncols, negative != nullptr, matched_mask != nullptr,
                              negative_mask != nullptr);
        if ((int64_t)r->sz.total() > srv->budget)
            fail(EBIC_EBUDGET, "request needs " + std::to_string(r->sz.total()) + " device bytes, budget is " +
                                   std::to_string(srv->budget));
        if (n_ind > 0) {
            r->offsets.assign(offsets, offsets + n_ind + 1);
            r->cols.assign(cols ? cols : offsets, cols ? cols + ncols : offsets);
            r->checks = r->rows * (int64_t)std::max(0, offsets[n_ind] - offsets[0]);
        }
        r->t_submit = now_s();
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) fail(EBIC_EBUSY, "server is shutting down");
        ++srv->submitted;
        if (n_ind == 0) {
            complete_locked(srv, std::move(r), EBIC_OK, now_s());
            srv->cv_done.notify_all();
            return;
        }
        srv->pending.push_back(std::move(r));
        srv->cv_sched.notify_one();
    });
}

ebic_status ebic_server_poll(ebic_server *srv, uint64_t *tags, ebic_status *statuses, int32_t max_tags,
                             int32_t timeout_us, int32_t *n_done)
{
    return guarded([&] {
        if (!srv || !tags || !n_done || max_tags < 1) fail(EBIC_EINVAL, "bad poll arguments");
        *n_done = 0;
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->done.empty() && timeout_us > 0)
            srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !srv->done.empty(); });
        int32_t k = 0;
        while (k < max_tags && !srv->done.empty()) {
            tags[k] = srv->done.front().first;
            if (statuses) statuses[k] = srv->done.front().second;
            srv->done.pop_front();
            ++k;
        }
        *n_done = k;
    });
}

ebic_status ebic_server_cancel(ebic_server *srv, uint64_t tag)
{
    return guarded([&] {
        if (!srv) fail(EBIC_EINVAL, "server is NULL");
        std::unique_ptr<Req> r;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            for (auto it = srv->pending.begin(); it != srv->pending.end(); ++it) {
                if ((*it)->tag == tag) {
                    r = std::move(*it);
                    srv->pending.erase(it);
                    break;
                }
            }
            if (!r) {
                for (auto &sl : srv->slots)
                    for (auto &q : sl->batch)
                        if (q && q->tag == tag) fail(EBIC_EBUSY, "request is already on the device");
                fail(EBIC_ENOENT, "no queued request has tag " + std::to_string(tag));
            }
            // (the matrix reference is dropped after the server lock, with r)
            const uint64_t t = r->tag;
            const double t_submit = r->t_submit;
            auto stub = std::make_unique<Req>();
            stub->tag = t;
            stub->t_submit = t_submit;
            complete_locked(srv, std::move(stub), EBIC_ECANCELED, now_s());
            srv->cv_done.notify_all();
            srv->cv_sched.notify_all();
        }
        log_msg(2, "cancelled serving request " + std::to_string(tag));
    });
}

ebic_status ebic_server_set_paused(ebic_server *srv, int32_t paused)
{
    return guarded([&] {
        if (!srv) fail(EBIC_EINVAL, "server is NULL");
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->paused = paused != 0;
        srv->cv_sched.notify_all();
    });
}

ebic_status ebic_server_get_stats(ebic_server *srv, ebic_server_stats *out, int32_t reset)
{
    return guarded([&] {
        if (!srv || !out) fail(EBIC_EINVAL, "server and out are required");
        std::lock_guard<std::mutex> lk(srv->mu);
        ebic_server_stats s{};
        s.submitted = srv->submitted;
        s.completed = srv->completed;
        s.batches = srv->batches;
        s.pending = (int64_t)srv->pending.size();
        s.reserved_bytes = srv->reserved;
        s.high_water_bytes = srv->high_water;
        s.budget_bytes = srv->budget;
        s.nominal_checks = srv->checks;
        s.mean_batch = srv->batches ? (double)srv->batched_requests / (double)srv->batches : 0.0;
        s.staging_grows = srv->staging_grows;
        s.cancelled = srv->cancelled;
        {
            std::lock_guard<std::mutex> lk2(srv->ctx->mu);
            s.graph_captures = srv->ctx->graph_captures;
        }
        std::vector<double> v = srv->latencies_ms;
        if (!v.empty()) s.latency_max_ms = *std::max_element(v.begin(), v.end());
        {
            std::vector<double> q = srv->queue_ms;
            if (!q.empty()) {
                const size_t i = std::min(q.size() - 1, (size_t)(0.99 * (double)(q.size() - 1) + 0.5));
                std::nth_element(q.begin(), q.begin() + (ptrdiff_t)i, q.end());
                s.queue_p99_ms = q[i];
            }
        }
        if (!v.empty()) {
            auto pct = [&](double q) {
                const size_t i = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
                std::nth_element(v.begin(), v.begin() + (ptrdiff_t)i, v.end());
                return v[i];
            };
            s.latency_p50_ms = pct(0.50);
            s.latency_p99_ms = pct(0.99);
        }
        *out = s;
        if (reset) {
            srv->submitted -= srv->completed;
            srv->submitted -= srv->cancelled;
            srv->completed = 0;
            srv->cancelled = 0;
            srv->batches = 0;
            srv->batched_requests = 0;
            srv->checks = 0;
            srv->high_water = srv->reserved;
            srv->latencies_ms.clear();
            srv->queue_ms.clear();
        }
    });
}

}  // extern "C"
