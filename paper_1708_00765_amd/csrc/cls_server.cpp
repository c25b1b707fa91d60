// Continuous-batching CLS server.
//
// Requests (a problem, a history count and a seed) are admitted in arrival
// order while the summed device footprint of admitted requests stays within
// the HBM budget; an admitted request's tallies stay resident until it
// completes. A worker thread issues "rounds": one batched persistent launch of
// the tracking kernel over the next chunks of every admitted request of one
// kernel variant (round-robin over variants), of at least round_histories and
// at least kRoundChunksPerWave of the largest chunks per wave, shared equally
// between the requests, largest chunks first in the work queue.
// Requests admitted while others are on the GPU join the next round, so their
// work overlaps on the device; up to max_inflight_rounds launches are queued
// at once on two streams. A request whose last chunk has completed gets its
// finalize kernel and result copy; it is done when that copy has landed.
//
// Every history keeps the stream keyed by (seed, history index), and chunks
// are fixed by the request's history count, so a request's results do not
// depend on what it was batched with (integer tallies bitwise, FP64 sums up to
// the order of atomic additions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "cls_runtime.hpp"

using namespace cls;
using namespace cls::rt;

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { RQ_PENDING, RQ_ACTIVE, RQ_FINALIZING, RQ_DONE, RQ_FAILED };

struct Request {
    uint64_t ticket = 0;
    cls_problem *p = nullptr;
    uint64_t histories = 0, seed = 0;
    uint64_t chunk = 0, n_chunks = 0, next_chunk = 0, done_chunks = 0;
    size_t footprint = 0;
    ReqState state = RQ_PENDING;
    cls_status error = CLS_OK;
    Clock::time_point t_submit, t_admit, t_done;
    uint32_t rounds = 0;
    int stream = 0;
    bool prepared = false;   // device side done (prepare)
    uint64_t *host_record = nullptr;   // device address of the problem's pinned record (0: finalize kernel)
};

struct RoundPart {
    Request *r;
    uint64_t chunks;
};

struct RoundSlot {
    char *dev = nullptr, *host = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool busy = false;
    int stream = 0;
    std::vector<RoundPart> parts;
};

}  // namespace

struct cls_server {
    cls_server_config cfg{};
    int device = -1;
    DeviceInfo di;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::deque<Request *> pending;
    std::vector<Request *> active;       // admitted, not yet done
    std::set<const cls_problem *> in_flight;   // problems with a request being submitted, pending or active
    std::map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    uint32_t next_stream = 0;
    size_t in_use = 0, peak = 0;
    hipStream_t streams[2] = {nullptr, nullptr};
    std::vector<RoundSlot> slots;
    int next_variant = 0;
    uint64_t rounds = 0, completed = 0, failed = 0, hist_done = 0;
    Clock::time_point t0;
    cls_status worker_error = CLS_OK;
};

namespace {

double seconds_since(const cls_server *s, Clock::time_point t)
{
    return std::chrono::duration<double>(t - s->t0).count();
}

// A request reaches its final state (under the lock); waiters are woken on
// every path, failures included.
void finish(cls_server *s, Request *r, cls_status err)
{
    r->state = err == CLS_OK ? RQ_DONE : RQ_FAILED;
    r->error = err;
    r->t_done = Clock::now();
    s->in_use -= r->footprint;
    if (err == CLS_OK) {
        ++s->completed;
        s->hist_done += r->histories;
    } else {
        ++s->failed;
    }
    s->active.erase(std::find(s->active.begin(), s->active.end(), r));
    s->in_flight.erase(r->p);
    s->cv_done.notify_all();
}

// Device side of a request, done once before it is admitted: the problem's
// workspace, its chunking, its record and the reset of its tallies on the
// request's stream (which the other stream waits for). Called from the
// submitting thread when it runs on the server's device, else by the worker
// at admission; the request is not yet visible to any round.
cls_status prepare(cls_server *s, Request *r)
{
    cls_problem *p = r->p;
    cls_status st = ensure_device(p, 0);
    if (st != CLS_OK) return st;
    // chunks fixed by the request alone (never by the mix it meets): rounds
    // are shared, so a small request need not be cut into a chunk per wave;
    // a chunk stays within a round's share of one wave
    int grid, block, stride;
    size_t lds;
    LaunchShape sh;
    st = shape_for(variant_of(p), p->nbins, s->di, &grid, &block, &lds, &stride, &sh);
    if (st != CLS_OK) return st;
    const uint64_t waves_total = (uint64_t)grid * (uint64_t)(block / 64);
    const uint64_t round_share = std::max<uint64_t>(1, s->cfg.round_histories / waves_total);
    r->chunk = grouped_chunk_size(r->histories, waves_total, (uint64_t)sh.max_chunk, round_share);
    r->n_chunks = (r->histories + r->chunk - 1) / r->chunk;
    if (p->has_run && !p->done_synced) HIP_TRY(hipEventSynchronize(p->ev_done));
    fill_dev_problem(p, r->histories, r->seed, r->chunk, 0, p->h_prob);
    hipStream_t st_ = s->streams[r->stream];
    HIP_TRY(hipMemcpyAsync(p->d_prob, p->h_prob, sizeof(DevProblem), hipMemcpyHostToDevice, st_));
    HIP_TRY(launch_reset(p->d_prob, 1, p->d_items + 2, st_));
    // both streams must see the reset before any round touches the tallies
    HIP_TRY(hipEventRecord(p->ev_k0, st_));
    HIP_TRY(hipStreamWaitEvent(s->streams[r->stream ^ 1], p->ev_k0, 0));
    // the round that completes the request writes its record straight into the
    // pinned host record when the device can address it; else a finalize
    // kernel and a copy follow the request's last round
    void *dptr = nullptr;
    r->host_record = s->cfg.record_path == 0 && hipHostGetDevicePointer(&dptr, p->h_record, 0) == hipSuccess
                          ? (uint64_t *)dptr
                          : nullptr;
    r->prepared = true;
    return CLS_OK;
}

// Admission (under the lock).
cls_status admit(cls_server *s, Request *r)
{
    if (!r->prepared) {
        const cls_status st = prepare(s, r);
        if (st != CLS_OK) return st;
    }
    r->t_admit = Clock::now();
    r->state = RQ_ACTIVE;
    return CLS_OK;
}

cls_status ensure_slot(cls_server *s, RoundSlot &sl, size_t bytes)
{
    if (sl.bytes >= bytes) return CLS_OK;
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.host) (void)hipHostFree(sl.host);
    sl.dev = sl.host = nullptr;
    sl.bytes = 0;
    const size_t want = std::max<size_t>(bytes * 2, 1 << 16);
    hipError_t e = hipMalloc((void **)&sl.dev, want);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sl.host, want, hipHostMallocDefault);
    if (e != hipSuccess) return fail(CLS_ERR_OUT_OF_MEMORY, std::string("round buffers: ") + hipGetErrorString(e));
    sl.bytes = want;
    (void)s;
    return CLS_OK;
}

// Build and launch one round into a free slot. Returns true if launched.
bool launch_round(cls_server *s, RoundSlot &sl, cls_status *err)
{
    // variants with chunks left, in a fixed order
    std::vector<Variant> vars;
    for (Request *r : s->active)
        if (r->state == RQ_ACTIVE && r->next_chunk < r->n_chunks) {
            const Variant v = variant_of(r->p);
            bool seen = false;
            for (const Variant &w : vars) seen = seen || same_variant(v, w);
            if (!seen) vars.push_back(v);
        }
    if (vars.empty()) return false;
    const Variant v = vars[(size_t)s->next_variant % vars.size()];
    ++s->next_variant;
    std::vector<Request *> reqs;
    for (Request *r : s->active)
        if (r->state == RQ_ACTIVE && r->next_chunk < r->n_chunks && same_variant(variant_of(r->p), v))
            reqs.push_back(r);
    // Launch shape first: its wave count sizes the round. Chunks were fixed at
    // admission, so the share of histories in small chunks does not depend on
    // the grid.
    auto small_share_of = [](const std::vector<RoundPart> &parts) {
        double small = 0.0, all = 0.0;
        for (const RoundPart &part : parts) {
            const double h = (double)part.chunks * (double)part.r->chunk;
            all += h;
            if (part.r->chunk < kSingleSlotMinChunk) small += h;
        }
        return all > 0.0 ? small / all : 1.0;
    };
    int max_bins = 1;
    uint64_t max_chunk = 1;
    sl.parts.clear();
    for (Request *r : reqs) {
        sl.parts.push_back({r, r->n_chunks - r->next_chunk});
        max_bins = std::max(max_bins, r->p->nbins);
        max_chunk = std::max(max_chunk, r->chunk);
    }
    int grid = 0, block = 0, stride = 0;
    size_t lds = 0;
    LaunchShape used;
    const double backlog_share = small_share_of(sl.parts);
    *err = shape_for(v, max_bins, s->di, &grid, &block, &lds, &stride, &used,
                     [backlog_share](uint64_t, uint64_t) { return backlog_share; });
    // Round size (sched::round_budget), shared by water-filling: requests with
    // less left than an equal share finish in this round, the others get the
    // equal share of what remains (at least one chunk each).
    const uint64_t waves = *err == CLS_OK ? (uint64_t)grid * (uint64_t)(block / 64) : 1;
    const double budget = sched::round_budget((double)s->cfg.round_histories, waves, max_chunk);
    std::vector<sched::RoundClaim> claims;
    for (Request *r : reqs) claims.push_back({r->chunk, r->n_chunks - r->next_chunk});
    const std::vector<uint64_t> take = sched::water_fill(claims, budget);
    sl.parts.clear();
    for (size_t i = 0; i < reqs.size(); ++i) sl.parts.push_back({reqs[i], take[i]});
    // largest chunks first: the work queue hands items out in order, so the
    // small chunks fill the waves that finish early
    std::stable_sort(sl.parts.begin(), sl.parts.end(),
                     [](const RoundPart &a, const RoundPart &b) { return a.r->chunk > b.r->chunk; });
    const int n = (int)sl.parts.size();
    const size_t probs_bytes = align256((size_t)n * sizeof(DevProblem));
    // item prefix sums, the queue head and the count of waves that have left
    const size_t items_bytes = align256(((size_t)n + 3) * sizeof(uint64_t));
    if (*err == CLS_OK) {
        const double share = small_share_of(sl.parts);
        *err = shape_for(v, max_bins, s->di, &grid, &block, &lds, &stride, &used,
                         [share](uint64_t, uint64_t) { return share; });
    }
    if (*err == CLS_OK) *err = ensure_slot(s, sl, probs_bytes + items_bytes);
    if (*err != CLS_OK) {
        // these requests cannot be launched: fail them rather than retry forever
        for (RoundPart &part : sl.parts) finish(s, part.r, *err);
        sl.parts.clear();
        return false;
    }
    DevProblem *h_probs = (DevProblem *)sl.host;
    uint64_t *h_items = (uint64_t *)(sl.host + probs_bytes);
    h_items[0] = 0;
    for (int i = 0; i < n; ++i) {
        Request *r = sl.parts[i].r;
        fill_dev_problem(r->p, r->histories, r->seed, r->chunk, 0, &h_probs[i]);
        h_probs[i].chunk_base = r->next_chunk;
        if (r->host_record) {
            h_probs[i].final_chunks = r->n_chunks;
            h_probs[i].host_record = r->host_record;
        }
        h_items[i + 1] = h_items[i] + sl.parts[i].chunks;
    }
    h_items[n + 1] = 0;
    h_items[n + 2] = 0;
    hipStream_t st = s->streams[sl.stream];
    TrackArgs a;
    a.probs = (const DevProblem *)sl.dev;
    a.item_start = (const uint64_t *)(sl.dev + probs_bytes);
    a.queue_head = (uint64_t *)(sl.dev + probs_bytes) + n + 1;
    a.nprobs = n;
    a.lds_stride = stride;
    a.refill_min = used.refill_min;
    a.slots = used.slots;
    a.exit_count = (unsigned long long *)(sl.dev + probs_bytes) + n + 2;
    hipError_t e = hipMemcpyAsync(sl.dev, sl.host, probs_bytes + items_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_track(v, a, grid, block, lds, st);
    if (e == hipSuccess) e = hipEventRecord(sl.ev, st);
    if (e != hipSuccess) {
        *err = hip_fail(e, "round launch");
        for (RoundPart &part : sl.parts) finish(s, part.r, *err);
        sl.parts.clear();
        return false;
    }
    for (RoundPart &part : sl.parts) {
        part.r->next_chunk += part.chunks;
        ++part.r->rounds;
    }
    sl.busy = true;
    ++s->rounds;
    return true;
}

// A request whose results are in its problem's host record.
void complete(cls_server *s, Request *r)
{
    cls_problem *p = r->p;
    p->has_run = true;
    p->done_synced = true;
    p->timed_by_events = false;
    p->track_ms = 0.0f;
    p->histories = r->histories;
    p->seed = r->seed;
    p->trace_n = 0;
    finish(s, r, p->h_record[C_CAPPED] ? CLS_ERR_EVENT_CAP : CLS_OK);
}

// A request whose chunks all completed (no device-addressable host record):
// finalize and copy its results back.
cls_status start_finalize(cls_server *s, Request *r)
{
    cls_problem *p = r->p;
    hipStream_t st = s->streams[r->stream];
    HIP_TRY(launch_finalize(p->d_prob, 1, st));
    HIP_TRY(hipMemcpyAsync(p->h_record, p->d_record, record_words(p->nbins) * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(p->ev_done, st));
    p->done_synced = false;
    r->state = RQ_FINALIZING;
    return CLS_OK;
}

void worker_main(cls_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // admit in arrival order while the footprint fits
        while (!s->pending.empty()) {
            Request *r = s->pending.front();
            if (s->in_use + r->footprint > s->cfg.hbm_budget_bytes && !s->active.empty()) break;
            s->pending.pop_front();
            s->active.push_back(r);
            s->in_use += r->footprint;
            s->peak = std::max(s->peak, s->in_use);
            const cls_status st = admit(s, r);
            if (st != CLS_OK) finish(s, r, st);
        }
        // retire completed rounds
        for (RoundSlot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            sl.busy = false;
            for (RoundPart &part : sl.parts) {
                Request *r = part.r;
                if (q != hipSuccess) {
                    if (r->state == RQ_ACTIVE) finish(s, r, hip_fail(q, "round"));
                    continue;
                }
                r->done_chunks += part.chunks;
                if (r->state == RQ_ACTIVE && r->done_chunks == r->n_chunks) {
                    if (r->host_record) {
                        // every round with its chunks has completed, and the last
                        // of them wrote the record into the pinned host record
                        complete(s, r);
                    } else {
                        const cls_status st = start_finalize(s, r);
                        if (st != CLS_OK) finish(s, r, st);
                    }
                }
            }
            sl.parts.clear();
        }
        // results that have landed
        for (size_t i = 0; i < s->active.size();) {
            Request *r = s->active[i];
            if (r->state == RQ_FINALIZING) {
                const hipError_t q = hipEventQuery(r->p->ev_done);
                if (q != hipErrorNotReady) {
                    if (q == hipSuccess) {
                        complete(s, r);            // ev_done was seen complete above
                    } else {
                        finish(s, r, hip_fail(q, "result copy"));
                    }
                    continue;      // finish() removed active[i]
                }
            }
            ++i;
        }
        // launch rounds into free slots
        bool launched = false;
        for (RoundSlot &sl : s->slots) {
            if (sl.busy) continue;
            cls_status err = CLS_OK;
            if (launch_round(s, sl, &err)) launched = true;
            else if (err != CLS_OK) s->worker_error = err;
            if (!launched) break;
        }
        bool busy = false;
        for (const RoundSlot &sl : s->slots) busy = busy || sl.busy;
        bool finalizing = false;
        for (Request *r : s->active) finalizing = finalizing || r->state == RQ_FINALIZING;
        if (s->stop && s->pending.empty() && s->active.empty() && !busy) break;
        if (!busy && !finalizing && s->pending.empty() && !launched) {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        } else if (!launched) {
            // the GPU is working: poll again shortly, without the lock
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(100));
            lk.lock();
        }
    }
}

}  // namespace

extern "C" {

cls_status cls_server_create(const cls_server_config *cfg, cls_server **out)
{
    if (!out) return fail(CLS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    DeviceInfo di;
    cls_status st = device_info(&di);
    if (st != CLS_OK) return st;
    cls_server *s = new (std::nothrow) cls_server();
    if (!s) return fail(CLS_ERR_OUT_OF_MEMORY, "host allocation failed");
    if (cfg) s->cfg = *cfg;
    if (s->cfg.hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)1 << 32;
        s->cfg.hbm_budget_bytes = free_b / 10 * 8;
    }
    if (s->cfg.round_histories == 0) s->cfg.round_histories = 30000000ull;
    if (s->cfg.record_path != 0 && s->cfg.record_path != 1) {
        delete s;
        return fail(CLS_ERR_INVALID_ARG, "record_path must be 0 or 1");
    }
    if (s->cfg.max_inflight_rounds <= 0) s->cfg.max_inflight_rounds = 2;
    s->cfg.max_inflight_rounds = std::min(s->cfg.max_inflight_rounds, 8);
    s->device = di.id;
    s->di = di;
    s->t0 = Clock::now();
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    s->slots.resize((size_t)s->cfg.max_inflight_rounds);
    for (size_t i = 0; i < s->slots.size() && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&s->slots[i].ev, hipEventDisableTiming);
        s->slots[i].stream = (int)(i & 1);
    }
    if (e != hipSuccess) {
        cls_server_destroy(s);
        return hip_fail(e, "server streams");
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return CLS_OK;
}

cls_status cls_server_submit(cls_server *s, cls_problem *p, uint64_t histories, uint64_t seed, uint64_t *ticket)
{
    if (!s || !p || !ticket) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    if (histories == 0) return fail(CLS_ERR_INVALID_ARG, "histories must be >= 1");
    if (p->flags & CLS_F_TRACE) return fail(CLS_ERR_INVALID_ARG, "served requests do not record traces");
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(CLS_ERR_OUT_OF_MEMORY, "host allocation failed");
    r->p = p;
    r->histories = histories;
    r->seed = seed;
    r->footprint = workspace_bytes(p->nbins, 0);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return fail(CLS_ERR_STATE, "server is shutting down");
        }
        if (!s->in_flight.insert(p).second) {
            delete r;
            return fail(CLS_ERR_STATE, "this problem already has a request in flight");
        }
        r->stream = (int)(s->next_stream++ & 1u);
    }
    // The request's device side (allocation, chunking, record, tally reset)
    // is done here, in the caller's thread, when it runs on the server's
    // device, so that the worker does not hold the rounds back for it; no
    // other request of this problem can be in the server now.
    int dev = -1;
    cls_status st = CLS_OK;
    if (hipGetDevice(&dev) == hipSuccess && dev == s->device) st = prepare(s, r);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (st == CLS_OK && s->stop) st = fail(CLS_ERR_STATE, "server is shutting down");
        if (st != CLS_OK) {
            s->in_flight.erase(p);
            delete r;
            return st;
        }
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->pending.push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return CLS_OK;
}

cls_status cls_server_poll(cls_server *s, uint64_t ticket)
{
    if (!s) return fail(CLS_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(CLS_ERR_INVALID_ARG, "unknown ticket");
    const Request *r = it->second;
    if (r->state == RQ_DONE) return CLS_OK;
    if (r->state == RQ_FAILED) return fail(r->error, "request failed");
    return CLS_ERR_NOT_READY;
}

cls_status cls_server_wait(cls_server *s, uint64_t ticket, double timeout_s)
{
    if (!s) return fail(CLS_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                             std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 1e9));
    for (;;) {
        // looked up again after every wake: another thread may have released it
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return fail(CLS_ERR_INVALID_ARG, "unknown or released ticket");
        const Request *r = it->second;
        if (r->state == RQ_DONE) return CLS_OK;
        if (r->state == RQ_FAILED) return fail(r->error, "request failed");
        if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            it = s->all.find(ticket);
            if (it == s->all.end()) return fail(CLS_ERR_INVALID_ARG, "unknown or released ticket");
            if (it->second->state == RQ_DONE) return CLS_OK;
            if (it->second->state == RQ_FAILED) return fail(it->second->error, "request failed");
            return CLS_ERR_NOT_READY;
        }
    }
}

cls_status cls_server_request_info(cls_server *s, uint64_t ticket, cls_request_info *info)
{
    if (!s || !info) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(CLS_ERR_INVALID_ARG, "unknown ticket");
    const Request *r = it->second;
    std::memset(info, 0, sizeof *info);
    info->histories = r->histories;
    info->rounds = r->rounds;
    info->submit_s = seconds_since(s, r->t_submit);
    info->admit_s = r->state == RQ_PENDING ? -1.0 : seconds_since(s, r->t_admit);
    info->done_s = (r->state == RQ_DONE || r->state == RQ_FAILED) ? seconds_since(s, r->t_done) : -1.0;
    return CLS_OK;
}

cls_status cls_server_release(cls_server *s, uint64_t ticket)
{
    if (!s) return fail(CLS_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(CLS_ERR_INVALID_ARG, "unknown ticket");
    if (it->second->state != RQ_DONE && it->second->state != RQ_FAILED)
        return fail(CLS_ERR_NOT_READY, "request still running");
    delete it->second;
    s->all.erase(it);
    return CLS_OK;
}

cls_status cls_server_get_stats(cls_server *s, cls_server_stats *out)
{
    if (!s || !out) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof *out);
    out->submitted = s->next_ticket - 1;
    out->completed = s->completed;
    out->failed = s->failed;
    out->pending = s->pending.size();
    out->active = s->active.size();
    out->rounds = s->rounds;
    out->histories_completed = s->hist_done;
    out->hbm_in_use = s->in_use;
    out->hbm_peak = s->peak;
    out->hbm_budget = s->cfg.hbm_budget_bytes;
    out->worker_status = s->worker_error;
    return CLS_OK;
}

void cls_server_destroy(cls_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (RoundSlot &sl : s->slots) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    for (auto &kv : s->all) delete kv.second;
    delete s;
}

}  // extern "C"
