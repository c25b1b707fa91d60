// Continuous-batching CLS server.
//
// Requests (a problem, a history count and a seed) are admitted in arrival
// order while the device memory of their tallies fits the HBM budget: the
// tallies of admitted requests live in a server-owned device pool whose slabs
// are allocated, within the budget, only when admission needs them.
//
// A worker thread keeps one persistent tracking launch ("round") open at a
// time; the served kernel handles every geometry, estimator and source of one
// precision, so one round serves the whole mix of that precision. The worker
// feeds it through a queue of chunks in pinned host memory that the running
// kernel reads (ServedFeed): small requests are published whole as they
// arrive, large ones metered, about one chunk per wave ahead of the waves. A
// wave takes the next item index with one fetch-add on a device counter (a
// compare-and-swap claim collapses when thousands of waves contend for it) and
// runs the item once it is published. Requests that arrive while the round is
// open join it at once. The worker closes the round when it has nothing left
// to publish and its waves start running out of work (waves waiting in a
// round slow the waves that run; while most are still busy, requests that
// arrive join it at once instead of waiting for its last chunks and a fresh
// round), or after a time slice when a request it cannot take waits (the other
// precision, or a mesh finer than the round's LDS buffers); closing appends
// one leave item per wave, so every item before them runs and every wave
// leaves.
//
// The wave that flushes a request's last chunk stores the request's tag into
// its done word (pinned); the worker then launches a finalize kernel (one wave
// per request) that writes the record straight into the problem's pinned host
// record (or into device memory and a copy, record_path 1) and clears the
// tallies for the next request of that pool memory. Rounds leave a few
// workgroup slots free, so the finalize kernel runs while they do. A request
// whose chunks have all run without its done word, a wave that waited too long
// for its item, and an item the kernel refuses stop the server with an error:
// no request is left waiting for a completion that cannot come.
//
// Every history keeps the stream keyed by (seed, history index), and chunks
// are fixed by the request's history count, so a request's results do not
// depend on what it was batched with (integer tallies bitwise, FP64 sums up to
// the order of atomic additions).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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

// Round capacities: table entries (requests) and items (the last `waves` of
// them kept for the leave items that end the round).
constexpr int kMaxEntries = 4096;
constexpr uint64_t kMaxItems = 1u << 20;
// Workgroup slots a round leaves free for the finalize kernel.
constexpr int kReservedSlots = 8;
// Chunks of large requests published ahead of the waves' tickets, per wave.
constexpr uint64_t kBulkAheadPerWave = 1;
// A request of at most this many histories per resident wave is published
// whole when it arrives (about one chunk-time of the GPU).
constexpr uint64_t kPriorityHistoriesPerWave = 256;
// Time a round stays open while a request it cannot take is waiting.
constexpr double kSliceSeconds = 0.010;
// A round with nothing left to publish stays open while fewer than
// 1 / kIdleCloseShare of its waves wait for an item, for at most kDrySeconds
// (well within the waves' own wait limit).
constexpr uint64_t kIdleCloseShare = 8;
constexpr double kDrySeconds = 0.5;
// Mesh capacity of a round's LDS buffers, at least (the served mix fits).
constexpr int kServedMinBins = 1024;
// A wave with nothing to run gives up on its ticket after about kWaitSeconds
// of idle passes (a broken round), each s_sleep 127: 8128 shader cycles,
// 3.4 us at the top clock of 2.4 GHz and longer below it.
constexpr double kWaitSeconds = 5.0;
constexpr double kIdlePassSeconds = 127.0 * 64.0 / 2.4e9;
// Requests finalized by one finalize launch, and launches in flight.
constexpr int kFinalizeBatch = 256;
constexpr int kFinalizeSlots = 4;
// Pool: block sizes are powers of two from kBlockMin; a slab holds up to
// kSlabBlocks blocks of one size; kInitialBlocks blocks of each size up to
// kInitialMaxBlock are allocated and zeroed when the server is created.
constexpr size_t kBlockMin = 4096;
constexpr size_t kSlabBlocks = 64;
constexpr size_t kInitialBlocks = 16;
constexpr size_t kInitialMaxBlock = 64 * 1024;

enum ReqState { RQ_PENDING, RQ_ACTIVE, RQ_FINALIZING, RQ_DONE, RQ_FAILED };

struct Request {
    uint64_t ticket = 0;
    cls_problem *p = nullptr;
    Variant v;
    uint64_t histories = 0, seed = 0;
    uint64_t chunk = 0, n_chunks = 0;
    uint64_t next_chunk = 0;             // chunks not yet published
    uint64_t ran = 0;                    // chunks run in rounds that have ended
    bool priority = false;
    size_t footprint = 0;                // pool block bytes
    char *block = nullptr;               // device: counters, sums, [device record]
    ReqState state = RQ_PENDING;
    cls_status error = CLS_OK;
    Clock::time_point t_submit, t_admit, t_done;
    Clock::time_point t_publish, t_signal, t_finalize;
    bool published_any = false, signalled = false, finalize_launched = false;
    uint32_t rounds = 0;
    int last_round = -1;                 // round serial that last took chunks of it
    uint64_t tag = 0;
    uint64_t *done_host = nullptr;       // pinned done word
    uint64_t *done_dev = nullptr;
    uint64_t *host_record_dev = nullptr; // device address of p->h_record (record_path 0)
    int finalize_slot = -1;

    bool has_unpublished() const { return next_chunk < n_chunks; }
    uint64_t unpublished() const { return n_chunks - next_chunk; }
};

// Fixed pinned and device buffers of one round slot.
struct RoundSlot {
    int stream = 0;
    hipEvent_t ev = nullptr;
    bool busy = false;                   // launched, not yet retired
    bool open = false;                   // still fed (no leave items yet)
    int serial = -1;
    Variant v;
    Clock::time_point opened;
    bool dry = false;                    // nothing left to publish, since dry_since
    Clock::time_point dry_since;
    int grid = 0, block = 0, waves = 0, max_bins = 0;   // max_bins: mesh capacity of its LDS buffers
    size_t lds = 0;
    // pinned host: feed, items, the table of entry records
    char *host = nullptr;
    ServedFeed *feed = nullptr;
    uint64_t *items = nullptr;
    DevProblem *table = nullptr;
    ServedDev *dev_copy = nullptr;       // the round's ServedDev, copied back after it
    // their device addresses
    ServedFeed *feed_d = nullptr;
    uint64_t *items_d = nullptr;
    DevProblem *table_d = nullptr;
    // device: the ticket counter
    char *dev = nullptr;
    ServedDev *served_d = nullptr;
    uint64_t n_items = 0;               // items published, leave items included
    std::vector<Request *> entries;
    std::map<Request *, int> entry_of;
};

struct FinalizeSlot {
    DevProblem *host = nullptr, *dev = nullptr;   // pinned records and their device address
    hipEvent_t ev = nullptr;
    std::vector<Request *> reqs;
    bool busy = false;
};

struct Slab {
    char *base = nullptr;
    size_t block = 0, count = 0;
    hipEvent_t ready = nullptr;          // zeroing done (null: zeroed synchronously)
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
    std::set<const cls_problem *> in_flight;
    std::map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    size_t in_use = 0, peak = 0, pool_bytes = 0;
    hipStream_t streams[3] = {nullptr, nullptr, nullptr};   // two round streams, finalize
    RoundSlot slots[2];
    FinalizeSlot fin[kFinalizeSlots];
    std::vector<Slab> slabs;
    std::map<size_t, std::vector<char *>> free_blocks;     // block size -> free blocks
    // done words: pinned pages that never move, free words as (host, device)
    std::vector<uint64_t *> done_pages;
    std::vector<std::pair<uint64_t *, uint64_t *>> free_done;
    int round_serial = 0;
    uint64_t rounds = 0, completed = 0, failed = 0, hist_done = 0;
    uint64_t wave_ticks_alive = 0, wave_ticks_idle = 0;   // over the rounds retired
    bool dead = false;                   // a protocol error stopped the server
    Clock::time_point t0;
    cls_status worker_error = CLS_OK;
};

namespace {

double seconds_since(const cls_server *s, Clock::time_point t)
{
    return std::chrono::duration<double>(t - s->t0).count();
}

// The served kernel of the problem's precision (every kind of problem).
Variant served_variant(const cls_problem *p)
{
    Variant v = variant_of(p);
    v.geom = GEOM_ANY;
    v.est = -1;
    v.src = -1;
    v.served = true;
    return v;
}

// Mesh capacity of a round (or of the launch shape a request's chunks follow).
int served_bins(int nbins) { return std::min(CLS_MAX_BINS, std::max(kServedMinBins, nbins)); }

// ---------------------------------------------------------------------------
// device pool of request tallies (budgeted)
// ---------------------------------------------------------------------------
// A pool block: counters, sums, then (record_path 1) the device record.
size_t record_offset(int nbins)
{
    return align256(C_COUNT * sizeof(uint64_t)) + align256(sums_words(nbins) * sizeof(double));
}

size_t block_bytes(const cls_server *s, int nbins)
{
    size_t b = record_offset(nbins);
    if (s->cfg.record_path == 1) b += align256(record_words(nbins) * sizeof(uint64_t));
    size_t c = kBlockMin;
    while (c < b) c *= 2;
    return c;
}

// A slab of `count` blocks of `bytes`, zeroed before its blocks are handed out
// (synchronously, or on the finalize stream with an event to wait for).
cls_status add_slab(cls_server *s, size_t bytes, size_t count, bool sync)
{
    Slab sl;
    sl.block = bytes;
    sl.count = count;
    hipError_t e = hipMalloc((void **)&sl.base, bytes * count);
    if (e != hipSuccess) return fail(CLS_ERR_OUT_OF_MEMORY, std::string("server pool: ") + hipGetErrorString(e));
    if (sync) {
        e = hipMemset(sl.base, 0, bytes * count);
    } else {
        e = hipMemsetAsync(sl.base, 0, bytes * count, s->streams[2]);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(sl.ready, s->streams[2]);
    }
    if (e != hipSuccess) {
        (void)hipFree(sl.base);
        if (sl.ready) (void)hipEventDestroy(sl.ready);
        return hip_fail(e, "server pool zeroing");
    }
    s->slabs.push_back(sl);
    s->pool_bytes += bytes * count;
    auto &fl = s->free_blocks[bytes];
    for (size_t i = 0; i < count; ++i) fl.push_back(sl.base + i * bytes);
    return CLS_OK;
}

// A block of `bytes` from the pool into *out, or nullptr (wait) while none is
// free: a new slab is allocated when the budget allows it (and zeroed on the
// finalize stream before its blocks are handed out); when nothing else is
// admitted, one is allocated even beyond the budget, so a request never waits
// for memory that no other request will free. Free blocks are zero.
cls_status pool_alloc(cls_server *s, size_t bytes, char **out)
{
    *out = nullptr;
    auto &fl = s->free_blocks[bytes];
    bool zeroing = false;
    for (size_t i = 0; i < fl.size(); ++i) {
        char *b = fl[i];
        bool ready = true;
        for (Slab &sl : s->slabs)
            if (b >= sl.base && b < sl.base + sl.block * sl.count && sl.ready) {
                ready = hipEventQuery(sl.ready) == hipSuccess;
                if (ready) {
                    (void)hipEventDestroy(sl.ready);
                    sl.ready = nullptr;
                }
            }
        if (!ready) {
            zeroing = true;
            continue;
        }
        fl.erase(fl.begin() + (long)i);
        *out = b;
        return CLS_OK;
    }
    if (zeroing) return CLS_OK;
    const size_t room = s->cfg.hbm_budget_bytes > s->pool_bytes ? s->cfg.hbm_budget_bytes - s->pool_bytes : 0;
    size_t count = std::min<size_t>(kSlabBlocks, room / bytes);
    if (count == 0) {
        if (!s->active.empty()) return CLS_OK;
        count = 1;
    }
    const cls_status st = add_slab(s, bytes, count, false);
    return st;   // its blocks are usable once zeroed
}

void pool_free(cls_server *s, char *b, size_t bytes)
{
    if (b) s->free_blocks[bytes].push_back(b);
}

// ---------------------------------------------------------------------------
// requests
// ---------------------------------------------------------------------------
// A request reaches its final state (under the lock); waiters are woken on
// every path, failures included. Its pool block must be clear by then (the
// finalize kernel clears it) or is cleared here.
void finish(cls_server *s, Request *r, cls_status err)
{
    r->state = err == CLS_OK ? RQ_DONE : RQ_FAILED;
    r->error = err;
    r->t_done = Clock::now();
    if (r->block) s->in_use -= r->footprint;
    if (r->block) {
        if (err != CLS_OK) {
            // its tallies may be partly written: clear them before reuse
            (void)hipMemsetAsync(r->block, 0, r->footprint, s->streams[2]);
            (void)hipStreamSynchronize(s->streams[2]);
        }
        pool_free(s, r->block, r->footprint);
        r->block = nullptr;
    }
    if (err == CLS_OK) {
        ++s->completed;
        s->hist_done += r->histories;
    } else {
        ++s->failed;
    }
    s->active.erase(std::find(s->active.begin(), s->active.end(), r));
    s->in_flight.erase(r->p);
    if (r->done_host) s->free_done.push_back({r->done_host, r->done_dev});
    r->done_host = nullptr;
    s->cv_done.notify_all();
}

// The record a round's kernel uses for entry r (in the round's pinned table).
void entry_record(cls_server *s, Request *r, DevProblem *out)
{
    fill_dev_problem(r->p, r->histories, r->seed, r->chunk, 0, out);
    out->counters = (uint64_t *)r->block;
    out->sums = (double *)(r->block + align256(C_COUNT * sizeof(uint64_t)));
    out->record = nullptr;
    out->final_chunks = r->n_chunks;
    out->host_record = nullptr;
    out->done_word = r->done_dev;
    out->tag = r->tag;
}

// Admission (under the lock): a pool block within the budget.
bool admit(cls_server *s, Request *r, cls_status *err)
{
    char *b = nullptr;
    *err = pool_alloc(s, r->footprint, &b);
    if (*err != CLS_OK || !b) return false;
    r->block = b;
    r->t_admit = Clock::now();
    r->state = RQ_ACTIVE;
    s->in_use += r->footprint;
    s->peak = std::max(s->peak, s->in_use);
    return true;
}

// ---------------------------------------------------------------------------
// rounds
// ---------------------------------------------------------------------------
cls_status slot_buffers(cls_server *s, RoundSlot &sl)
{
    if (sl.host) return CLS_OK;
    const size_t feed_b = align256(sizeof(ServedFeed));
    const size_t items_b = align256(kMaxItems * sizeof(uint64_t));
    const size_t table_b = align256((size_t)kMaxEntries * sizeof(DevProblem));
    HIP_TRY(hipHostMalloc((void **)&sl.host, feed_b + items_b + table_b + align256(sizeof(ServedDev)),
                          hipHostMallocDefault));
    sl.feed = (ServedFeed *)sl.host;
    sl.items = (uint64_t *)(sl.host + feed_b);
    sl.table = (DevProblem *)(sl.host + feed_b + items_b);
    sl.dev_copy = (ServedDev *)(sl.host + feed_b + items_b + table_b);
    void *d = nullptr;
    HIP_TRY(hipHostGetDevicePointer(&d, sl.host, 0));
    char *hd = (char *)d;
    sl.feed_d = (ServedFeed *)hd;
    sl.items_d = (uint64_t *)(hd + feed_b);
    sl.table_d = (DevProblem *)(hd + feed_b + items_b);
    HIP_TRY(hipMalloc((void **)&sl.dev, align256(sizeof(ServedDev))));
    sl.served_d = (ServedDev *)sl.dev;
    HIP_TRY(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    (void)s;
    return CLS_OK;
}

// Whether request r may run in round sl: same kernel variant, and a mesh that
// fits the round's LDS tally buffers (fixed at launch).
bool fits(const RoundSlot &sl, const Request *r)
{
    return same_variant(r->v, sl.v) && r->p->nbins <= sl.max_bins;
}

// Items of the open round that are not leave items may use the queue up to
// here: the last `waves` places are kept for the leave items.
uint64_t item_room(const RoundSlot &sl)
{
    const uint64_t cap = kMaxItems - (uint64_t)sl.waves;
    return sl.n_items < cap ? cap - sl.n_items : 0;
}

// Publish up to `max_items` chunks of request r to the open round (the host
// writes the entry's record and the items, then raises `published`). Returns
// the count.
uint64_t publish(cls_server *s, RoundSlot &sl, Request *r, uint64_t max_items)
{
    if (!r->has_unpublished() || max_items == 0) return 0;
    auto it = sl.entry_of.find(r);
    int e;
    if (it == sl.entry_of.end()) {
        if ((int)sl.entries.size() >= kMaxEntries) return 0;
        e = (int)sl.entries.size();
        entry_record(s, r, &sl.table[e]);
        sl.entries.push_back(r);
        sl.entry_of[r] = e;
    } else {
        e = it->second;
    }
    uint64_t n = 0;
    const uint64_t room = item_room(sl);
    while (n < max_items && n < room && r->has_unpublished()) {
        sl.items[sl.n_items + n] = ((uint64_t)e << 32) | r->next_chunk++;
        ++n;
    }
    if (n) {
        sl.n_items += n;
        __atomic_store_n(&sl.feed->published, sl.n_items, __ATOMIC_RELEASE);
        if (!r->published_any) {
            r->published_any = true;
            r->t_publish = Clock::now();
        }
        if (r->last_round != sl.serial) {
            r->last_round = sl.serial;
            ++r->rounds;
        }
    }
    return n;
}

// The round takes no more work: one leave item per wave follows its items, so
// that every wave leaves once the items before them have all been taken.
void close_round(RoundSlot &sl)
{
    if (!sl.open) return;
    sl.open = false;
    for (int w = 0; w < sl.waves; ++w) sl.items[sl.n_items + (uint64_t)w] = kServedLeave;
    sl.n_items += (uint64_t)sl.waves;
    __atomic_store_n(&sl.feed->published, sl.n_items, __ATOMIC_RELEASE);
}

// Feed the open round: small requests whole as they come, large ones metered
// to kBulkAheadPerWave chunks per wave beyond the tickets the waves reported.
void feed_round(cls_server *s, RoundSlot &sl)
{
    bool full = false;
    for (Request *r : s->active) {
        if (r->state != RQ_ACTIVE || !r->priority || !fits(sl, r) || !r->has_unpublished()) continue;
        publish(s, sl, r, r->unpublished());
        full = full || r->has_unpublished();
    }
    const uint64_t seen = __atomic_load_n(&sl.feed->seen, __ATOMIC_ACQUIRE);
    const uint64_t target = (uint64_t)sl.waves * kBulkAheadPerWave + 64;
    uint64_t ahead = sl.n_items > seen ? sl.n_items - seen : 0;
    for (Request *r : s->active) {
        if (ahead >= target) break;
        if (r->state != RQ_ACTIVE || r->priority || !fits(sl, r) || !r->has_unpublished()) continue;
        ahead += publish(s, sl, r, target - ahead);
        full = full || (r->has_unpublished() && ahead < target);
    }
    // a round that cannot take more entries or items is closed
    if (full || item_room(sl) == 0) close_round(sl);
}

bool round_has_work(cls_server *s, const RoundSlot &sl)
{
    for (Request *r : s->active)
        if (r->state == RQ_ACTIVE && fits(sl, r) && r->has_unpublished()) return true;
    return false;
}

// Whether the round's waves run out of work: at least 1 / kIdleCloseShare of
// them hold a ticket beyond the published items (the waves report every 32nd
// ticket they take).
bool round_draining(const RoundSlot &sl)
{
    const uint64_t seen = __atomic_load_n(&sl.feed->seen, __ATOMIC_ACQUIRE);
    const uint64_t waiting = seen > sl.n_items ? seen - sl.n_items : 0;
    return waiting * kIdleCloseShare >= (uint64_t)sl.waves;
}

// Launch a round of variant v in a free slot, fed with what is waiting.
cls_status open_round(cls_server *s, RoundSlot &sl, const Variant &v)
{
    cls_status st = slot_buffers(s, sl);
    if (st != CLS_OK) return st;
    // the mesh capacity of the round's LDS buffers: kServedMinBins, or the
    // finest mesh waiting; a request with a finer one that arrives later waits
    // for a later round
    int max_bins = kServedMinBins;
    for (Request *r : s->active)
        if (r->state == RQ_ACTIVE && same_variant(r->v, v) && r->has_unpublished())
            max_bins = std::max(max_bins, r->p->nbins);
    max_bins = served_bins(max_bins);
    int grid, block, stride;
    size_t lds;
    LaunchShape used;
    // one LDS tally buffer per wave (about twice the resident waves of two):
    // a round is shaped when it opens, before most of the requests it will
    // carry have arrived, and the served mix's histories are nearly all in
    // large chunks; the small requests' chunks pay the wait for their last
    // history (measured: saturated mix 1.52e10 against 1.10e10 histories/s,
    // a lone request of 1e4 histories 0.87 against 0.65 ms)
    st = shape_for(v, max_bins, s->di, &grid, &block, &lds, &stride, &used,
                   [](uint64_t, uint64_t) { return 0.0; });
    if (st != CLS_OK) return st;
    grid = std::max(1, grid - kReservedSlots);
    sl.v = v;
    sl.serial = s->round_serial++;
    sl.grid = grid;
    sl.block = block;
    sl.lds = lds;
    sl.waves = grid * (block / 64);
    sl.max_bins = max_bins;
    sl.n_items = 0;
    sl.entries.clear();
    sl.entry_of.clear();
    std::memset(sl.feed, 0, sizeof(ServedFeed));
    sl.open = true;
    sl.opened = Clock::now();
    sl.dry = false;
    // only requests whose mesh fits the round's buffers are fed to it
    feed_round(s, sl);
    hipStream_t stream = s->streams[sl.stream];
    HIP_TRY(hipMemsetAsync(sl.dev, 0, sizeof(ServedDev), stream));
    TrackArgs a;
    a.probs = sl.table_d;
    a.item_start = nullptr;
    a.queue_head = nullptr;
    a.nprobs = kMaxEntries;
    a.lds_stride = stride;
    a.refill_min = used.refill_min;
    a.slots = used.slots;
    a.feed = sl.feed_d;
    a.items = sl.items_d;
    a.served = sl.served_d;
    a.wait_passes = (uint64_t)(kWaitSeconds / kIdlePassSeconds);
    HIP_TRY(launch_track(v, a, grid, block, lds, stream));
    HIP_TRY(hipMemcpyAsync(sl.dev_copy, sl.dev, sizeof(ServedDev), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipEventRecord(sl.ev, stream));
    sl.busy = true;
    ++s->rounds;
    return CLS_OK;
}

// A round whose launch has completed: chunks it published but never ran go
// back to their requests.
// A protocol error: every request not yet finalizing fails with `err`, and
// the server takes no more (its rounds drain; destroy still works).
void stop_server(cls_server *s, cls_status err)
{
    s->dead = true;
    s->worker_error = err;
    while (!s->pending.empty()) {
        s->active.push_back(s->pending.front());
        s->pending.pop_front();
    }
    std::vector<Request *> victims;
    for (Request *r : s->active)
        if (r->state == RQ_ACTIVE || r->state == RQ_PENDING) victims.push_back(r);
    for (Request *r : victims) finish(s, r, err);
}

// A round whose launch has completed: its waves took every item before the
// leave items, so every chunk it published has run.
void retire_round(cls_server *s, RoundSlot &sl, hipError_t q)
{
    sl.busy = false;
    sl.open = false;
    if (q == hipSuccess) {
        s->wave_ticks_alive += sl.dev_copy->alive_ticks;
        s->wave_ticks_idle += sl.dev_copy->idle_ticks;
    }
    for (uint64_t i = 0; i < sl.n_items; ++i)
        if (sl.items[i] != kServedLeave) ++sl.entries[(size_t)(sl.items[i] >> 32)]->ran;
    if (q != hipSuccess) {
        const cls_status err = hip_fail(q, "served round");
        s->worker_error = err;
        for (Request *r : sl.entries)
            if (r->state == RQ_ACTIVE) finish(s, r, err);
    } else if (const uint64_t code = __atomic_load_n(&sl.feed->error, __ATOMIC_ACQUIRE)) {
        const uint64_t it = __atomic_load_n(&sl.feed->error_item, __ATOMIC_ACQUIRE);
        stop_server(s, fail(CLS_ERR_DEVICE,
                            code == kServedErrWait
                                ? "served round: a wave waited too long for item " + std::to_string(it)
                                : "served round refused item (entry " + std::to_string(it >> 32) + ", chunk " +
                                      std::to_string(it & 0xFFFFFFFFull) + "): not a chunk of a request in its table"));
    } else {
        // the launch has completed, so the done word of a request whose chunks
        // have all run is visible by now
        for (Request *r : sl.entries)
            if (r->state == RQ_ACTIVE && r->ran == r->n_chunks &&
                __atomic_load_n(r->done_host, __ATOMIC_ACQUIRE) != r->tag) {
                stop_server(s, fail(CLS_ERR_DEVICE, "served request " + std::to_string(r->ticket) +
                                                        ": every chunk ran but no completion was signalled"));
                break;
            }
    }
    sl.entries.clear();
    sl.entry_of.clear();
}

// ---------------------------------------------------------------------------
// finalize
// ---------------------------------------------------------------------------
cls_status fin_buffers(FinalizeSlot &f)
{
    if (f.host) return CLS_OK;
    HIP_TRY(hipHostMalloc((void **)&f.host, kFinalizeBatch * sizeof(DevProblem), hipHostMallocDefault));
    void *d = nullptr;
    HIP_TRY(hipHostGetDevicePointer(&d, f.host, 0));
    f.dev = (DevProblem *)d;
    HIP_TRY(hipEventCreateWithFlags(&f.ev, hipEventDisableTiming));
    return CLS_OK;
}

// Finalize the requests whose done word is set (one launch per batch).
void start_finalizes(cls_server *s)
{
    std::vector<Request *> ready;
    for (Request *r : s->active)
        if (r->state == RQ_ACTIVE && __atomic_load_n(r->done_host, __ATOMIC_ACQUIRE) == r->tag) {
            if (!r->signalled) {
                r->signalled = true;
                r->t_signal = Clock::now();
            }
            ready.push_back(r);
        }
    size_t k = 0;
    while (k < ready.size()) {
        FinalizeSlot *f = nullptr;
        for (FinalizeSlot &x : s->fin)
            if (!x.busy) f = &x;
        if (!f) return;   // all in flight: the rest waits for the next pass
        cls_status st = fin_buffers(*f);
        if (st != CLS_OK) {
            s->worker_error = st;
            return;
        }
        f->reqs.clear();
        for (; k < ready.size() && (int)f->reqs.size() < kFinalizeBatch; ++k) {
            Request *r = ready[k];
            DevProblem *rec = &f->host[f->reqs.size()];
            entry_record(s, r, rec);
            rec->record = s->cfg.record_path == 0 && r->host_record_dev
                              ? r->host_record_dev
                              : (uint64_t *)(r->block + record_offset(r->p->nbins));
            r->state = RQ_FINALIZING;
            r->finalize_launched = true;
            r->t_finalize = Clock::now();
            f->reqs.push_back(r);
        }
        hipStream_t st_ = s->streams[2];
        hipError_t e = launch_finalize_clear(f->dev, (int)f->reqs.size(), st_);
        for (size_t i = 0; i < f->reqs.size() && e == hipSuccess; ++i) {
            Request *r = f->reqs[i];
            if (f->host[i].record != r->host_record_dev || !r->host_record_dev)
                e = hipMemcpyAsync(r->p->h_record, f->host[i].record, record_words(r->p->nbins) * sizeof(uint64_t),
                                   hipMemcpyDeviceToHost, st_);
        }
        if (e == hipSuccess) e = hipEventRecord(f->ev, st_);
        if (e != hipSuccess) {
            const cls_status err = hip_fail(e, "served finalize");
            for (Request *r : f->reqs) finish(s, r, err);
            f->reqs.clear();
            continue;
        }
        f->busy = true;
    }
}

// A request whose record is in its problem's host record.
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

void retire_finalizes(cls_server *s)
{
    for (FinalizeSlot &f : s->fin) {
        if (!f.busy) continue;
        const hipError_t q = hipEventQuery(f.ev);
        if (q == hipErrorNotReady) continue;
        f.busy = false;
        for (Request *r : f.reqs) {
            if (q == hipSuccess) complete(s, r);
            else finish(s, r, hip_fail(q, "served finalize"));
        }
        f.reqs.clear();
    }
}

// ---------------------------------------------------------------------------
// worker
// ---------------------------------------------------------------------------
void worker_main(cls_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // admit in arrival order while the pool allows
        while (!s->pending.empty()) {
            Request *r = s->pending.front();
            cls_status err = CLS_OK;
            const bool ok = admit(s, r, &err);
            if (!ok && err == CLS_OK) break;   // waits for memory
            s->pending.pop_front();
            s->active.push_back(r);
            if (!ok) finish(s, r, err);
        }
        // results: done words -> finalize -> host records
        retire_finalizes(s);
        start_finalizes(s);
        // retire rounds whose launch completed
        for (RoundSlot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            retire_round(s, sl, q);
        }
        // feed the open round. It is closed once it has nothing left to
        // publish and its waves start to run out of work (waves waiting in a
        // round slow the ones that run, so they leave soon; while most are
        // busy with their last chunks, a request that arrives joins the round
        // at once), and after a slice when a request it cannot take waits
        // (other precision, finer mesh).
        RoundSlot *open = nullptr;
        for (RoundSlot &sl : s->slots)
            if (sl.busy && sl.open) open = &sl;
        if (open) {
            bool other = false;
            for (Request *r : s->active)
                if (r->state == RQ_ACTIVE && r->has_unpublished() && !fits(*open, r)) other = true;
            const Clock::time_point now = Clock::now();
            const double age = std::chrono::duration<double>(now - open->opened).count();
            const bool has_work = round_has_work(s, *open);
            if (has_work) {
                open->dry = false;
            } else if (!open->dry) {
                open->dry = true;
                open->dry_since = now;
            }
            const bool dry_long =
                open->dry && std::chrono::duration<double>(now - open->dry_since).count() >= kDrySeconds;
            if ((!has_work && (round_draining(*open) || dry_long)) || (other && age >= kSliceSeconds)) {
                close_round(*open);
                open = nullptr;
            } else {
                feed_round(s, *open);
                if (!open->open) open = nullptr;
            }
        }
        // open a round for the precision of the oldest waiting request
        if (!open && !s->dead) {
            Request *oldest = nullptr;
            for (Request *r : s->active)
                if (r->state == RQ_ACTIVE && r->has_unpublished()) {
                    bool running_open = false;
                    for (RoundSlot &sl : s->slots) running_open = running_open || (sl.busy && sl.open && fits(sl, r));
                    if (!running_open && (!oldest || r->ticket < oldest->ticket)) oldest = r;
                }
            if (oldest) {
                for (RoundSlot &sl : s->slots) {
                    if (sl.busy) continue;
                    const cls_status st = open_round(s, sl, oldest->v);
                    if (st != CLS_OK) {
                        s->worker_error = st;
                        const Variant v = oldest->v;
                        std::vector<Request *> victims;
                        for (Request *r : s->active)
                            if (r->state == RQ_ACTIVE && same_variant(r->v, v)) victims.push_back(r);
                        for (Request *r : victims) finish(s, r, st);
                    }
                    break;
                }
            }
        }
        bool busy = false;
        for (const RoundSlot &sl : s->slots) busy = busy || sl.busy;
        for (const FinalizeSlot &f : s->fin) busy = busy || f.busy;
        if (s->stop && s->pending.empty() && s->active.empty() && !busy) break;
        if (!busy && s->active.empty() && s->pending.empty()) {
            s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        } else {
            // the GPU is working: poll again shortly, without the lock
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            lk.lock();
        }
    }
}

// Pinned result record of the problem (host side only) and its device address.
cls_status host_record_of(cls_problem *p, uint64_t **dev)
{
    if (!p->h_record)
        HIP_TRY(hipHostMalloc((void **)&p->h_record, record_words(p->nbins) * sizeof(uint64_t), hipHostMallocDefault));
    void *d = nullptr;
    *dev = hipHostGetDevicePointer(&d, p->h_record, 0) == hipSuccess ? (uint64_t *)d : nullptr;
    return CLS_OK;
}

}  // namespace

extern "C" {

cls_status cls_server_create(const cls_server_config *cfg, cls_server **out)
{
    if (!out) return fail(CLS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (cfg && cfg->record_path != 0 && cfg->record_path != 1)
        return fail(CLS_ERR_INVALID_ARG, "record_path must be 0 or 1");
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
    s->cfg.max_inflight_rounds = 2;
    s->device = di.id;
    s->di = di;
    s->t0 = Clock::now();
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    for (int i = 0; i < 2; ++i) s->slots[i].stream = i;
    if (e != hipSuccess) {
        cls_server_destroy(s);
        return hip_fail(e, "server streams");
    }
    // buffers of the rounds and finalize launches, and a first slab of each
    // small block size within the budget, before any request waits for them
    for (int i = 0; i < 2 && st == CLS_OK; ++i) st = slot_buffers(s, s->slots[i]);
    for (int i = 0; i < kFinalizeSlots && st == CLS_OK; ++i) st = fin_buffers(s->fin[i]);
    for (size_t b = kBlockMin; b <= kInitialMaxBlock && st == CLS_OK; b *= 2)
        if (s->pool_bytes + kInitialBlocks * b <= s->cfg.hbm_budget_bytes) st = add_slab(s, b, kInitialBlocks, true);
    if (st != CLS_OK) {
        cls_server_destroy(s);
        return st;
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
    if (p->device >= 0 && p->device != s->device)
        return fail(CLS_ERR_STATE, "problem was first run on another device");
    if (p->nbins > CLS_MAX_BINS) return fail(CLS_ERR_INVALID_ARG, "nbins above CLS_MAX_BINS");
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(CLS_ERR_OUT_OF_MEMORY, "host allocation failed");
    r->p = p;
    r->v = served_variant(p);
    r->histories = histories;
    r->seed = seed;
    r->t_submit = Clock::now();
    // chunks fixed by the request alone (never by the mix it meets), for the
    // waves of a round (one LDS buffer per wave, as open_round shapes it): at
    // least kMinErrorBatches when the history count allows, up to one wave's
    // share of round_histories, a whole number per wave for large requests
    int grid, block, stride;
    size_t lds;
    LaunchShape sh;
    cls_status st = shape_for(r->v, served_bins(p->nbins), s->di, &grid, &block, &lds, &stride, &sh,
                              [](uint64_t, uint64_t) { return 0.0; });
    uint64_t *rec_dev = nullptr;
    if (st == CLS_OK) st = host_record_of(p, &rec_dev);
    if (st != CLS_OK) {
        delete r;
        return st;
    }
    const uint64_t waves_total = (uint64_t)std::max(1, grid - kReservedSlots) * (uint64_t)(block / 64);
    const uint64_t round_share = std::max<uint64_t>(1, s->cfg.round_histories / waves_total);
    r->chunk = served_chunk_size(histories, waves_total, (uint64_t)sh.max_chunk, round_share);
    r->n_chunks = (histories + r->chunk - 1) / r->chunk;
    r->priority = histories <= kPriorityHistoriesPerWave * waves_total;
    r->footprint = block_bytes(s, p->nbins);
    r->host_record_dev = rec_dev;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return fail(CLS_ERR_STATE, "server is shutting down");
        }
        if (s->dead) {
            delete r;
            return fail(CLS_ERR_STATE, "server stopped after a device error");
        }
        if (!s->in_flight.insert(p).second) {
            delete r;
            return fail(CLS_ERR_STATE, "this problem already has a request in flight");
        }
        // a done word (pinned) for the request, from pages of 1024
        if (s->free_done.empty()) {
            constexpr size_t kPage = 1024;
            uint64_t *page = nullptr;
            void *d = nullptr;
            if (hipHostMalloc((void **)&page, kPage * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
                s->in_flight.erase(p);
                delete r;
                return fail(CLS_ERR_OUT_OF_MEMORY, "done words");
            }
            s->done_pages.push_back(page);
            if (hipHostGetDevicePointer(&d, page, 0) != hipSuccess) {
                s->in_flight.erase(p);
                delete r;
                return fail(CLS_ERR_DEVICE, "done words are not device-addressable");
            }
            std::memset(page, 0, kPage * sizeof(uint64_t));
            for (size_t i = 0; i < kPage; ++i) s->free_done.push_back({page + i, (uint64_t *)d + i});
        }
        r->done_host = s->free_done.back().first;
        r->done_dev = s->free_done.back().second;
        s->free_done.pop_back();
        r->ticket = s->next_ticket++;
        r->tag = r->ticket;
        __atomic_store_n(r->done_host, 0ull, __ATOMIC_RELEASE);
        s->all[r->ticket] = r;
        s->pending.push_back(r);
        p->device = s->device;
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
    info->publish_s = r->published_any ? seconds_since(s, r->t_publish) : -1.0;
    info->signal_s = r->signalled ? seconds_since(s, r->t_signal) : -1.0;
    info->finalize_s = r->finalize_launched ? seconds_since(s, r->t_finalize) : -1.0;
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
    out->wave_idle_share = s->wave_ticks_alive ? (double)s->wave_ticks_idle / (double)s->wave_ticks_alive : 0.0;
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
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamSynchronize(st);
    for (RoundSlot &sl : s->slots) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    for (FinalizeSlot &f : s->fin) {
        if (f.host) (void)hipHostFree(f.host);
        if (f.ev) (void)hipEventDestroy(f.ev);
    }
    for (Slab &sl : s->slabs) {
        if (sl.base) (void)hipFree(sl.base);
        if (sl.ready) (void)hipEventDestroy(sl.ready);
    }
    for (uint64_t *page : s->done_pages) (void)hipHostFree(page);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    for (auto &kv : s->all) delete kv.second;
    delete s;
}

}  // extern "C"
