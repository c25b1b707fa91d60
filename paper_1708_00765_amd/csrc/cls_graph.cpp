// Graph-captured batches: the reset -> track -> finalize -> copy-back sequence
// of one batched persistent launch is captured once in a hipGraph and replayed
// for every later run of the same set of problems. The graph reads the
// problem records and work-queue prefix sums from pinned host memory that each
// run rewrites, so histories and seeds may change between replays; the launch
// shape (grid, workgroup, LDS buffers per wave) is chosen for the history
// counts of the first run and fixed at its capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "cls_runtime.hpp"

using namespace cls;
using namespace cls::rt;

struct cls_batch {
    std::vector<cls_problem *> probs;
    Variant v{};
    int device = -1;
    hipStream_t stream = nullptr;
    char *dev = nullptr;
    char *host = nullptr;
    size_t probs_bytes = 0, items_bytes = 0, rec_words = 0;
    int max_bins = 1;
    int grid = 0, block = 0, stride = 0, refill_min = 1, slots = 2;
    size_t lds = 0;
    uint64_t max_chunk = 0, waves_total = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr, done = nullptr;
};

static void batch_release(cls_batch *b)
{
    if (b->done) (void)hipEventSynchronize(b->done);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dev) (void)hipFree(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    if (b->t0) (void)hipEventDestroy(b->t0);
    if (b->t1) (void)hipEventDestroy(b->t1);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

// Capture the launch sequence on the batch's own stream.
static cls_status capture(cls_batch *b)
{
    const int n = (int)b->probs.size();
    DevProblem *d_probs = (DevProblem *)b->dev;
    uint64_t *d_items = (uint64_t *)(b->dev + b->probs_bytes);
    uint64_t *d_rec = (uint64_t *)(b->dev + b->probs_bytes + b->items_bytes);
    uint64_t *h_rec = (uint64_t *)(b->host + b->probs_bytes + b->items_bytes);
    TrackArgs a;
    a.probs = d_probs;
    a.item_start = d_items;
    a.queue_head = d_items + n + 1;
    a.nprobs = n;
    a.lds_stride = b->stride;
    a.refill_min = b->refill_min;
    a.slots = b->slots;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipMemcpyAsync(b->dev, b->host, b->probs_bytes + b->items_bytes, hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess) e = launch_reset(d_probs, n, d_items + n + 1, b->stream);
    if (e == hipSuccess) e = launch_track(b->v, a, b->grid, b->block, b->lds, b->stream);
    if (e == hipSuccess) e = launch_finalize(d_probs, n, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_rec, d_rec, b->rec_words * sizeof(uint64_t), hipMemcpyDeviceToHost, b->stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e, "graph capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return CLS_OK;
}

extern "C" {

cls_status cls_batch_create(cls_problem *const *problems, int n, cls_batch **out)
{
    if (!out) return fail(CLS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    cls_status st = check_problem_set(problems, n, nullptr, nullptr, "batch");
    if (st != CLS_OK) return st;
    for (int i = 0; i < n; ++i)
        if (problems[i]->flags & CLS_F_TRACE) return fail(CLS_ERR_INVALID_ARG, "graph batches do not record traces");
    DeviceInfo di;
    st = device_info(&di);
    if (st != CLS_OK) return st;
    cls_batch *b = new (std::nothrow) cls_batch();
    if (!b) return fail(CLS_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->probs.assign(problems, problems + n);
    b->v = variant_of(problems[0]);
    b->device = di.id;
    for (int i = 0; i < n; ++i) {
        st = ensure_device(problems[i], 0);
        if (st != CLS_OK) { batch_release(b); delete b; return st; }
        b->max_bins = std::max(b->max_bins, problems[i]->nbins);
        b->rec_words += record_words(problems[i]->nbins);
    }
    b->probs_bytes = align256((size_t)n * sizeof(DevProblem));
    b->items_bytes = align256(((size_t)n + 2) * sizeof(uint64_t));
    const size_t bytes = b->probs_bytes + b->items_bytes + align256(b->rec_words * sizeof(uint64_t));
    hipError_t e = hipMalloc((void **)&b->dev, bytes);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->host, bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&b->t0);
    if (e == hipSuccess) e = hipEventCreate(&b->t1);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_release(b);
        delete b;
        return fail(CLS_ERR_OUT_OF_MEMORY, std::string("batch allocation: ") + hipGetErrorString(e));
    }
    *out = b;
    return CLS_OK;
}

cls_status cls_batch_run(cls_batch *b, const uint64_t *histories, const uint64_t *seeds)
{
    if (!b || !histories || !seeds) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    const int n = (int)b->probs.size();
    uint64_t total = 0;
    const cls_status chk = check_problem_set(b->probs.data(), n, histories, &total, "batch");
    if (chk != CLS_OK) return chk;
    for (cls_problem *p : b->probs)
        if (p->has_run && !p->done_synced) HIP_TRY(hipEventSynchronize(p->ev_done));
    DevProblem *h_probs = (DevProblem *)b->host;
    uint64_t *h_items = (uint64_t *)(b->host + b->probs_bytes);
    uint64_t *h_rec = (uint64_t *)(b->host + b->probs_bytes + b->items_bytes);
    uint64_t *d_rec = (uint64_t *)(b->dev + b->probs_bytes + b->items_bytes);
    h_items[0] = 0;
    size_t off = 0;
    if (!b->exec) {
        // launch shape for the history counts of this (first) run
        DeviceInfo di;
        cls_status st = device_info(&di);
        if (st != CLS_OK) return st;
        LaunchShape used;
        st = shape_for(b->v, b->max_bins, di, &b->grid, &b->block, &b->lds, &b->stride, &used,
                       [&](uint64_t waves_total, uint64_t max_chunk) {
                           double small = 0.0;
                           for (int i = 0; i < n; ++i)
                               if (batch_chunk_size(histories[i], total, waves_total, max_chunk) <
                                   kSingleSlotMinChunk)
                                   small += (double)histories[i];
                           return small / (double)total;
                       });
        if (st != CLS_OK) return st;
        b->refill_min = used.refill_min;
        b->slots = used.slots;
        b->max_chunk = (uint64_t)used.max_chunk;
        b->waves_total = (uint64_t)b->grid * (uint64_t)(b->block / 64);
    }
    for (int i = 0; i < n; ++i) {
        cls_problem *p = b->probs[i];
        const uint64_t chunk = batch_chunk_size(histories[i], total, b->waves_total, b->max_chunk);
        fill_dev_problem(p, histories[i], seeds[i], chunk, 0, &h_probs[i]);
        h_probs[i].batch_max = batch_limit(histories[i], chunk, current_shape());
        h_probs[i].record = d_rec + off;
        off += record_words(p->nbins);
        h_items[i + 1] = h_items[i] + (histories[i] + chunk - 1) / chunk;
    }
    h_items[n + 1] = 0;
    if (!b->exec) {
        const cls_status st = capture(b);
        if (st != CLS_OK) return st;
    }
    HIP_TRY(hipEventRecord(b->t0, b->stream));
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    HIP_TRY(hipEventRecord(b->t1, b->stream));
    HIP_TRY(hipEventRecord(b->done, b->stream));
    HIP_TRY(hipEventSynchronize(b->done));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, b->t0, b->t1));
    off = 0;
    bool capped = false;
    for (int i = 0; i < n; ++i) {
        cls_problem *p = b->probs[i];
        std::memcpy(p->h_record, h_rec + off, record_words(p->nbins) * sizeof(uint64_t));
        off += record_words(p->nbins);
        p->has_run = true;
        p->done_synced = true;
        p->timed_by_events = false;
        p->track_ms = ms;
        p->histories = histories[i];
        p->seed = seeds[i];
        p->trace_n = 0;
        capped = capped || p->h_record[C_CAPPED] != 0;
    }
    if (capped) return fail(CLS_ERR_EVENT_CAP, "a history reached the flight cap");
    return CLS_OK;
}

cls_status cls_batch_last_ms(const cls_batch *b, double *ms)
{
    if (!b || !ms) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    float f = 0.0f;
    HIP_TRY(hipEventElapsedTime(&f, b->t0, b->t1));
    *ms = f;
    return CLS_OK;
}

void cls_batch_destroy(cls_batch *b)
{
    if (!b) return;
    batch_release(b);
    delete b;
}

}  // extern "C"
