// Allocation-free run of one CLS problem (cls_run_static).
//
// For callers that cannot allocate device or pinned memory (work captured into
// a HIP graph, tight serving loops, harnesses that forbid hipMalloc): the
// run's device workspace -- the problem record, the work-queue prefix and
// head, the integer tallies and the FP64 flux sums -- lives in the file-scope
// array `scratch` below, which the library holds on every device it runs on
// until the process ends. The problem's parameters reach the device as kernel
// arguments of a set-up kernel that also zeroes the tallies (a kernel rather
// than a memset, so the sequence can be captured in a graph); the tracking and
// finalize kernels are those of cls_run_async, and the finalize kernel writes
// the result record straight into the caller's device buffer.
//
// All calls on one device share its array and each call overwrites it: calls
// that overlap on a device (two streams, or two host threads) race and give
// wrong results. Sequential calls, on any streams ordered by the caller, are
// independent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "cls_runtime.hpp"

using namespace cls;
using namespace cls::rt;

namespace {

// Largest flux mesh of an allocation-free run (below CLS_MAX_BINS, to keep the
// array modest), and the scratch size it needs: the problem record, the queue
// words, C_COUNT counters and 3 + 3K sums, each section 256-byte aligned (50 KB
// for 2048 bins).
constexpr int kStaticMaxBins = 2048;
constexpr size_t kScratchBytes = 64 * 1024;

constexpr size_t kProbOff = 0;
constexpr size_t kItemsOff = 512;                       // >= align256(sizeof(DevProblem))
constexpr size_t kCountersOff = kItemsOff + 256;        // [0] = 0, [1] = items, [2] = queue head
constexpr size_t kSumsOff = kCountersOff + 256;         // C_COUNT u64 counters
static_assert(sizeof(DevProblem) <= kItemsOff - kProbOff, "problem record exceeds its scratch section");
static_assert(C_COUNT * sizeof(uint64_t) <= 256, "counters exceed their scratch section");
static_assert(kSumsOff + sums_words(kStaticMaxBins) * sizeof(double) <= kScratchBytes,
              "flux sums of the largest mesh exceed the scratch array");

}  // namespace

// The device workspace of allocation-free runs. Host code never uses this
// name as an address: it takes the device address from hipGetSymbolAddress
// (see scratch_address) and passes that to the kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Writes the problem record into the workspace and zeroes the tallies and the
// work-queue head; items = number of work chunks of the run.
__global__ void static_setup_kernel(DevProblem prob, DevProblem *dst, uint64_t *items, uint64_t n_items)
{
    const int t = (int)threadIdx.x;
    if (t == 0) {
        *dst = prob;
        items[0] = 0;
        items[1] = n_items;
        items[2] = 0;   // queue head
        items[3] = 0;
    }
    for (int i = t; i < C_COUNT; i += (int)blockDim.x) prob.counters[i] = 0ull;
    for (int i = t; i < (int)sums_words(prob.nbins); i += (int)blockDim.x) prob.sums[i] = 0.0;
}

// Device address of `scratch` per device, taken once per device with that
// device current.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char *g_scratch[kMaxDevices] = {};

cls_status scratch_address(int device, char **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(CLS_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr & 255u)) return fail(CLS_ERR_DEVICE, "scratch array has no aligned address");
        g_scratch[device] = (char *)ptr;
    }
    *out = g_scratch[device];
    return CLS_OK;
}

}  // namespace

extern "C" cls_status cls_run_static(const cls_problem *p, uint64_t histories, uint64_t seed, void *hip_stream,
                                     void *d_record, size_t record_bytes)
{
    if (!p || !d_record) return fail(CLS_ERR_INVALID_ARG, "NULL problem or record");
    if (histories == 0) return fail(CLS_ERR_INVALID_ARG, "histories must be >= 1");
    if (p->flags & CLS_F_TRACE) return fail(CLS_ERR_INVALID_ARG, "allocation-free runs record no trace");
    if (p->nbins > kStaticMaxBins)
        return fail(CLS_ERR_INVALID_ARG, "allocation-free runs take meshes of at most " +
                                             std::to_string(kStaticMaxBins) + " bins");
    if (record_bytes < record_words(p->nbins) * sizeof(uint64_t))
        return fail(CLS_ERR_INVALID_ARG, "record buffer smaller than (24 + 2 nbins) x 8 bytes");
    if ((uintptr_t)d_record & 7u) return fail(CLS_ERR_INVALID_ARG, "record buffer must be 8-byte aligned");
    DeviceInfo di;
    cls_status st = device_info(&di);
    if (st != CLS_OK) return st;
    char *base = nullptr;
    st = scratch_address(di.id, &base);
    if (st != CLS_OK) return st;
    // launch shape and chunks exactly as cls_run_async chooses them, so the
    // results equal that entry point's (integer tallies bitwise)
    const Variant v = variant_of(p);
    int grid, block, stride;
    size_t lds;
    LaunchShape used;
    st = shape_for(v, p->nbins, di, &grid, &block, &lds, &stride, &used,
                   [histories](uint64_t waves_total, uint64_t max_chunk) {
                       return chunk_size(histories, waves_total, max_chunk) < kSingleSlotMinChunk ? 1.0 : 0.0;
                   });
    if (st != CLS_OK) return st;
    const uint64_t waves_total = (uint64_t)grid * (uint64_t)(block / 64);
    const uint64_t chunk = chunk_size(histories, waves_total, (uint64_t)used.max_chunk);
    const uint64_t n_items = (histories + chunk - 1) / chunk;
    DevProblem prob;
    fill_dev_problem(p, histories, seed, chunk, 0, &prob);
    prob.batch_max = batch_limit(histories, chunk, used);
    prob.counters = (uint64_t *)(base + kCountersOff);
    prob.sums = (double *)(base + kSumsOff);
    prob.record = (uint64_t *)d_record;
    prob.trace_hash = nullptr;
    prob.trace_len = nullptr;
    DevProblem *d_prob = (DevProblem *)(base + kProbOff);
    uint64_t *d_items = (uint64_t *)(base + kItemsOff);
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(static_setup_kernel, dim3(1), dim3(256), 0, s, prob, d_prob, d_items, n_items);
    HIP_TRY(hipGetLastError());
    TrackArgs a;
    a.probs = d_prob;
    a.item_start = d_items;
    a.queue_head = d_items + 2;
    a.nprobs = 1;
    a.lds_stride = stride;
    a.refill_min = used.refill_min;
    a.slots = used.slots;
    HIP_TRY(launch_track(v, a, grid, block, lds, s));
    HIP_TRY(launch_finalize(d_prob, 1, s));
    return CLS_OK;
}
