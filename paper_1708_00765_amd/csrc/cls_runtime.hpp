// Private host runtime of the CLS library: the problem object behind the
// opaque C handle and the helpers that the problem, batch, graph, autotuning
// and serving entry points share. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <functional>
#include <string>

#include "cls.h"
#include "cls_internal.hpp"
#include "cls_sched.hpp"

struct QuenchedState;   // quenched-disorder workspace (cls_quenched_api.cpp)

// ---------------------------------------------------------------------------
// problem object
// ---------------------------------------------------------------------------
struct cls_problem {
    // parameters
    int d = 0, geom = 0, src = 0, est = 0, nbins = 0;
    uint32_t flags = 0;
    double L = 0, sigma[2] = {0, 0}, c[2] = {0, 0}, lam[2] = {0, 0};
    uint64_t trace_request = 0;
    // runtime
    hipStream_t stream = nullptr;
    int device = -1;
    char *dev = nullptr;          // workspace base
    size_t dev_bytes = 0;
    bool dev_owned = false;
    size_t trace_cap = 0;         // histories the workspace trace holds
    // workspace sections
    cls::DevProblem *d_prob = nullptr;
    uint64_t *d_items = nullptr;  // [0] = 0, [1] = n_items, [2] = queue head
    uint64_t *d_counters = nullptr;
    double *d_sums = nullptr;
    uint64_t *d_record = nullptr;
    uint64_t *d_trace_hash = nullptr;
    uint32_t *d_trace_len = nullptr;
    // pinned host mirrors
    cls::DevProblem *h_prob = nullptr;
    uint64_t *h_items = nullptr;
    uint64_t *h_record = nullptr;   // counters, then doubles (record_words(K))
    // run state
    hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr, ev_done = nullptr;
    bool has_run = false;
    bool done_synced = false;       // the last run is known complete (a synchronous path waited for it)
    bool timed_by_events = false;   // track_ms comes from ev_k0/ev_k1
    float track_ms = 0.0f;
    uint64_t histories = 0, seed = 0, trace_n = 0;
    // quenched-disorder runs (d = 1), allocated on first use
    QuenchedState *quenched = nullptr;
};


namespace cls {
namespace rt {

cls_status fail(cls_status s, const std::string &msg);
cls_status hip_fail(hipError_t e, const char *what);

#define HIP_TRY(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return ::cls::rt::hip_fail(e_, #call);    \
    } while (0)

struct DeviceInfo {
    int id = -1;
    int cus = 0;
    size_t lds_per_block = 0;
};

cls_status device_info(DeviceInfo *out);
LaunchShape current_shape();
size_t align256(size_t v);
size_t workspace_bytes(int nbins, uint64_t trace_n);
cls_status ensure_device(cls_problem *p, uint64_t trace_n);
// The same with the current device's info already at hand (loops over problems).
cls_status ensure_device(cls_problem *p, uint64_t trace_n, const DeviceInfo &di);
uint64_t trace_count(const cls_problem *p, uint64_t histories);
using sched::batch_chunk_size;
using sched::chunk_size;
using sched::grouped_chunk_size;
using sched::served_chunk_size;
uint32_t unit_threshold(double q);
// The device record of a run of p; every chunk is its own error batch
// (batch_max = chunk) until the caller sets batch_max (batch_limit).
void fill_dev_problem(const cls_problem *p, uint64_t histories, uint64_t seed, uint64_t chunk,
                      uint64_t trace_n, DevProblem *out);
// Histories one error batch of a batch launch of shape s may gather
// (DevProblem::batch_max): sched::batch_histories, or one chunk when
// s.chunk_batches == 1.
uint32_t batch_limit(uint64_t histories, uint64_t chunk, const LaunchShape &s);
Variant variant_of(const cls_problem *p);
bool same_variant(const Variant &a, const Variant &b);
// Arguments of a launch over several problems: no NULL problem, one kernel
// variant, no problem twice; when histories is given, every count >= 1 and
// their sum (stored in *total) below 2^64. `what` names the caller's rule.
cls_status check_problem_set(cls_problem *const *problems, int n, const uint64_t *histories,
                             uint64_t *total, const char *what);
// One LDS tally buffer per wave (instead of two) doubles the waves an LDS-bound
// launch keeps resident, but a wave then waits for the last histories of its
// chunk before it claims the next; that wait pays only for chunks of at least
// kSingleSlotMinChunk histories. small_share(waves_total, max_chunk) returns
// the share of the launch's histories that sit in smaller chunks on a grid of
// waves_total waves; one buffer per wave is considered only when it is at most
// kSingleSlotMaxSmallShare. Empty when the chunks are not known at launch-shape
// time (graph batches): then every wave gets two buffers.
constexpr uint64_t kSingleSlotMinChunk = 2048;
constexpr double kSingleSlotMaxSmallShare = 0.2;
using SmallShareFn = std::function<double(uint64_t waves_total, uint64_t max_chunk)>;
cls_status shape_for(const Variant &v, int max_bins, const DeviceInfo &di, int *grid, int *block,
                     size_t *lds, int *lds_stride, LaunchShape *used,
                     const SmallShareFn &small_share = SmallShareFn());
// cls_run_batch, or a part of it: with fraction < 1 each problem runs only the
// first ceil(fraction x its chunks) chunks (at least one), cut and launched
// exactly as in the whole batch (same launch shape, chunk sizes and batch
// totals); *processed (may be NULL) receives the histories run. The problems'
// results are then those of the part (autotuner calibration).
cls_status run_batch_part(cls_problem *const *problems, const uint64_t *histories, const uint64_t *seeds, int n,
                          double fraction, uint64_t *processed);
void quenched_release(cls_problem *p);

}  // namespace rt
}  // namespace cls
