// Internal types shared by the host runtime and the HIP kernels of the CLS
// library. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cls {

enum Geom : int { GEOM_ROD = 0, GEOM_SLAB = 1, GEOM_EXT2D = 2, GEOM_CUBE3D = 3 };
enum Est : int { EST_COLLISION = 0, EST_TRACK = 1 };
enum Src : int { SRC_FACE = 0, SRC_VOLUME = 1 };

// Served rounds run one kernel per precision for every geometry, estimator
// and source: each problem record carries its kind, and the kernel branches
// on it per problem (a wave-uniform branch).
constexpr int GEOM_ANY = -1;
constexpr int problem_kind(int geom, int est, int src) { return geom | (est << 2) | (src << 3); }

// Trace event codes (same numbering as the documented trace format).
enum Event : int {
    EV_SOURCE = 0, EV_INTERFACE = 1, EV_SCATTER = 2, EV_ABSORB = 3,
    EV_LEAK_XLO = 4, EV_LEAK_XHI = 5,
    EV_REFL_YLO = 6, EV_REFL_YHI = 7, EV_REFL_ZLO = 8, EV_REFL_ZHI = 9,
    EV_CAP = 10, EV_NONE = 15
};

// Integer tallies of one problem (u64 slots in device memory).
enum Counter : int {
    C_HISTORIES = 0, C_TRANSMITTED, C_REFLECTED, C_ABSORBED, C_CAPPED,
    C_FLIGHTS, C_COLLISIONS, C_SCATTERS, C_INTERFACES, C_LATERAL, C_BATCHES,
    C_DONE_CHUNKS,              // chunks flushed (in-kernel finalize of served requests)
    C_QUEUE_HEAD,               // chunks of the problem handed out in a batch launch (its work queue)
    C_COUNT = 16
};

// Result record written by the finalize kernel, in 8-byte words: the
// C_COUNT integer tallies, then R_HEADER doubles, then flux[K] and
// flux_sigma[K] (per source history).
enum Result : int {
    R_T = 0, R_R, R_A, R_SIGMA_T, R_SIGMA_R, R_SIGMA_A, R_TOTAL, R_SIGMA_TOTAL,
    R_HEADER = 8
};

inline size_t record_words(int nbins) { return (size_t)C_COUNT + R_HEADER + 2 * (size_t)nbins; }

// Sums of a problem (doubles): [0] the history score sum, [1] its square sum;
// over the batches b of the flux error (n_b histories, per-bin sums s_b):
// [2, 2 + K) S_k = sum s_b, [2 + K, 2 + 2K) P_k = sum s_b^2,
// [2 + 2K, 2 + 3K) R_k = sum n_b s_b, and [2 + 3K] M = sum n_b^2.
__host__ __device__ constexpr size_t sums_words(int nbins) { return 3 + 3 * (size_t)nbins; }

// Per-problem parameters and output pointers, one record per problem of a
// launch (device memory, or pinned host memory for a served round's table).
// 128-byte aligned and a multiple of 128 bytes, so that no cache line holds
// parts of two records: the host writes a served round's record while the
// kernel reads other records of that table.
struct alignas(128) DevProblem {
    double L, inv_dx, dx;
    double sigma[2], c[2], lam[2];
    double p0;                  // Lambda_0 / (Lambda_0 + Lambda_1)
    double isig[2];             // 1 / Sigma_i
    // FP32 copies for the FP32 tracking kernel
    float Lf, p0f;
    float isigf[2], cf[2], lamf[2];
    // FP32 flight-distance scales: a distance is log2(U) times -ln2 / Sigma_i
    // (collision) or -ln2 Lambda_i (interface)
    float dsigf[2], dlamf[2];
    // Decisions on a uniform U = (k + 1/2) 2^-23 against a probability q are
    // taken on the integer k: U < q exactly when the bit pattern of the float
    // 1 + k 2^-23 is below 0x3F800000 + ceil(q 2^23 - 1/2). Both precisions
    // then take the FP64 decision (scattering with c_i, source material with
    // p_0) bit for bit.
    uint32_t cthr[2];           // scattering, per material
    uint32_t p0thr;             // source material 0
    int32_t trace_bins;         // trace hash includes the bin of each event (else events and materials only)
    uint64_t seed;
    uint64_t histories;
    uint64_t chunk;             // histories per work item
    uint64_t chunk_base;        // chunk index of this launch's first work item of the problem
    uint64_t trace_n;           // histories with a recorded trace
    uint64_t max_steps;         // flight cap per history
    int32_t nbins;
    float dxf;                  // FP32 copy of dx
    int32_t kind;               // problem_kind(geometry, estimator, source)
    // Histories one wave may gather into one batch of the flux error: in a
    // batch launch a wave adds the next chunk of the same problem to the batch
    // it is filling while the sum stays within batch_max (batch_max == chunk:
    // every chunk is a batch of its own, as in served rounds).
    uint32_t batch_max;
    uint64_t *counters;         // C_COUNT u64
    double *sums;               // sums_words(K) doubles
    uint64_t *record;           // finalize output, record_words(K) words
    uint64_t *trace_hash;
    uint32_t *trace_len;
    // Served requests (final_chunks != 0): the request's total chunk count;
    // the wave that flushes its last chunk writes the finalized record into
    // host_record (device address of pinned host memory) when it is set and
    // clears the tallies for the next request of that memory, then stores
    // `tag` into *done_word (pinned) to tell the host the request is complete.
    uint64_t final_chunks;
    uint64_t *host_record;
    uint64_t *done_word;
    uint64_t tag;
};
static_assert(sizeof(DevProblem) % 128 == 0, "problem records span whole cache lines");

// Work queue of a served round, in pinned host memory that the kernel reads
// while it runs. An item is (table entry << 32) | chunk index, or
// kServedLeave. The host writes an entry's record into the round's table
// (pinned too) before the entry's first item, writes items, and then raises
// `published`. A wave takes the next item index (a ticket) with one fetch-add
// on the device-side head and runs the item once `published` covers it; until
// then it keeps stepping the histories it has and looks again, at growing
// intervals (counted in loop passes: a waiting wave does not read the clock,
// whose reads share the scalar memory path with the working waves). Tickets go out in order, so every item before the first
// kServedLeave is run before any wave receives one. To end a round the host
// publishes one kServedLeave per wave after the last item: each wave leaves on
// the first it receives, so every wave leaves and every published item runs.
// A wave that waits longer than wait_passes for its ticket, or receives an item
// it refuses (an entry outside the table), reports it in `error` and leaves; an
// entry of an unknown kind of problem ends its histories at once as capped; the
// host writes only chunks of an entry's own range. A broken round ends in an
// error, never in a wave that cannot finish.
struct ServedFeed {
    uint64_t published;          // items written (host)
    uint64_t seen;               // a recent ticket, reported by the waves (every 32nd)
    uint64_t error;              // kServedErr* of the last failure, 0 if none
    uint64_t error_item;         // the item (or ticket) concerned
    uint64_t pad[4];
};

constexpr uint64_t kServedLeave = ~0ull;
enum ServedError : uint64_t { kServedErrBadItem = 1, kServedErrWait = 2 };

// Device side of a served round: the ticket counter, and the device
// wall-clock ticks its waves were alive and, of those, idle (no history to
// step) while waiting for their ticket to be published.
struct ServedDev {
    uint64_t head;
    unsigned long long alive_ticks, idle_ticks;
    uint64_t pad[5];
};

// Everything one tracking launch needs.
struct TrackArgs {
    const DevProblem *probs;
    const uint64_t *item_start;  // nprobs + 1 prefix sums of work items
    uint64_t *queue_head;        // unused by batch launches (each problem's C_QUEUE_HEAD counts its chunks)
    int nprobs;
    int lds_stride;              // doubles per tally buffer (>= max nbins + 1, even)
    int refill_min;              // idle lanes a wave waits for before handing out histories
    int slots;                   // LDS tally buffers per wave: 2, or 1 (fine meshes, large chunks)
    // served rounds (feed != nullptr): work comes from the feed's queue
    // instead of item_start; probs is the round's table of entries (device
    // address of pinned host memory)
    ServedFeed *feed = nullptr;          // device address of the pinned feed
    const uint64_t *items = nullptr;     // device address of the pinned item array
    ServedDev *served = nullptr;         // zeroed before the launch
    uint64_t wait_passes = 0;            // idle passes (s_sleep 127 each) a wave waits for its ticket at most
};

// LDS per wave beyond its one or two tally buffers: score sums of two slots
// (4 doubles) and kSlotCounters 64-bit counters per slot (16 doubles).
constexpr int kSlotCounters = 8;
// ... then the per-material flight parameters of the problem each slot holds:
// 2 slots x 2 materials x 4 values, room for FP64 values.
constexpr int kMatTableDoubles = 16;
// ... then, in served rounds, the wave's claim state (see the kernel).
constexpr int kServedWaveWords = 8;
constexpr int kWaveExtraDoubles = 4 + 2 * kSlotCounters + kMatTableDoubles + kServedWaveWords;

struct LaunchShape {
    int waves_per_block;
    int blocks_per_cu;
    int max_chunk;
    int refill_min;
    int slots = 2;               // chosen by the launch sizing
    int slots_request = 0;       // the caller's choice (0: automatic, 1 or 2)
    int chunk_batches = 0;       // 1: every chunk is its own error batch (no gathering)
};

// Kernel variants: geometry x estimator x source x precision x trace, and
// whether the launch is a served round (work from a ServedFeed).
struct Variant {
    int geom, est, src;
    bool fp32, trace;
    bool served = false;
};

// Host launchers implemented next to the kernels. They enqueue on `stream`
// and return the HIP status of the launch.
hipError_t launch_reset(const DevProblem *d_probs, int nprobs, uint64_t *queue_head,
                        hipStream_t stream);
hipError_t launch_track(const Variant &v, const TrackArgs &args, int grid, int block,
                        size_t lds_bytes, hipStream_t stream);
hipError_t launch_finalize(const DevProblem *d_probs, int nprobs, hipStream_t stream);
// Served requests: record into P.record, then clear the tallies (one wave per
// problem; `probs` may be pinned host memory).
hipError_t launch_finalize_clear(const DevProblem *probs, int nprobs, hipStream_t stream);
// Resident workgroups per compute unit of the tracking kernel for a block of
// `block` threads with `lds_bytes` of dynamic LDS.
hipError_t track_occupancy(const Variant &v, int block, size_t lds_bytes, int *blocks_per_cu);

}  // namespace cls
