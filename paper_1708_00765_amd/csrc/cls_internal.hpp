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

// Per-problem parameters and output pointers, one record per problem of a
// launch (device memory).
struct alignas(16) DevProblem {
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
    uint64_t chunk;             // histories per work item (batch)
    uint64_t chunk_base;        // chunk index of this launch's first work item of the problem
    uint64_t trace_n;           // histories with a recorded trace
    uint64_t max_steps;         // flight cap per history
    int32_t nbins;
    float dxf;                  // FP32 copy of dx
    uint64_t *counters;         // C_COUNT u64
    double *sums;               // [0] score sum, [1] score square sum, [2..2+K) S_k, [2+K..2+2K) Q_k
    uint64_t *record;           // finalize output, record_words(K) words
    uint64_t *trace_hash;
    uint32_t *trace_len;
    // Served requests: the request's total chunk count, and the device address
    // of its pinned host record. When non-zero, the wave that flushes the last
    // chunk writes the finalized record there (no finalize kernel or copy).
    uint64_t final_chunks;
    uint64_t *host_record;
};

// Everything one tracking launch needs.
struct TrackArgs {
    const DevProblem *probs;
    const uint64_t *item_start;  // nprobs + 1 prefix sums of work items
    uint64_t *queue_head;        // work-item counter (zeroed before the launch)
    int nprobs;
    int lds_stride;              // doubles per tally buffer (>= max nbins + 1, even)
    int refill_min;              // idle lanes a wave waits for before handing out histories
    int slots;                   // LDS tally buffers per wave: 2, or 1 (fine meshes, large chunks)
    unsigned long long *exit_count = nullptr;   // served rounds: waves that have left (zeroed before)
};

// LDS per wave beyond its one or two tally buffers: score sums of two slots
// (4 doubles) and kSlotCounters 32-bit counters per slot (8 doubles).
constexpr int kSlotCounters = 8;
// ... then the per-material flight parameters of the problem each slot holds:
// 2 slots x 2 materials x 4 values, room for FP64 values.
constexpr int kMatTableDoubles = 16;
constexpr int kWaveExtraDoubles = 4 + kSlotCounters + kMatTableDoubles;

struct LaunchShape {
    int waves_per_block;
    int blocks_per_cu;
    int max_chunk;
    int refill_min;
    int slots = 2;               // chosen by the launch sizing, not by the caller
};

// Kernel variants: geometry x estimator x source x precision x trace.
struct Variant {
    int geom, est, src;
    bool fp32, trace;
};

// Host launchers implemented next to the kernels. They enqueue on `stream`
// and return the HIP status of the launch.
hipError_t launch_reset(const DevProblem *d_probs, int nprobs, uint64_t *queue_head,
                        hipStream_t stream);
hipError_t launch_track(const Variant &v, const TrackArgs &args, int grid, int block,
                        size_t lds_bytes, hipStream_t stream);
hipError_t launch_finalize(const DevProblem *d_probs, int nprobs, hipStream_t stream);
// Resident workgroups per compute unit of the tracking kernel for a block of
// `block` threads with `lds_bytes` of dynamic LDS.
hipError_t track_occupancy(const Variant &v, int block, size_t lds_bytes, int *blocks_per_cu);

}  // namespace cls
