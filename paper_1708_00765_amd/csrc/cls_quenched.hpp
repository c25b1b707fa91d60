// Private definitions shared by the quenched-disorder kernels and their host
// entry points (d = 1, Section 3 of Larmier et al., arXiv 1708.00765). Not
// part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cls {

// Counters of a quenched run (u64, device): realizations done, histories,
// outcomes, events, layers.
enum QCounter : int {
    Q_REALIZATIONS = 0, Q_HISTORIES, Q_TRANSMITTED, Q_REFLECTED, Q_ABSORBED, Q_CAPPED,
    Q_FLIGHTS, Q_COLLISIONS, Q_SCATTERS, Q_CROSSINGS, Q_LAYERS, Q_COUNT
};

// Per-realization observables (history means) whose ensemble mean and spread
// are accumulated: T, R, A, total flux (track length per history), leakage
// (T + R)/2.
enum QObs : int { QO_T = 0, QO_R, QO_A, QO_TOTAL, QO_LEAK, QO_COUNT };

// Finalize record: Q_COUNT counters (u64 words), then QO_COUNT means,
// QO_COUNT standard errors of the means and QO_COUNT spreads (doubles), then
// the binned flux mean[K] and its standard error[K].
constexpr int kQRecordHeader = Q_COUNT + 3 * QO_COUNT;
inline size_t q_record_words(int nbins) { return (size_t)kQRecordHeader + 2 * (size_t)nbins; }

// Device record of one quenched run.
struct alignas(16) DevQuenched {
    double L, inv_dx, dx;
    double sigma[2], c[2];
    double rho;                 // Poisson point density 1/Lambda_0 + 1/Lambda_1
    double p0;                  // probability of material 0 per cell
    uint64_t seed;
    uint64_t realizations;      // M
    uint64_t histories;         // N per realization
    uint64_t max_steps;         // flight cap per history
    int32_t nbins;
    int32_t layer_cap;          // layers a wave's LDS holds
    int32_t lds_stride;         // doubles per wave of LDS (layer bounds, then the tally buffer)
    int32_t pad0;
    uint64_t *counters;         // Q_COUNT
    double *sums;               // [0, QO_COUNT) sums of per-realization observables,
                                // [QO_COUNT, 2 QO_COUNT) sums of squares, then S_b[K], Q_b[K]
    uint64_t *queue;            // realization counter (zeroed before the launch)
    uint32_t *overflow;         // set when a realization has more than layer_cap layers
    uint64_t *record;           // finalize output, q_record_words(K) words
};

struct QVariant {
    bool slab;                  // slab angular model (else rod)
    int src;                    // 0 face source, 1 interior source
    int est;                    // 0 collision estimator, 1 track length
};

hipError_t launch_quenched(const QVariant &v, const DevQuenched *d_rec, int grid, int block, size_t lds,
                           hipStream_t stream);
hipError_t launch_quenched_reset(const DevQuenched *d_rec, int nbins, hipStream_t stream);
hipError_t launch_quenched_finalize(const DevQuenched *d_rec, hipStream_t stream);
hipError_t quenched_occupancy(const QVariant &v, int block, size_t lds, int *blocks_per_cu);

}  // namespace cls
