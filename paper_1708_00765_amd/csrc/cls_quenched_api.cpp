// Host entry points of the quenched-disorder reference solutions in d = 1
// (Section 3): workspace, launch shape, run and read-back. The kernels are in
// cls_quenched.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "cls_quenched.hpp"
#include "cls_runtime.hpp"

using namespace cls;
using namespace cls::rt;

namespace {

constexpr int kMaxExpectedLayers = 1024;
constexpr double kMaxExpectedCells = 1e6;
constexpr size_t kQLdsLimit = 65536;
constexpr uint64_t kQMaxSteps = 100000000ull;

// Expected layer count of a realization: the first layer plus the expected
// number of material changes, 2 L / (Lambda_0 + Lambda_1) for the stationary
// two-state medium.
double expected_layers(const cls_problem *p) { return 1.0 + 2.0 * p->L / (p->lam[0] + p->lam[1]); }

// Layers a wave's LDS holds: far above the expected count (the count is a sum
// of independent switches with about that mean).
int layer_capacity(double e)
{
    const double c = e + 8.0 * std::sqrt(e) + 32.0;
    return (int)std::min(2048.0, std::max(64.0, std::ceil(c)));
}

}  // namespace

struct QuenchedState {
    int device = -1;
    int nbins = 0;
    char *dev = nullptr;
    DevQuenched *d_rec = nullptr;
    uint64_t *d_counters = nullptr, *d_queue = nullptr, *d_record = nullptr;
    double *d_sums = nullptr;
    uint32_t *d_overflow = nullptr;
    char *host = nullptr;            // pinned: record in, results and overflow flag out
    DevQuenched *h_rec = nullptr;
    uint64_t *h_record = nullptr;
    uint32_t *h_overflow = nullptr;
    hipEvent_t k0 = nullptr, k1 = nullptr;
    bool has_run = false;
    float ms = 0.0f;
};

namespace cls {
namespace rt {

void quenched_release(cls_problem *p)
{
    QuenchedState *q = p->quenched;
    if (!q) return;
    if (q->dev) (void)hipFree(q->dev);
    if (q->host) (void)hipHostFree(q->host);
    if (q->k0) (void)hipEventDestroy(q->k0);
    if (q->k1) (void)hipEventDestroy(q->k1);
    delete q;
    p->quenched = nullptr;
}

}  // namespace rt
}  // namespace cls

static cls_status quenched_workspace(cls_problem *p, int device)
{
    QuenchedState *q = p->quenched;
    if (q && q->device == device && q->nbins == p->nbins) return CLS_OK;
    quenched_release(p);
    q = new (std::nothrow) QuenchedState();
    if (!q) return fail(CLS_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->quenched = q;
    q->device = device;
    q->nbins = p->nbins;
    const int K = p->nbins;
    const size_t rec = align256(sizeof(DevQuenched));
    const size_t ctr = align256(Q_COUNT * sizeof(uint64_t));
    const size_t sums = align256((2 * QO_COUNT + 2 * (size_t)K) * sizeof(double));
    const size_t misc = align256(2 * sizeof(uint64_t));
    const size_t out = align256(q_record_words(K) * sizeof(uint64_t));
    hipError_t e = hipMalloc((void **)&q->dev, rec + ctr + sums + misc + out);
    if (e == hipSuccess) e = hipHostMalloc((void **)&q->host, rec + out + 256, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreate(&q->k0);
    if (e == hipSuccess) e = hipEventCreate(&q->k1);
    if (e != hipSuccess) {
        quenched_release(p);
        return fail(CLS_ERR_OUT_OF_MEMORY, std::string("quenched workspace: ") + hipGetErrorString(e));
    }
    char *d = q->dev;
    q->d_rec = (DevQuenched *)d;
    q->d_counters = (uint64_t *)(d + rec);
    q->d_sums = (double *)(d + rec + ctr);
    q->d_queue = (uint64_t *)(d + rec + ctr + sums);
    q->d_overflow = (uint32_t *)(q->d_queue + 1);
    q->d_record = (uint64_t *)(d + rec + ctr + sums + misc);
    q->h_rec = (DevQuenched *)q->host;
    q->h_record = (uint64_t *)(q->host + rec);
    q->h_overflow = (uint32_t *)(q->host + rec + out);
    return CLS_OK;
}

extern "C" {

cls_status cls_run_quenched(cls_problem *p, uint64_t realizations, uint64_t histories, uint64_t seed)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    if (p->d != 1) return fail(CLS_ERR_INVALID_ARG, "quenched reference solutions are built for d = 1");
    if (p->flags & (CLS_F_FP32 | CLS_F_TRACE))
        return fail(CLS_ERR_INVALID_ARG, "quenched runs track in FP64 and record no trace");
    if (realizations == 0 || histories == 0)
        return fail(CLS_ERR_INVALID_ARG, "realizations and histories must be >= 1");
    // a lane counts the outcomes of its histories of a realization in 32 bits
    if (histories > 0xFFFFFFFFull) return fail(CLS_ERR_INVALID_ARG, "histories per realization must be < 2^32");
    // global history indices k * histories + h must fit in 64 bits
    if ((double)realizations * (double)histories >= 0x1p62)
        return fail(CLS_ERR_INVALID_ARG, "realizations x histories must be < 2^62");
    const double e = expected_layers(p);
    if (e > kMaxExpectedLayers)
        return fail(CLS_ERR_INVALID_ARG, "medium too fragmented: more than 1024 expected layers per realization");
    // cells before merging: rho L per realization on average
    if ((1.0 / p->lam[0] + 1.0 / p->lam[1]) * p->L > kMaxExpectedCells)
        return fail(CLS_ERR_INVALID_ARG, "more than 10^6 expected Poisson cells per realization");
    DeviceInfo di;
    cls_status st = device_info(&di);
    if (st != CLS_OK) return st;
    st = quenched_workspace(p, di.id);
    if (st != CLS_OK) return st;
    QuenchedState *q = p->quenched;
    const int K = p->nbins;

    // launch shape: 4-wave workgroups unless the per-wave LDS forces fewer
    const int cap = layer_capacity(e);
    int stride = cap + 1 + K + 1;
    stride += stride & 1;
    const size_t per_wave = (size_t)stride * sizeof(double);
    const size_t limit = std::min(kQLdsLimit, di.lds_per_block ? di.lds_per_block : kQLdsLimit);
    int waves = 4;
    while (waves > 1 && per_wave * (size_t)waves > limit) waves /= 2;
    if (per_wave > limit) return fail(CLS_ERR_INVALID_ARG, "flux mesh and layer capacity exceed the LDS");
    const size_t lds = per_wave * (size_t)waves;
    const QVariant v{(p->flags & CLS_F_D1_SLAB) != 0, p->src, p->est};
    int bpc = 0;
    HIP_TRY(quenched_occupancy(v, waves * 64, lds, &bpc));
    bpc = std::max(bpc, 1);
    const uint64_t need = (realizations + (uint64_t)waves - 1) / (uint64_t)waves;
    const int grid = (int)std::min<uint64_t>((uint64_t)di.cus * (uint64_t)bpc, need);

    DevQuenched &r = *q->h_rec;
    std::memset(&r, 0, sizeof r);
    r.L = p->L;
    r.inv_dx = (double)K / p->L;
    r.dx = p->L / (double)K;
    for (int i = 0; i < 2; ++i) {
        r.sigma[i] = p->sigma[i];
        r.c[i] = p->c[i];
    }
    r.rho = 1.0 / p->lam[0] + 1.0 / p->lam[1];
    r.p0 = p->lam[0] / (p->lam[0] + p->lam[1]);
    r.seed = seed;
    r.realizations = realizations;
    r.histories = histories;
    r.max_steps = kQMaxSteps;
    r.nbins = K;
    r.layer_cap = cap;
    r.lds_stride = stride;
    r.counters = q->d_counters;
    r.sums = q->d_sums;
    r.queue = q->d_queue;
    r.overflow = q->d_overflow;
    r.record = q->d_record;

    hipStream_t s = p->stream;
    HIP_TRY(hipMemcpyAsync(q->d_rec, q->h_rec, sizeof(DevQuenched), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_quenched_reset(q->d_rec, K, s));
    HIP_TRY(hipEventRecord(q->k0, s));
    HIP_TRY(launch_quenched(v, q->d_rec, grid, waves * 64, lds, s));
    HIP_TRY(hipEventRecord(q->k1, s));
    HIP_TRY(launch_quenched_finalize(q->d_rec, s));
    HIP_TRY(hipMemcpyAsync(q->h_record, q->d_record, q_record_words(K) * sizeof(uint64_t), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipMemcpyAsync(q->h_overflow, q->d_overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventElapsedTime(&q->ms, q->k0, q->k1));
    q->has_run = true;
    if (*q->h_overflow) return fail(CLS_ERR_CAPACITY, "a realization had more layers than the workspace holds");
    if (q->h_record[Q_CAPPED]) return fail(CLS_ERR_EVENT_CAP, "a history reached the flight cap");
    return CLS_OK;
}

cls_status cls_read_quenched(const cls_problem *p, cls_quenched_tallies *out, double *flux, double *flux_sigma,
                             int nbins)
{
    if (!p || !out) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    const QuenchedState *q = p->quenched;
    if (!q || !q->has_run) return fail(CLS_ERR_STATE, "no quenched run yet");
    if ((flux || flux_sigma) && nbins != p->nbins) return fail(CLS_ERR_INVALID_ARG, "nbins differs from the problem's");
    const uint64_t *c = q->h_record;
    const double *d = (const double *)(c + Q_COUNT);
    out->realizations = c[Q_REALIZATIONS];
    out->histories = c[Q_HISTORIES];
    out->transmitted = c[Q_TRANSMITTED];
    out->reflected = c[Q_REFLECTED];
    out->absorbed = c[Q_ABSORBED];
    out->capped = c[Q_CAPPED];
    out->flights = c[Q_FLIGHTS];
    out->collisions = c[Q_COLLISIONS];
    out->scatters = c[Q_SCATTERS];
    out->crossings = c[Q_CROSSINGS];
    out->layers = c[Q_LAYERS];
    double *means[QO_COUNT] = {&out->T, &out->R, &out->A, &out->total_flux, &out->Lk};
    double *ses[QO_COUNT] = {&out->sigma_T, &out->sigma_R, &out->sigma_A, &out->sigma_total_flux, &out->sigma_Lk};
    double *sps[QO_COUNT] = {&out->spread_T, &out->spread_R, &out->spread_A, &out->spread_total_flux,
                             &out->spread_Lk};
    for (int j = 0; j < QO_COUNT; ++j) {
        *means[j] = d[j];
        *ses[j] = d[QO_COUNT + j];
        *sps[j] = d[2 * QO_COUNT + j];
    }
    out->track_ms = q->ms;
    const double *fl = d + 3 * QO_COUNT;
    if (flux) std::memcpy(flux, fl, sizeof(double) * (size_t)nbins);
    if (flux_sigma) std::memcpy(flux_sigma, fl + nbins, sizeof(double) * (size_t)nbins);
    return CLS_OK;
}

}  // extern "C"
