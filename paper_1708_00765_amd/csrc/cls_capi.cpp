// Host runtime and C ABI of the Chord Length Sampling library.
//
// A problem object holds the parameters of one CLS problem (Section 2 of
// Larmier et al., arXiv 1708.00765: box of side L leaking on the x-faces and
// mirroring on the lateral ones, two Markov-mixed materials with Sigma_i, c_i,
// Lambda_i) and the device memory of its tallies. A run enqueues four steps
// on the problem's stream: reset of the tallies, the persistent tracking
// kernel, the finalize kernel (means and errors) and one device-to-host copy
// into pinned memory owned by the problem.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "cls_runtime.hpp"

using namespace cls;
using namespace cls::rt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

namespace cls {
namespace rt {

cls_status fail(cls_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

cls_status hip_fail(hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    // the failure is reported here; clear the thread's last HIP error so that
    // the next launch check (hipGetLastError) does not report it again
    (void)hipGetLastError();
    return fail(CLS_ERR_DEVICE, m);
}

}  // namespace rt
}  // namespace cls

// ---------------------------------------------------------------------------
// device and launch shape
// ---------------------------------------------------------------------------
namespace {
std::mutex g_mu;
std::vector<DeviceInfo> g_devices;
LaunchShape g_shape = {0, 0, 0, 0};

constexpr int kDefaultWavesPerBlock = 0;   // 0: chosen per kernel (most resident waves)
constexpr int kDefaultBlocksPerCu = 0;     // 0: as many as fit (occupancy query)
constexpr int kDefaultMaxChunk = 16384;
constexpr size_t kLdsLimit = 65536;
constexpr int kDefaultRefillMin = 4;
}  // namespace

namespace cls {
namespace rt {

cls_status device_info(DeviceInfo *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(CLS_ERR_NO_DEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &d : g_devices)
        if (d.id == dev) { *out = d; return CLS_OK; }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CLS_ERR_NO_DEVICE, std::string("library built for gfx950, device is ") + prop.gcnArchName);
    DeviceInfo d;
    d.id = dev;
    d.cus = prop.multiProcessorCount;
    d.lds_per_block = prop.sharedMemPerBlock;
    g_devices.push_back(d);
    *out = d;
    return CLS_OK;
}

LaunchShape current_shape()
{
    std::lock_guard<std::mutex> lk(g_mu);
    LaunchShape s = g_shape;
    if (s.waves_per_block <= 0) s.waves_per_block = kDefaultWavesPerBlock;   // may stay 0
    if (s.blocks_per_cu <= 0) s.blocks_per_cu = kDefaultBlocksPerCu;   // may stay 0
    if (s.max_chunk <= 0) s.max_chunk = kDefaultMaxChunk;
    if (s.refill_min <= 0) s.refill_min = kDefaultRefillMin;
    return s;
}

size_t align256(size_t v) { return (v + 255u) & ~(size_t)255u; }

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

size_t workspace_bytes(int nbins, uint64_t trace_n)
{
    size_t b = 0;
    b += align256(sizeof(DevProblem));
    b += align256(4 * sizeof(uint64_t));
    b += align256(C_COUNT * sizeof(uint64_t));
    b += align256(sums_words(nbins) * sizeof(double));
    b += align256(record_words(nbins) * sizeof(uint64_t));
    b += align256((size_t)trace_n * sizeof(uint64_t));
    b += align256((size_t)trace_n * sizeof(uint32_t));
    return b;
}

static void carve(cls_problem *p, size_t trace_n)
{
    char *q = p->dev;
    p->d_prob = (DevProblem *)q; q += align256(sizeof(DevProblem));
    p->d_items = (uint64_t *)q; q += align256(4 * sizeof(uint64_t));
    p->d_counters = (uint64_t *)q; q += align256(C_COUNT * sizeof(uint64_t));
    p->d_sums = (double *)q; q += align256(sums_words(p->nbins) * sizeof(double));
    p->d_record = (uint64_t *)q; q += align256(record_words(p->nbins) * sizeof(uint64_t));
    p->d_trace_hash = trace_n ? (uint64_t *)q : nullptr; q += align256(trace_n * sizeof(uint64_t));
    p->d_trace_len = trace_n ? (uint32_t *)q : nullptr;
    p->trace_cap = trace_n;
}

static void release_device(cls_problem *p)
{
    if (p->ev_done) (void)hipEventSynchronize(p->ev_done);
    if (p->dev && p->dev_owned) (void)hipFree(p->dev);
    p->dev = nullptr;
    p->dev_bytes = 0;
    p->dev_owned = false;
}

// Make sure the problem has host mirrors, events and a workspace that holds
// `trace_n` trace entries.
cls_status ensure_device(cls_problem *p, uint64_t trace_n)
{
    DeviceInfo di;
    const cls_status st = device_info(&di);
    if (st != CLS_OK) return st;
    return ensure_device(p, trace_n, di);
}

cls_status ensure_device(cls_problem *p, uint64_t trace_n, const DeviceInfo &di)
{
    if (p->device >= 0 && p->device != di.id)
        return fail(CLS_ERR_STATE, "problem was first run on another device");
    p->device = di.id;
    // each piece on its own, so that a call after a failed one completes the set
    if (!p->h_prob) HIP_TRY(hipHostMalloc((void **)&p->h_prob, sizeof(DevProblem), hipHostMallocDefault));
    if (!p->h_items) HIP_TRY(hipHostMalloc((void **)&p->h_items, 4 * sizeof(uint64_t), hipHostMallocDefault));
    if (!p->h_record)
        HIP_TRY(hipHostMalloc((void **)&p->h_record, record_words(p->nbins) * sizeof(uint64_t),
                              hipHostMallocDefault));
    if (!p->ev_k0) HIP_TRY(hipEventCreate(&p->ev_k0));
    if (!p->ev_k1) HIP_TRY(hipEventCreate(&p->ev_k1));
    if (!p->ev_done) HIP_TRY(hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming));
    const size_t need = workspace_bytes(p->nbins, trace_n);
    if (p->dev && p->dev_bytes >= need) {
        if (trace_n > p->trace_cap || p->trace_cap == 0) carve(p, trace_n);
        return CLS_OK;
    }
    if (p->dev && !p->dev_owned)
        return fail(CLS_ERR_INVALID_ARG, "bound device memory is smaller than cls_footprint()");
    release_device(p);
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, need);
    if (e != hipSuccess) return fail(CLS_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    p->dev = (char *)mem;
    p->dev_bytes = need;
    p->dev_owned = true;
    carve(p, trace_n);
    return CLS_OK;
}

// Integer form of the test U < q for the uniforms U = (k + 1/2) 2^-23 of the
// random-number stream: U < q exactly when k < ceil(q 2^23 - 1/2) (both sides
// are exact in FP64), i.e. when the bit pattern 0x3F800000 | k that the
// kernels hold is below 0x3F800000 + ceil(q 2^23 - 1/2).
uint32_t unit_threshold(double q)
{
    double t = std::ceil(std::ldexp(q, 23) - 0.5);
    t = std::min(std::max(t, 0.0), 8388608.0);
    return 0x3F800000u + (uint32_t)t;
}

uint32_t batch_limit(uint64_t histories, uint64_t chunk, const LaunchShape &s)
{
    return (uint32_t)(s.chunk_batches == 1 ? chunk : sched::batch_histories(histories, chunk));
}

void fill_dev_problem(const cls_problem *p, uint64_t histories, uint64_t seed, uint64_t chunk,
                             uint64_t trace_n, DevProblem *out)
{
    std::memset(out, 0, sizeof *out);
    out->L = p->L;
    out->inv_dx = (double)p->nbins / p->L;
    out->dx = p->L / (double)p->nbins;
    for (int i = 0; i < 2; ++i) {
        out->sigma[i] = p->sigma[i];
        out->c[i] = p->c[i];
        out->lam[i] = p->lam[i];
    }
    out->p0 = p->lam[0] / (p->lam[0] + p->lam[1]);
    out->Lf = (float)p->L;
    out->dxf = (float)out->dx;
    out->p0f = (float)out->p0;
    for (int i = 0; i < 2; ++i) {
        out->isig[i] = 1.0 / p->sigma[i];
        out->isigf[i] = (float)out->isig[i];
        out->cf[i] = (float)p->c[i];
        out->lamf[i] = (float)p->lam[i];
        out->dsigf[i] = (float)(-0.69314718055994530942 / p->sigma[i]);
        out->dlamf[i] = (float)(-0.69314718055994530942 * p->lam[i]);
        out->cthr[i] = unit_threshold(p->c[i]);
    }
    out->p0thr = unit_threshold(out->p0);
    out->trace_bins = (p->flags & CLS_F_TRACE_NO_BINS) ? 0 : 1;
    out->seed = seed;
    out->histories = histories;
    out->chunk = chunk;
    out->chunk_base = 0;
    out->trace_n = trace_n;
    out->max_steps = sched::flight_cap(chunk);
    out->nbins = p->nbins;
    out->kind = problem_kind(p->geom, p->est, p->src);
    out->batch_max = (uint32_t)chunk;
    out->counters = p->d_counters;
    out->sums = p->d_sums;
    out->record = p->d_record;
    out->trace_hash = p->d_trace_hash;
    out->trace_len = p->d_trace_len;
}

uint64_t trace_count(const cls_problem *p, uint64_t histories)
{
    return (p->flags & CLS_F_TRACE) ? std::min(histories, p->trace_request) : 0;
}

bool same_variant(const Variant &a, const Variant &b)
{
    return a.geom == b.geom && a.est == b.est && a.src == b.src && a.fp32 == b.fp32 && a.trace == b.trace &&
           a.served == b.served;
}

cls_status check_problem_set(cls_problem *const *problems, int n, const uint64_t *histories,
                             uint64_t *total, const char *what)
{
    if (!problems || n < 1) return fail(CLS_ERR_INVALID_ARG, "empty or NULL problem list");
    for (int i = 0; i < n; ++i) {
        if (!problems[i]) return fail(CLS_ERR_INVALID_ARG, "NULL problem in the list");
        if (!same_variant(variant_of(problems[0]), variant_of(problems[i])))
            return fail(CLS_ERR_INVALID_ARG, std::string(what) +
                                                 " problems must share geometry, source, estimator and precision");
    }
    std::vector<cls_problem *> sorted(problems, problems + n);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(CLS_ERR_INVALID_ARG, "a problem appears twice in the list");
    if (histories) {
        uint64_t sum = 0;
        for (int i = 0; i < n; ++i) {
            if (histories[i] == 0) return fail(CLS_ERR_INVALID_ARG, "histories must be >= 1");
            if (histories[i] > UINT64_MAX - sum) return fail(CLS_ERR_INVALID_ARG, "total histories exceed 2^64 - 1");
            sum += histories[i];
        }
        if (total) *total = sum;
    }
    return CLS_OK;
}

Variant variant_of(const cls_problem *p)
{
    Variant v;
    v.geom = p->geom;
    v.est = p->est;
    v.src = p->src;
    v.fp32 = (p->flags & CLS_F_FP32) != 0;
    v.trace = (p->flags & CLS_F_TRACE) != 0;
    return v;
}

// Occupancy of a tracking-kernel variant for a workgroup size and LDS size on
// the current device, cached: the answer never changes within a process, and
// the query is a runtime call that every launch-shape choice makes up to
// eight times.
static hipError_t occupancy_cached(const Variant &v, int device, int block, size_t lds, int *bpc)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, bool, bool, bool, int, size_t>, int> cache;
    const auto key = std::make_tuple(device, v.geom, v.est, v.src, v.fp32, v.trace, v.served, block, lds);
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = cache.find(key);
        if (it != cache.end()) {
            *bpc = it->second;
            return hipSuccess;
        }
    }
    const hipError_t e = track_occupancy(v, block, lds, bpc);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = *bpc;
    return hipSuccess;
}

// Launch shape. Each wave needs one or two LDS tally buffers (two let a
// wave start its next chunk while the last histories of the previous one
// finish; one halves the LDS, at the cost of waiting for those histories,
// which only pays when nearly all of the launch's histories sit in chunks of
// several thousand histories);
// a workgroup uses at most kLdsLimit. Unless the caller fixed them, the
// workgroup size (1, 2, 4 or 8 waves) and the buffer count are the ones
// that keep the most waves resident per compute unit (occupancy query; ties
// go to two buffers, and to 4, then 8, 2 and 1 waves: 4-wave workgroups
// measured fastest at equal residency) and the persistent grid holds as
// many workgroups as the compute units keep resident at once.
cls_status shape_for(const Variant &v, int max_bins, const DeviceInfo &di, int *grid, int *block,
                     size_t *lds, int *lds_stride, LaunchShape *used, const SmallShareFn &small_share)
{
    LaunchShape s = current_shape();
    int kp = max_bins + 1;
    kp += kp & 1;
    auto wave_bytes = [&](int slots) { return ((size_t)slots * (size_t)kp + kWaveExtraDoubles) * sizeof(double); };
    // workgroups take at most kLdsLimit, except for a mesh whose one buffer
    // needs more than 32 KB (beyond ~4050 bins): then up to the device's limit
    // per workgroup (gfx950: the CU's 160 KB), where two-wave workgroups fit
    // (the occupancy query reports no room for one-wave workgroups of 48 KB
    // or more of these kernels, measured on MI355X)
    size_t limit = std::min(kLdsLimit, di.lds_per_block ? di.lds_per_block : kLdsLimit);
    if (wave_bytes(1) > 32768 && di.lds_per_block > limit) limit = di.lds_per_block;
    if (wave_bytes(1) > limit) return fail(CLS_ERR_INVALID_ARG, "flux mesh too large for LDS");
    int best_waves = 0, best_bpc = 0, best_slots = 2;
    const int candidates[4] = {4, 8, 2, 1};
    for (int slots = 2; slots >= 1; --slots) {
        // a requested buffer count is the only one tried
        if (s.slots_request != 0 && slots != s.slots_request) continue;
        const size_t pw = wave_bytes(slots);
        for (int c : candidates) {
            if (s.waves_per_block > 0 && c != s.waves_per_block) continue;
            if (pw * (size_t)c > limit) continue;
            int bpc = s.blocks_per_cu;
            if (bpc <= 0) {
                const hipError_t e = occupancy_cached(v, di.id, c * 64, pw * (size_t)c, &bpc);
                if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
            }
            if (slots == 1 && s.slots_request == 0) {
                const uint64_t waves_total = (uint64_t)di.cus * (uint64_t)std::max(bpc, 1) * (uint64_t)c;
                if (!small_share || small_share(waves_total, (uint64_t)s.max_chunk) > kSingleSlotMaxSmallShare)
                    continue;
            }
            if (bpc * c > best_bpc * best_waves) { best_waves = c; best_bpc = bpc; best_slots = slots; }
        }
    }
    const size_t per_wave = wave_bytes(best_waves ? best_slots : 1);
    if (best_waves == 0) best_slots = 1;
    if (best_waves == 0) {   // a fixed workgroup size that does not fit: shrink it
        if (s.waves_per_block <= 0) return fail(CLS_ERR_INVALID_ARG, "no workgroup shape fits this flux mesh");
        best_waves = s.waves_per_block;
        while (best_waves > 1 && per_wave * (size_t)best_waves > limit) --best_waves;
        best_bpc = s.blocks_per_cu;
        if (best_bpc <= 0) {
            const hipError_t e = occupancy_cached(v, di.id, best_waves * 64, per_wave * (size_t)best_waves, &best_bpc);
            if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        }
    }
    best_bpc = std::max(best_bpc, 1);
    *block = best_waves * 64;
    *lds = per_wave * (size_t)best_waves;
    *lds_stride = kp;
    *grid = di.cus * best_bpc;
    s.waves_per_block = best_waves;
    s.blocks_per_cu = best_bpc;
    s.slots = best_slots;
    *used = s;
    return CLS_OK;
}

}  // namespace rt
}  // namespace cls

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *cls_version(void) { return "cls-mi355x 0.1"; }

const char *cls_status_string(cls_status s)
{
    switch (s) {
    case CLS_OK: return "CLS_OK";
    case CLS_ERR_INVALID_ARG: return "CLS_ERR_INVALID_ARG";
    case CLS_ERR_OUT_OF_MEMORY: return "CLS_ERR_OUT_OF_MEMORY";
    case CLS_ERR_DEVICE: return "CLS_ERR_DEVICE";
    case CLS_ERR_NOT_READY: return "CLS_ERR_NOT_READY";
    case CLS_ERR_EVENT_CAP: return "CLS_ERR_EVENT_CAP";
    case CLS_ERR_STATE: return "CLS_ERR_STATE";
    case CLS_ERR_NO_DEVICE: return "CLS_ERR_NO_DEVICE";
    case CLS_ERR_CAPACITY: return "CLS_ERR_CAPACITY";
    }
    return "CLS_ERR_UNKNOWN";
}

const char *cls_last_error(void) { return g_last_error.c_str(); }

cls_status cls_create_problem(int d, double L, const double sigma_t[2], const double c[2],
                              const double lambda[2], int source, uint32_t boundaries, int nbins,
                              uint32_t flags, cls_problem **out)
{
    if (!out) return fail(CLS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!sigma_t || !c || !lambda) return fail(CLS_ERR_INVALID_ARG, "parameter array is NULL");
    if (d < 1 || d > 3) return fail(CLS_ERR_INVALID_ARG, "d must be 1, 2 or 3");
    if (!finite_pos(L)) return fail(CLS_ERR_INVALID_ARG, "L must be finite and > 0");
    for (int i = 0; i < 2; ++i) {
        if (!finite_pos(sigma_t[i])) return fail(CLS_ERR_INVALID_ARG, "sigma_t must be finite and > 0");
        if (!(c[i] >= 0.0 && c[i] <= 1.0)) return fail(CLS_ERR_INVALID_ARG, "c must lie in [0, 1]");
        if (!finite_pos(lambda[i])) return fail(CLS_ERR_INVALID_ARG, "lambda must be finite and > 0");
    }
    if (source != CLS_SRC_FACE_X0 && source != CLS_SRC_VOLUME)
        return fail(CLS_ERR_INVALID_ARG, "source must be CLS_SRC_FACE_X0 or CLS_SRC_VOLUME");
    if (nbins < 1 || nbins > CLS_MAX_BINS) return fail(CLS_ERR_INVALID_ARG, "nbins out of [1, CLS_MAX_BINS]");
    const uint32_t known = CLS_F_D1_SLAB | CLS_F_COLLISION_FLUX | CLS_F_FP32 | CLS_F_TRACE | CLS_F_TRACE_NO_BINS;
    if (flags & ~known) return fail(CLS_ERR_INVALID_ARG, "unknown flag bits");
    if ((flags & CLS_F_D1_SLAB) && d != 1) return fail(CLS_ERR_INVALID_ARG, "CLS_F_D1_SLAB requires d = 1");
    if ((flags & CLS_F_TRACE_NO_BINS) && !(flags & CLS_F_TRACE))
        return fail(CLS_ERR_INVALID_ARG, "CLS_F_TRACE_NO_BINS requires CLS_F_TRACE");
    uint32_t paper_bc = 0;
    if (d >= 2) paper_bc |= CLS_BC_FACE(2) | CLS_BC_FACE(3);
    if (d >= 3) paper_bc |= CLS_BC_FACE(4) | CLS_BC_FACE(5);
    if (boundaries != CLS_BC_DEFAULT && boundaries != paper_bc)
        return fail(CLS_ERR_INVALID_ARG,
                    "boundaries must leak on both x-faces and reflect on every lateral face");
    cls_problem *p = new (std::nothrow) cls_problem();
    if (!p) return fail(CLS_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->d = d;
    p->geom = d == 1 ? ((flags & CLS_F_D1_SLAB) ? GEOM_SLAB : GEOM_ROD) : (d == 2 ? GEOM_EXT2D : GEOM_CUBE3D);
    p->src = source == CLS_SRC_VOLUME ? SRC_VOLUME : SRC_FACE;
    p->est = (flags & CLS_F_COLLISION_FLUX) ? EST_COLLISION : EST_TRACK;
    p->nbins = nbins;
    p->flags = flags;
    p->L = L;
    for (int i = 0; i < 2; ++i) {
        p->sigma[i] = sigma_t[i];
        p->c[i] = c[i];
        p->lam[i] = lambda[i];
    }
    *out = p;
    return CLS_OK;
}

void cls_destroy_problem(cls_problem *p)
{
    if (!p) return;
    release_device(p);
    quenched_release(p);
    if (p->h_prob) (void)hipHostFree(p->h_prob);
    if (p->h_items) (void)hipHostFree(p->h_items);
    if (p->h_record) (void)hipHostFree(p->h_record);
    if (p->ev_k0) (void)hipEventDestroy(p->ev_k0);
    if (p->ev_k1) (void)hipEventDestroy(p->ev_k1);
    if (p->ev_done) (void)hipEventDestroy(p->ev_done);
    delete p;
}

cls_status cls_set_stream(cls_problem *p, void *hip_stream)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    p->stream = (hipStream_t)hip_stream;
    return CLS_OK;
}

cls_status cls_footprint(const cls_problem *p, uint64_t histories, size_t *bytes)
{
    if (!p || !bytes) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    uint64_t tn = (p->flags & CLS_F_TRACE) ? std::min(histories, p->trace_request) : 0;
    *bytes = workspace_bytes(p->nbins, tn);
    return CLS_OK;
}

cls_status cls_bind_device_memory(cls_problem *p, void *dev_ptr, size_t bytes)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    if (dev_ptr && ((uintptr_t)dev_ptr & 255u)) return fail(CLS_ERR_INVALID_ARG, "device memory must be 256-byte aligned");
    if (dev_ptr && bytes < workspace_bytes(p->nbins, 0))
        return fail(CLS_ERR_INVALID_ARG, "device memory is smaller than cls_footprint()");
    release_device(p);
    if (dev_ptr) {
        p->dev = (char *)dev_ptr;
        p->dev_bytes = bytes;
        p->dev_owned = false;
        size_t fixed = workspace_bytes(p->nbins, 0);
        size_t tn = 0;
        if (p->flags & CLS_F_TRACE) {
            tn = (bytes - fixed) / (sizeof(uint64_t) + sizeof(uint32_t));
            while (tn && workspace_bytes(p->nbins, tn) > bytes) --tn;
        }
        carve(p, tn);
    }
    p->has_run = false;
    return CLS_OK;
}

cls_status cls_set_trace_histories(cls_problem *p, uint64_t n)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    if (!(p->flags & CLS_F_TRACE)) return fail(CLS_ERR_INVALID_ARG, "problem was created without CLS_F_TRACE");
    p->trace_request = n;
    return CLS_OK;
}

cls_status cls_set_launch_config(const cls_launch_config *cfg)
{
    if (!cfg) return fail(CLS_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->waves_per_block < 0 || cfg->waves_per_block > 8 || cfg->blocks_per_cu < 0 ||
        cfg->blocks_per_cu > 32 || cfg->max_chunk < 0)
        return fail(CLS_ERR_INVALID_ARG, "launch config out of range");
    if (cfg->max_chunk > 0 && cfg->max_chunk < 64) return fail(CLS_ERR_INVALID_ARG, "max_chunk must be >= 64");
    if (cfg->refill_min < 0 || cfg->refill_min > 64) return fail(CLS_ERR_INVALID_ARG, "refill_min must lie in [0, 64]");
    if (cfg->waves_per_block != 0 && cfg->waves_per_block != 1 && cfg->waves_per_block != 2 &&
        cfg->waves_per_block != 4 && cfg->waves_per_block != 8)
        return fail(CLS_ERR_INVALID_ARG, "waves_per_block must be 0, 1, 2, 4 or 8");
    if (cfg->slots < 0 || cfg->slots > 2) return fail(CLS_ERR_INVALID_ARG, "slots must be 0, 1 or 2");
    if (cfg->chunk_batches < 0 || cfg->chunk_batches > 1)
        return fail(CLS_ERR_INVALID_ARG, "chunk_batches must be 0 or 1");
    std::lock_guard<std::mutex> lk(g_mu);
    g_shape.waves_per_block = cfg->waves_per_block;
    g_shape.blocks_per_cu = cfg->blocks_per_cu;
    g_shape.max_chunk = cfg->max_chunk;
    g_shape.refill_min = cfg->refill_min;
    g_shape.slots_request = cfg->slots;
    g_shape.chunk_batches = cfg->chunk_batches;
    return CLS_OK;
}

cls_status cls_get_launch_config(cls_launch_config *cfg)
{
    if (!cfg) return fail(CLS_ERR_INVALID_ARG, "cfg is NULL");
    LaunchShape s = current_shape();
    cfg->waves_per_block = s.waves_per_block;
    cfg->blocks_per_cu = s.blocks_per_cu;
    cfg->max_chunk = s.max_chunk;
    cfg->refill_min = s.refill_min;
    cfg->slots = s.slots_request;
    cfg->chunk_batches = s.chunk_batches;
    return CLS_OK;
}

cls_status cls_run_async(cls_problem *p, uint64_t histories, uint64_t seed)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    if (histories == 0) return fail(CLS_ERR_INVALID_ARG, "histories must be >= 1");
    const uint64_t trace_n = trace_count(p, histories);
    cls_status st = ensure_device(p, trace_n);
    if (st != CLS_OK) return st;
    if (trace_n > p->trace_cap) return fail(CLS_ERR_INVALID_ARG, "bound device memory too small for the trace");
    // the previous run must be done before its host mirrors are rewritten
    if (p->has_run && !p->done_synced) HIP_TRY(hipEventSynchronize(p->ev_done));
    DeviceInfo di;
    st = device_info(&di);
    if (st != CLS_OK) return st;
    int grid, block, stride;
    size_t lds;
    LaunchShape used;
    st = shape_for(variant_of(p), p->nbins, di, &grid, &block, &lds, &stride, &used,
                   [histories](uint64_t waves_total, uint64_t max_chunk) {
                       return chunk_size(histories, waves_total, max_chunk) < kSingleSlotMinChunk ? 1.0 : 0.0;
                   });
    if (st != CLS_OK) return st;
    const uint64_t waves_total = (uint64_t)grid * (uint64_t)(block / 64);
    const uint64_t chunk = chunk_size(histories, waves_total, (uint64_t)used.max_chunk);
    const uint64_t n_items = (histories + chunk - 1) / chunk;
    fill_dev_problem(p, histories, seed, chunk, trace_n, p->h_prob);
    p->h_prob->batch_max = batch_limit(histories, chunk, used);
    p->h_items[0] = 0;
    p->h_items[1] = n_items;
    p->h_items[2] = 0;
    p->h_items[3] = 0;
    hipStream_t s = p->stream;
    HIP_TRY(hipMemcpyAsync(p->d_prob, p->h_prob, sizeof(DevProblem), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(p->d_items, p->h_items, 4 * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_reset(p->d_prob, 1, p->d_items + 2, s));
    TrackArgs a;
    a.probs = p->d_prob;
    a.item_start = p->d_items;
    a.queue_head = p->d_items + 2;
    a.nprobs = 1;
    a.lds_stride = stride;
    a.refill_min = used.refill_min;
    a.slots = used.slots;
    HIP_TRY(hipEventRecord(p->ev_k0, s));
    HIP_TRY(launch_track(variant_of(p), a, grid, block, lds, s));
    HIP_TRY(hipEventRecord(p->ev_k1, s));
    HIP_TRY(launch_finalize(p->d_prob, 1, s));
    HIP_TRY(hipMemcpyAsync(p->h_record, p->d_record, record_words(p->nbins) * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(p->ev_done, s));
    p->has_run = true;
    p->done_synced = false;
    p->timed_by_events = true;
    p->histories = histories;
    p->seed = seed;
    p->trace_n = trace_n;
    return CLS_OK;
}

cls_status cls_query(const cls_problem *p)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    if (!p->has_run) return fail(CLS_ERR_STATE, "no run");
    hipError_t e = hipEventQuery(p->ev_done);
    if (e == hipSuccess) return CLS_OK;
    if (e == hipErrorNotReady) return CLS_ERR_NOT_READY;
    return hip_fail(e, "hipEventQuery");
}

cls_status cls_synchronize(cls_problem *p)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    if (!p->has_run) return fail(CLS_ERR_STATE, "no run");
    HIP_TRY(hipEventSynchronize(p->ev_done));
    p->done_synced = true;
    return CLS_OK;
}

cls_status cls_run(cls_problem *p, uint64_t histories, uint64_t seed)
{
    cls_status st = cls_run_async(p, histories, seed);
    if (st != CLS_OK) return st;
    st = cls_synchronize(p);
    if (st != CLS_OK) return st;
    if (p->h_record[C_CAPPED]) return fail(CLS_ERR_EVENT_CAP, "a history reached the flight cap");
    return CLS_OK;
}

cls_status cls_read_tallies(const cls_problem *p, cls_tallies *out, double *flux, double *flux_sigma,
                            int nbins)
{
    if (!p || !out) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_run) return fail(CLS_ERR_STATE, "no completed run");
    if ((flux || flux_sigma) && nbins != p->nbins) return fail(CLS_ERR_INVALID_ARG, "nbins does not match the problem");
    if (!p->done_synced) {
        const hipError_t e = hipEventQuery(p->ev_done);
        if (e == hipErrorNotReady) return fail(CLS_ERR_NOT_READY, "the last run has not completed");
        if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
    }
    const uint64_t *C = p->h_record;
    const double *Rz = (const double *)(p->h_record + C_COUNT);
    std::memset(out, 0, sizeof *out);
    out->histories = C[C_HISTORIES];
    out->transmitted = C[C_TRANSMITTED];
    out->reflected = C[C_REFLECTED];
    out->absorbed = C[C_ABSORBED];
    out->capped = C[C_CAPPED];
    out->flights = C[C_FLIGHTS];
    out->collisions = C[C_COLLISIONS];
    out->scatters = C[C_SCATTERS];
    out->interface_crossings = C[C_INTERFACES];
    out->lateral_reflections = C[C_LATERAL];
    out->batches = C[C_BATCHES];
    out->T = Rz[R_T];
    out->R = Rz[R_R];
    out->A = Rz[R_A];
    out->sigma_T = Rz[R_SIGMA_T];
    out->sigma_R = Rz[R_SIGMA_R];
    out->sigma_A = Rz[R_SIGMA_A];
    out->total_flux = Rz[R_TOTAL];
    out->sigma_total_flux = Rz[R_SIGMA_TOTAL];
    float ms = p->track_ms;
    if (p->timed_by_events && hipEventElapsedTime(&ms, p->ev_k0, p->ev_k1) != hipSuccess) ms = 0.0f;
    out->track_ms = ms;
    if (flux) std::memcpy(flux, Rz + R_HEADER, sizeof(double) * (size_t)p->nbins);
    if (flux_sigma) std::memcpy(flux_sigma, Rz + R_HEADER + p->nbins, sizeof(double) * (size_t)p->nbins);
    if (C[C_CAPPED]) return fail(CLS_ERR_EVENT_CAP, "a history reached the flight cap");
    return CLS_OK;
}

cls_status cls_read_trace(const cls_problem *p, uint64_t *hash, uint32_t *flights, uint64_t n)
{
    if (!p) return fail(CLS_ERR_INVALID_ARG, "problem is NULL");
    if (!(p->flags & CLS_F_TRACE)) return fail(CLS_ERR_INVALID_ARG, "problem was created without CLS_F_TRACE");
    if (!p->has_run) return fail(CLS_ERR_STATE, "no completed run");
    if (n > p->trace_n) return fail(CLS_ERR_INVALID_ARG, "n exceeds the recorded trace");
    HIP_TRY(hipEventSynchronize(p->ev_done));
    if (n == 0) return CLS_OK;
    if (hash) HIP_TRY(hipMemcpy(hash, p->d_trace_hash, n * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (flights) HIP_TRY(hipMemcpy(flights, p->d_trace_len, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return CLS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched runs: one persistent launch over the work items of many problems
// ---------------------------------------------------------------------------
namespace {

struct BatchSpace {
    int device = -1;
    char *dev = nullptr;
    size_t dev_bytes = 0;
    char *host = nullptr;
    size_t host_bytes = 0;
    hipEvent_t k0 = nullptr, k1 = nullptr, done = nullptr;
};

std::mutex g_batch_mu;
std::vector<BatchSpace> g_batch;

cls_status batch_space(int device, size_t bytes, BatchSpace **out)
{
    BatchSpace *bs = nullptr;
    for (auto &b : g_batch)
        if (b.device == device) bs = &b;
    if (!bs) {
        g_batch.emplace_back();
        bs = &g_batch.back();
        bs->device = device;
    }
    // each event on its own, so that a call after a failed one completes the set
    if (!bs->k0) HIP_TRY(hipEventCreate(&bs->k0));
    if (!bs->k1) HIP_TRY(hipEventCreate(&bs->k1));
    if (!bs->done) HIP_TRY(hipEventCreateWithFlags(&bs->done, hipEventDisableTiming));
    if (bs->dev_bytes < bytes) {
        if (bs->dev) (void)hipFree(bs->dev);
        if (bs->host) (void)hipHostFree(bs->host);
        bs->dev = nullptr;
        bs->host = nullptr;
        bs->dev_bytes = bs->host_bytes = 0;
        const size_t want = bytes + bytes / 2;
        hipError_t e = hipMalloc((void **)&bs->dev, want);
        if (e != hipSuccess) return fail(CLS_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
        e = hipHostMalloc((void **)&bs->host, want, hipHostMallocDefault);
        if (e != hipSuccess) return fail(CLS_ERR_OUT_OF_MEMORY, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        bs->dev_bytes = bs->host_bytes = want;
    }
    *out = bs;
    return CLS_OK;
}

}  // namespace

namespace cls {
namespace rt {

cls_status run_batch_part(cls_problem *const *problems, const uint64_t *histories, const uint64_t *seeds, int n,
                          double fraction, uint64_t *processed)
{
    if (!histories || !seeds) return fail(CLS_ERR_INVALID_ARG, "NULL histories or seeds");
    uint64_t total_hist = 0;
    cls_status st = check_problem_set(problems, n, histories, &total_hist, "batch");
    if (st != CLS_OK) return st;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    DeviceInfo di;
    st = device_info(&di);
    if (st != CLS_OK) return st;
    int max_bins = 1;
    size_t rec_words = 0;
    for (int i = 0; i < n; ++i) {
        cls_problem *p = problems[i];
        // a part of the run records no trace (not every traced history runs)
        const uint64_t tn = fraction >= 1.0 ? trace_count(p, histories[i]) : 0;
        st = ensure_device(p, tn, di);
        if (st != CLS_OK) return st;
        if (tn > p->trace_cap) return fail(CLS_ERR_INVALID_ARG, "bound device memory too small for the trace");
        if (p->has_run && !p->done_synced) HIP_TRY(hipEventSynchronize(p->ev_done));
        max_bins = std::max(max_bins, p->nbins);
        rec_words += record_words(p->nbins);
    }
    int grid, block, stride;
    size_t lds;
    LaunchShape used;
    st = shape_for(variant_of(problems[0]), max_bins, di, &grid, &block, &lds, &stride, &used,
                   [&](uint64_t waves_total, uint64_t max_chunk) {
                       double small = 0.0;
                       for (int i = 0; i < n; ++i)
                           if (batch_chunk_size(histories[i], total_hist, waves_total, max_chunk) <
                               kSingleSlotMinChunk)
                               small += (double)histories[i];
                       return small / (double)total_hist;
                   });
    if (st != CLS_OK) return st;
    const size_t probs_bytes = align256((size_t)n * sizeof(DevProblem));
    const size_t items_bytes = align256(((size_t)n + 2) * sizeof(uint64_t));
    const size_t rec_bytes = align256(rec_words * sizeof(uint64_t));
    BatchSpace *bs = nullptr;
    st = batch_space(di.id, probs_bytes + items_bytes + rec_bytes, &bs);
    if (st != CLS_OK) return st;
    DevProblem *h_probs = (DevProblem *)bs->host;
    uint64_t *h_items = (uint64_t *)(bs->host + probs_bytes);
    uint64_t *h_rec = (uint64_t *)(bs->host + probs_bytes + items_bytes);
    DevProblem *d_probs = (DevProblem *)bs->dev;
    uint64_t *d_items = (uint64_t *)(bs->dev + probs_bytes);
    uint64_t *d_rec = (uint64_t *)(bs->dev + probs_bytes + items_bytes);
    const uint64_t waves_total = (uint64_t)grid * (uint64_t)(block / 64);
    uint64_t done_hist = 0;
    h_items[0] = 0;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        cls_problem *p = problems[i];
        // a part of the run records no trace (not every traced history runs)
        const uint64_t tn = fraction >= 1.0 ? trace_count(p, histories[i]) : 0;
        const uint64_t chunk = batch_chunk_size(histories[i], total_hist, waves_total, (uint64_t)used.max_chunk);
        fill_dev_problem(p, histories[i], seeds[i], chunk, tn, &h_probs[i]);
        h_probs[i].batch_max = batch_limit(histories[i], chunk, used);
        h_probs[i].record = d_rec + off;
        off += record_words(p->nbins);
        const uint64_t items = (histories[i] + chunk - 1) / chunk;
        // a part of the run: its first chunks, cut exactly as in the whole run
        const uint64_t take = sched::part_items(items, fraction);
        h_items[i + 1] = h_items[i] + take;
        done_hist += std::min(histories[i], take * chunk);
    }
    h_items[n + 1] = 0;   // queue head
    hipStream_t s = problems[0]->stream;
    HIP_TRY(hipMemcpyAsync(bs->dev, bs->host, probs_bytes + items_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_reset(d_probs, n, d_items + n + 1, s));
    TrackArgs a;
    a.probs = d_probs;
    a.item_start = d_items;
    a.queue_head = d_items + n + 1;
    a.nprobs = n;
    a.lds_stride = stride;
    a.refill_min = used.refill_min;
    a.slots = used.slots;
    HIP_TRY(hipEventRecord(bs->k0, s));
    HIP_TRY(launch_track(variant_of(problems[0]), a, grid, block, lds, s));
    HIP_TRY(hipEventRecord(bs->k1, s));
    HIP_TRY(launch_finalize(d_probs, n, s));
    HIP_TRY(hipMemcpyAsync(h_rec, d_rec, rec_words * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    // the call is synchronous: once the batch event has fired every problem's
    // results are complete (done_synced below), so no per-problem event is recorded
    HIP_TRY(hipEventRecord(bs->done, s));
    HIP_TRY(hipEventSynchronize(bs->done));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, bs->k0, bs->k1));
    off = 0;
    bool capped = false;
    for (int i = 0; i < n; ++i) {
        cls_problem *p = problems[i];
        std::memcpy(p->h_record, h_rec + off, record_words(p->nbins) * sizeof(uint64_t));
        off += record_words(p->nbins);
        p->has_run = true;
        p->done_synced = true;
        p->timed_by_events = false;
        p->track_ms = ms;
        p->histories = histories[i];
        p->seed = seeds[i];
        p->trace_n = h_probs[i].trace_n;
        capped = capped || p->h_record[C_CAPPED] != 0;
    }
    if (processed) *processed = done_hist;
    if (capped) return fail(CLS_ERR_EVENT_CAP, "a history reached the flight cap");
    return CLS_OK;
}

}  // namespace rt
}  // namespace cls

extern "C" cls_status cls_run_batch(cls_problem *const *problems, const uint64_t *histories,
                                    const uint64_t *seeds, int n)
{
    return run_batch_part(problems, histories, seeds, n, 1.0, nullptr);
}
