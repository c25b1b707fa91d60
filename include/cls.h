/*
 * cls.h -- C ABI of the MI355X Chord Length Sampling library (libcls_hip.so).
 *
 * The library runs Algorithm A of Chord Length Sampling (CLS) -- Section 4 of
 * Larmier, Lam, Brantley, Malvagi, Palmer, Zoia, "Monte Carlo Chord Length
 * Sampling for d-dimensional Markov binary mixtures" (arXiv 1708.00765) -- for
 * single-speed, isotropically scattering particles in a binary Markov mixture,
 * on hand-written HIP kernels for gfx950 (AMD Instinct MI355X).
 *
 * Problem (Section 2): a box of side L with leakage on the two faces normal to
 * x and mirror reflection on the lateral faces; materials i = 0, 1 with total
 * cross section Sigma_i, scattering ratio c_i = Sigma_s,i / Sigma_i and mean
 * chord length Lambda_i; volume fractions p_i = Lambda_i / (Lambda_0 + Lambda_1).
 * Observables (Section 2): transmission T = current out of x = L, reflection
 * R = current out of x = 0, absorption A, and the scalar flux integrated over
 * the lateral coordinates and directions on a uniform x-mesh, all per source
 * history, each with a one-sigma statistical error.
 *
 * Conventions for every function below:
 *   - Every entry point returns cls_status (CLS_OK = 0); no C++ exception
 *     crosses the ABI. On failure nothing is modified and cls_last_error()
 *     returns a thread-local message naming the cause.
 *   - Host pointers are owned by the caller and only read or written during
 *     the call. Device pointers passed in stay owned by the caller and must
 *     outlive every run that uses them.
 *   - A problem handle is not thread-safe; distinct handles are independent.
 *   - Results are a function of (problem parameters, histories, seed) only:
 *     history h of a run uses the random stream keyed by (seed, h), whatever
 *     the batch, slot or launch shape. Integer tallies are bitwise
 *     reproducible; FP64 sums are reproducible up to the order of atomic
 *     additions (about 1e-15 relative).
 */
#ifndef CLS_H
#define CLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CLS_OK = 0,
    CLS_ERR_INVALID_ARG = 1,   /* a parameter is out of its documented range   */
    CLS_ERR_OUT_OF_MEMORY = 2, /* host or device allocation failed              */
    CLS_ERR_DEVICE = 3,        /* a HIP runtime call failed                     */
    CLS_ERR_NOT_READY = 4,     /* asynchronous work is still running            */
    CLS_ERR_EVENT_CAP = 5,     /* a history hit the per-history flight cap      */
    CLS_ERR_STATE = 6,         /* call out of order (e.g. read before any run)  */
    CLS_ERR_NO_DEVICE = 7,     /* no usable gfx950 device                       */
    CLS_ERR_CAPACITY = 8       /* a quenched realization exceeded the layer capacity */
} cls_status;

/* Source (Section 2): suite I = normalized incident angular flux on x = 0
 * (rod: entering along +x; slab/2D/3D: cosine-weighted inward direction,
 * Sec. 4.1-4.3); suite II = uniform isotropic interior source. */
enum { CLS_SRC_FACE_X0 = 0, CLS_SRC_VOLUME = 1 };

/* Boundary bits, one per face in the order x-, x+, y-, y+, z-, z+; a set bit
 * means mirror reflection, a clear bit leakage. The paper's box (Section 2)
 * leaks on x- and x+ and reflects on every lateral face that exists: y for
 * d = 2, y and z for d = 3. CLS_BC_DEFAULT selects exactly that; any other
 * value is accepted only if it equals it. */
enum { CLS_BC_DEFAULT = 0xFFFFFFFFu };
#define CLS_BC_FACE(i) (1u << (i))

/* Flags. */
enum {
    CLS_F_D1_SLAB = 1u << 0,        /* d = 1 is the paper's slab (continuous x-cosine,
                                       Sec. 4.1); without it d = 1 is the rod (+-x)   */
    CLS_F_COLLISION_FLUX = 1u << 1, /* collision estimator for the flux mesh; default
                                       is the track-length estimator (Sec. 3.3)       */
    CLS_F_FP32 = 1u << 2,           /* FP32 flight arithmetic, FP64 x-position and
                                       tallies; default is FP64 throughout            */
    CLS_F_TRACE = 1u << 3,          /* record an event hash and the flight count of
                                       the first histories (cls_read_trace)            */
    CLS_F_TRACE_NO_BINS = 1u << 4   /* with CLS_F_TRACE: hash the events and materials
                                       only, not the bin of each event (compares event
                                       sequences across tracking precisions, whose
                                       positions differ by rounding)                  */
};

/* Largest flux mesh. A wave's LDS tally buffer holds K + 1 doubles (plus ~350
 * bytes of per-wave state): meshes beyond ~8140 bins need more than 64 KB per
 * workgroup, which gfx950 allows (160 KB per CU), at 2 resident waves per CU. */
#define CLS_MAX_BINS 8192

typedef struct cls_problem cls_problem;

/* Create a problem (host only; no device work, so it is usable without a GPU).
 *   d          1 (rod, or slab with CLS_F_D1_SLAB), 2 (extruded: square of side L
 *              in x-y, infinite along z, directions in 3D, Sec. 4.2) or 3 (cube).
 *   L          box side, finite and > 0.
 *   sigma_t[2] total cross sections, finite and > 0.
 *   c[2]       scattering ratios in [0, 1].
 *   lambda[2]  mean chord lengths, finite and > 0.
 *   source     CLS_SRC_FACE_X0 or CLS_SRC_VOLUME.
 *   boundaries CLS_BC_DEFAULT or the equal explicit mask (see above).
 *   nbins      flux mesh size in [1, CLS_MAX_BINS]; bin k = [k L/K, (k+1) L/K),
 *              x = L belongs to the last bin.
 *   flags      CLS_F_* bits; CLS_F_TRACE_NO_BINS requires CLS_F_TRACE.
 *   out        receives the handle (library-owned; free with cls_destroy_problem).
 * Errors: CLS_ERR_INVALID_ARG for any value outside these ranges or a NaN/Inf;
 * CLS_ERR_OUT_OF_MEMORY. */
cls_status cls_create_problem(int d, double L, const double sigma_t[2], const double c[2],
                              const double lambda[2], int source, uint32_t boundaries,
                              int nbins, uint32_t flags, cls_problem **out);

/* Release a problem and the device memory the library allocated for it.
 * Waits for its pending work. NULL is a no-op. */
void cls_destroy_problem(cls_problem *p);

/* Launch subsequent runs of p on the given hipStream_t (NULL = the default
 * stream). The stream is borrowed, not owned. */
cls_status cls_set_stream(cls_problem *p, void *hip_stream);

/* Device bytes one run of p needs (tallies, results and its share of the work
 * queue); independent of the number of histories except for the trace buffer,
 * which grows with min(histories, trace_histories). */
cls_status cls_footprint(const cls_problem *p, uint64_t histories, size_t *bytes);

/* Use caller-owned device memory (e.g. a torch tensor) of at least
 * cls_footprint() bytes, 256-byte aligned, instead of library allocations.
 * Pass NULL to return to library-owned memory. */
cls_status cls_bind_device_memory(cls_problem *p, void *dev_ptr, size_t bytes);

/* Number of leading histories whose trace cls_read_trace returns (CLS_F_TRACE
 * problems only; default 0). */
cls_status cls_set_trace_histories(cls_problem *p, uint64_t n);

/* Run `histories` (>= 1) histories with stream key `seed`, replacing the previous
 * tallies. cls_run blocks until the results are on the host side of the
 * library; cls_run_async enqueues reset, tracking, finalize and the result copy
 * on the problem's stream and returns at once (poll with cls_query).
 * Errors: CLS_ERR_INVALID_ARG (histories == 0), CLS_ERR_NO_DEVICE,
 * CLS_ERR_DEVICE, CLS_ERR_OUT_OF_MEMORY, CLS_ERR_EVENT_CAP (reported by
 * cls_run / cls_read_tallies when a history was cut at the flight cap, see
 * cls_read_tallies). */
cls_status cls_run(cls_problem *p, uint64_t histories, uint64_t seed);
cls_status cls_run_async(cls_problem *p, uint64_t histories, uint64_t seed);

/* CLS_OK when the last run of p has completed, CLS_ERR_NOT_READY otherwise. */
cls_status cls_query(const cls_problem *p);

/* Block until the last run of p has completed. */
cls_status cls_synchronize(cls_problem *p);

typedef struct {
    uint64_t histories, transmitted, reflected, absorbed, capped;
    uint64_t flights, collisions, scatters, interface_crossings, lateral_reflections;
    uint64_t batches;            /* batches of the batch-means flux error               */
    double T, R, A;              /* per source history                                 */
    double sigma_T, sigma_R, sigma_A;
    double total_flux;           /* sum_k flux_k * dx: mean flux score per history     */
    double sigma_total_flux;     /* from per-history sums                              */
    double track_ms;             /* duration of the tracking kernel (HIP events)       */
} cls_tallies;

/* Copy the results of the last completed run. flux and flux_sigma (nbins doubles
 * each, may be NULL) receive the bin-averaged scalar flux per history and its
 * batch-means one-sigma error (batches of n_b histories with bin scores s_b:
 * sigma^2 = sum (s_b - n_b m)^2 / (N - sum n_b^2 / N) per history, unbiased for
 * any batch sizes; the error of the mean is sqrt(sigma^2 / N)); nbins must
 * equal the problem's mesh size. The event counts (flights, scatters,
 * crossings) are summed per lane and work chunk in 32 bits before they reach
 * these 64-bit totals, so a
 * history is cut (counted in `capped`, CLS_ERR_EVENT_CAP) after
 * min(10^8, floor((2^32 - 1) / histories per chunk)) flights: 2.6e5 flights
 * with the default max_chunk of 16384, 65535 with chunks of 65536 histories
 * (lower max_chunk with cls_set_launch_config for longer histories).
 * Errors: CLS_ERR_STATE (no completed run), CLS_ERR_NOT_READY, CLS_ERR_INVALID_ARG,
 * CLS_ERR_EVENT_CAP (results are still written). */
cls_status cls_read_tallies(const cls_problem *p, cls_tallies *out, double *flux,
                            double *flux_sigma, int nbins);

/* Copy the trace of histories 0 .. n-1 of the last run of a CLS_F_TRACE problem:
 * hash[i] = FNV-1a-64 over the 4-byte tuples (event code, material, bin low
 * byte, bin high byte) of history i -- with CLS_F_TRACE_NO_BINS both bin bytes
 * are 0 -- and flights[i] = its number of flights. Event codes: 0 source,
 * 1 interface crossing, 2 scattering, 3 absorption, 4 leak at x = 0, 5 leak at
 * x = L, 6/7 mirror at y = 0 / L, 8/9 mirror at z = 0 / L, 10 flight cap. FP32
 * and FP64 tracking draw the same uniforms, so a history's hash differs between
 * them only where FP32 rounding changed one of its events.
 * n must not exceed min(histories, trace_histories). */
cls_status cls_read_trace(const cls_problem *p, uint64_t *hash, uint32_t *flights, uint64_t n);

/* Run n problems in one persistent-kernel launch. All problems must share d,
 * the slab flag, source, estimator and precision (CLS_ERR_INVALID_ARG
 * otherwise); histories[i] and seeds[i] belong to problems[i]. Every problem
 * receives the same tallies it would get from cls_run with the same histories
 * and seed (counts exactly, FP64 sums up to the order of additions) except
 * flux_sigma and the batch count: the per-bin error is a batch-means estimate,
 * and a batch gathers the chunks one wave takes of a problem (chunk_batches in
 * cls_launch_config), with chunks sized for the whole batch, at least 256
 * batches per problem when its history count allows; flux_sigma is then an
 * equally valid estimate from other batches. The same holds for a different
 * launch configuration or another run. The launch uses the stream of
 * problems[0] and is synchronous. */
cls_status cls_run_batch(cls_problem *const *problems, const uint64_t *histories,
                         const uint64_t *seeds, int n);

/* Graph-captured batch: the same set of problems run repeatedly. The first
 * cls_batch_run captures reset, tracking, finalize and result copy of one
 * batched launch in a hipGraph on the batch's own stream; later runs replay it
 * with new history counts and seeds (the launch shape is the one chosen for
 * the first run's history counts).
 * Problems must satisfy the cls_run_batch rules, must not use CLS_F_TRACE, and
 * stay owned by the caller (they must outlive the batch). cls_batch_run is
 * synchronous; results are read with cls_read_tallies on each problem.
 * cls_batch_last_ms returns the duration of the last replay (HIP events). */
typedef struct cls_batch cls_batch;
cls_status cls_batch_create(cls_problem *const *problems, int n, cls_batch **out);
cls_status cls_batch_run(cls_batch *b, const uint64_t *histories, const uint64_t *seeds);
cls_status cls_batch_last_ms(const cls_batch *b, double *ms);
void cls_batch_destroy(cls_batch *b);

/* Launch shape used by every subsequent run of the process (0 in a field keeps
 * the automatic choice):
 *   waves_per_block  1, 2, 4 or 8 waves of 64 lanes per workgroup (automatic: the
 *                    size that keeps the most waves resident);
 *   blocks_per_cu    persistent workgroups per compute unit (automatic: as many as
 *                    are resident at once);
 *   max_chunk        largest number of histories per work chunk (>= 64; default
 *                    16384);
 *   refill_min       idle lanes a wave waits for before it hands out new
 *                    histories (1..64; default 4; 1 refills every step);
 *   slots            LDS tally buffers per wave, 1 or 2 (automatic: two, or one
 *                    when it keeps more waves resident and at most a fifth of
 *                    the histories are in chunks below 2048); a choice that
 *                    does not fit the LDS falls back to one;
 *   chunk_batches    1: every chunk is one batch of the per-bin flux error;
 *                    0 (default): in runs and batches (not served requests) a
 *                    wave gathers the chunks it takes of one problem into one
 *                    batch of up to max(chunk, n / 256) of the problem's n
 *                    histories, so that a problem keeps at least 256 batches
 *                    when its chunks allow and the flush traffic falls with the
 *                    batch count. Which histories share a batch then depends on
 *                    the order in which waves take chunks, so the batch count
 *                    and the per-bin flux errors (not the counts, the means or
 *                    the per-history errors) vary from run to run.
 * Values out of range give CLS_ERR_INVALID_ARG. */
typedef struct {
    int waves_per_block;
    int blocks_per_cu;
    int max_chunk;
    int refill_min;
    int slots;
    int chunk_batches;
} cls_launch_config;
cls_status cls_set_launch_config(const cls_launch_config *cfg);
cls_status cls_get_launch_config(cls_launch_config *cfg);

/* Autotuner: time candidate launch shapes on a calibration part of about
 * sample_histories histories (0: a
 * quarter of the summed histories, at least 2e7) of the batch cls_run_batch
 * would run for `problems` and `histories` (same rules): the first chunks of
 * every problem, cut as in the whole batch. The search runs in two stages:
 * LDS tally buffers per wave (automatic, 1, 2) x workgroup size (automatic, 2,
 * 4, 8 waves), then, for the fastest, chunk size (4096, 16384, 65536) x refill
 * threshold (1, 4, 16); chunk_batches stays as set. Makes the fastest shape the
 * process-wide launch configuration and returns it
 * in *best (and its rate in histories/s in *best_rate, 0 when it came from the
 * cache). When the environment variable CLS_AUTOTUNE_CACHE names a file,
 * results are cached there per device, kernel variant and mesh-size class.
 * The calibration runs use the problems themselves: afterwards their stored
 * results are those of the last calibration run, so run them again before
 * reading tallies. */
cls_status cls_autotune(cls_problem *const *problems, const uint64_t *histories, int n,
                        uint64_t sample_histories, cls_launch_config *best, double *best_rate);

/* Serving: continuous batching of independent requests.
 *   hbm_budget_bytes     admission limit on the summed device footprint of the
 *                        admitted requests (0: 80% of the free device memory);
 *                        a request that does not fit waits in arrival order
 *                        (one is always admitted when nothing else is);
 *   round_histories      bounds a request's chunk size (work item and error
 *                        batch) to about round_histories / resident waves
 *                        (0: 3e7), while a request keeps at least 256 chunks
 *                        when its history count allows;
 *   max_inflight_rounds  ignored (a server keeps at most two launches, one
 *                        open and one draining);
 *   record_path          0: the finalize kernel writes each request's result
 *                        record straight into the problem's pinned host record
 *                        (when the device can address it); 1: into device memory,
 *                        then a copy. Both give the same record.
 * A worker thread admits requests and keeps one persistent tracking launch (a
 * "round") open at a time: the served kernel handles every geometry,
 * estimator and source of one precision, and takes its work from a queue in
 * pinned host memory that the worker feeds while it runs (small requests whole
 * as they arrive, large ones metered chunk by chunk), so a request that
 * arrives while the round is open joins it at once. The round is closed (it
 * drains; a later request starts a new one) once it has nothing left to
 * publish and an eighth of its waves wait for work (at most 0.5 s after its
 * last item), and after a 10 ms slice when a request it cannot
 * take waits (the other precision, or a mesh finer than its LDS buffers, which
 * hold at least 1024 bins). The wave that flushes a request's last chunk
 * signals the worker, which launches a finalize kernel for it while the round
 * goes on. Each result is the one cls_run would give for the same problem,
 * histories and seed (integer tallies bitwise, FP64 sums up to atomic
 * ordering). A device-side protocol error (an item the kernel refuses, a wave
 * that waited too long for its work, or a request whose chunks all ran without
 * a completion signal) fails every unfinished request and stops the server
 * (worker_status is set; later submissions fail with CLS_ERR_STATE). */
typedef struct cls_server cls_server;
typedef struct {
    size_t hbm_budget_bytes;
    uint64_t round_histories;
    int max_inflight_rounds;
    int record_path;
} cls_server_config;
typedef struct {
    double submit_s, admit_s, done_s;   /* seconds since server creation (-1: not yet) */
    uint64_t histories;
    uint32_t rounds;                     /* launches that carried the request's chunks */
    /* stages (seconds since server creation, -1: not reached): first chunk
     * published to a round, completion signal seen by the worker, finalize
     * launched */
    double publish_s, signal_s, finalize_s;
} cls_request_info;
typedef struct {
    uint64_t submitted, completed, failed, pending, active, rounds, histories_completed;
    size_t hbm_in_use, hbm_peak, hbm_budget;
    int worker_status;                   /* last worker error (cls_status), 0 if none */
    double wave_idle_share;              /* of the time the rounds' waves were alive, the
                                            share they had no history to step and waited
                                            for work (rounds retired so far) */
} cls_server_stats;

/* cfg may be NULL (all defaults). Errors: CLS_ERR_NO_DEVICE, CLS_ERR_DEVICE. */
cls_status cls_server_create(const cls_server_config *cfg, cls_server **out);
/* Queue a run of p (not CLS_F_TRACE; one request per problem at a time; the
 * problem must not be used otherwise until the request is done). Host work
 * only (chunking, a done word, the problem's pinned result record); the
 * request's tallies are placed in the server's device pool when it is
 * admitted. Errors: CLS_ERR_INVALID_ARG, CLS_ERR_STATE (problem already in
 * flight, server stopping or stopped), CLS_ERR_OUT_OF_MEMORY. */
cls_status cls_server_submit(cls_server *s, cls_problem *p, uint64_t histories, uint64_t seed,
                             uint64_t *ticket);
/* CLS_OK when done (read results with cls_read_tallies on the problem),
 * CLS_ERR_NOT_READY while queued or running, or the request's error. */
cls_status cls_server_poll(cls_server *s, uint64_t ticket);
/* Block until done or timeout_s seconds (<= 0: no limit) have passed. */
cls_status cls_server_wait(cls_server *s, uint64_t ticket, double timeout_s);
cls_status cls_server_request_info(cls_server *s, uint64_t ticket, cls_request_info *info);
/* Forget a finished request (its ticket becomes unknown). */
cls_status cls_server_release(cls_server *s, uint64_t ticket);
cls_status cls_server_get_stats(cls_server *s, cls_server_stats *out);
/* Finish all submitted work, then stop the worker and free the server. */
void cls_server_destroy(cls_server *s);

/* ---------------------------------------------------------------------- */
/* Allocation-free run                                                    */
/* ---------------------------------------------------------------------- */
/* For callers that cannot allocate device or pinned memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Runs `histories` histories of p with stream key `seed` exactly as
 * cls_run_async would (same launch shape, chunks and kernels; integer tallies
 * bitwise equal, FP64 sums up to the order of additions), but allocates
 * nothing: the run's device workspace is a static 64 KB array that the library
 * holds on each device it runs on until the process ends, and nothing is
 * copied to the host.
 *   p            a problem from cls_create_problem (only read; CLS_F_TRACE is
 *                rejected; nbins <= 2048, the meshes whose sums fit the 64 KB).
 *   hip_stream   hipStream_t the work is enqueued on (NULL = default stream);
 *                the call returns at once, the caller synchronizes.
 *   d_record     caller-owned device memory, 8-byte aligned, of at least
 *                record_bytes = (24 + 2 nbins) x 8 bytes, receiving the result
 *                record: 16 uint64 counters (histories, transmitted, reflected,
 *                absorbed, capped, flights, collisions, scatters, interface
 *                crossings, lateral reflections, batches, then 5 reserved), 8
 *                doubles (T, R, A, sigma_T, sigma_R, sigma_A, total flux, its
 *                sigma), then flux[nbins] and flux_sigma[nbins] as in
 *                cls_read_tallies.
 * Every call on a device reuses that device's array: calls that overlap on one
 * device (two streams, two threads) race and give wrong results; calls ordered
 * by the caller are independent.
 * Errors: CLS_ERR_INVALID_ARG (NULL arguments, histories == 0, trace problem,
 * nbins above 2048, record buffer too small or misaligned),
 * CLS_ERR_NO_DEVICE, CLS_ERR_DEVICE. */
cls_status cls_run_static(const cls_problem *p, uint64_t histories, uint64_t seed, void *hip_stream,
                          void *d_record, size_t record_bytes);

/* ---------------------------------------------------------------------- */
/* Quenched-disorder reference solutions, d = 1 (Section 3)               */
/* ---------------------------------------------------------------------- */
/* Reference solutions average each observable over realizations of the
 * stochastic medium transported with their geometry frozen (Sec. 3.3). For a
 * d = 1 problem (the rod, or the slab with CLS_F_D1_SLAB), realization k is
 * the Poisson process on the line (Sec. 3.1) of density
 * rho = 1/Lambda_0 + 1/Lambda_1 cutting [0, L] into cells, each of material 0
 * with probability p_0 = Lambda_0 / (Lambda_0 + Lambda_1) (Sec. 3.2); cell i
 * draws its gap -ln(U_0)/rho and its material (U_1 < p_0) from the Philox
 * block (i, 3, lo32(k), hi32(k)) under `seed`, and neighbouring cells of one
 * material form one layer. Each realization transports `histories` histories
 * (history h of realization k is global history g = k * histories + h; its
 * event step j draws the block (j, 2, lo32(g), hi32(g))) with the problem's
 * source, materials and flux estimator; the observables of a realization
 * are its history means, and the results are their means over the
 * `realizations` realizations with the standard error of each mean.
 *
 * cls_run_quenched: synchronous; runs on the problem's stream (cls_set_stream)
 * or the default stream, allocating a small workspace with the problem on the
 * first call. Tracking is FP64 (CLS_F_FP32 and CLS_F_TRACE are rejected).
 * Errors: CLS_ERR_INVALID_ARG (d != 1, FP32 or trace problem, zero counts,
 * realizations x histories >= 2^62, a medium whose expected layer count
 * 1 + 2L/(Lambda_0 + Lambda_1) exceeds 1024 or whose expected cell count
 * rho L exceeds 10^6); CLS_ERR_CAPACITY if a realization had more layers than the
 * workspace holds (its results are then not valid); CLS_ERR_EVENT_CAP if a
 * history reached the flight cap; CLS_ERR_NO_DEVICE; CLS_ERR_DEVICE;
 * CLS_ERR_OUT_OF_MEMORY. */
cls_status cls_run_quenched(cls_problem *p, uint64_t realizations, uint64_t histories, uint64_t seed);

/* Results of the last cls_run_quenched. mean_* are ensemble means of the
 * per-realization history means; sigma_* the standard errors of those means
 * over the independent realizations (geometric spread and transport noise
 * together); spread_* the standard deviation of the per-realization values
 * (the sigma_G of Sec. 3.3). Lk is the leakage (T + R)/2 (suite II). */
typedef struct {
    uint64_t realizations, histories, transmitted, reflected, absorbed, capped;
    uint64_t flights, collisions, scatters, crossings, layers;
    double T, R, A, total_flux, Lk;
    double sigma_T, sigma_R, sigma_A, sigma_total_flux, sigma_Lk;
    double spread_T, spread_R, spread_A, spread_total_flux, spread_Lk;
    double track_ms;               /* GPU time of the transport kernel */
} cls_quenched_tallies;

/* Copies the last quenched results; flux and flux_sigma (caller-owned, nbins
 * doubles each, may be NULL) get the ensemble-mean scalar flux per bin and its
 * standard error. Errors: CLS_ERR_INVALID_ARG (NULL out, nbins differing from
 * the problem's when flux is given), CLS_ERR_STATE (no quenched run yet). */
cls_status cls_read_quenched(const cls_problem *p, cls_quenched_tallies *out, double *flux, double *flux_sigma,
                             int nbins);

/* Status name and the calling thread's last error detail. */
const char *cls_status_string(cls_status s);
const char *cls_last_error(void);

/* Library version string. */
const char *cls_version(void);

#ifdef __cplusplus
}
#endif
#endif
