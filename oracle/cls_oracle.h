/*
 * cls_oracle.h -- plain FP64 CPU reference for Chord Length Sampling.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may build, load or call this library.
 * It shares no code, header or constant table with the GPU library.
 *
 * Method: Algorithm A (Zimmerman and Adams) as restated in Section 4 of
 * Larmier, Lam, Brantley, Malvagi, Palmer, Zoia, "Monte Carlo Chord Length
 * Sampling for d-dimensional Markov binary mixtures" (arXiv 1708.00765),
 * with the benchmark geometry of Section 2 (box of side L, leakage on the two
 * x-faces, reflection on the lateral faces).
 */
#ifndef CLS_ORACLE_H
#define CLS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Geometry: the paper's d=1 slab (Sec. 4.1), 2D extruded (Sec. 4.2), 3D
 * (Sec. 4.3), plus the rod (d=1, directions +-x only). */
enum { ORC_ROD = 0, ORC_SLAB = 1, ORC_EXT2D = 2, ORC_CUBE3D = 3 };
/* Source: suite I = normalized incident flux on x=0; suite II = uniform
 * isotropic interior source (Sec. 2). */
enum { ORC_SRC_FACE = 0, ORC_SRC_VOLUME = 1 };
/* Scalar-flux estimator on the x-mesh (Sec. 3.3 / Sec. 4): collision or
 * track length. */
enum { ORC_EST_COLLISION = 0, ORC_EST_TRACK = 1 };

/* Event codes folded into the per-history trace hash. */
enum {
    ORC_EV_SOURCE = 0, ORC_EV_INTERFACE = 1, ORC_EV_SCATTER = 2, ORC_EV_ABSORB = 3,
    ORC_EV_LEAK_XLO = 4, ORC_EV_LEAK_XHI = 5,
    ORC_EV_REFL_YLO = 6, ORC_EV_REFL_YHI = 7, ORC_EV_REFL_ZLO = 8, ORC_EV_REFL_ZHI = 9,
    ORC_EV_CAP = 10
};

typedef struct {
    int geom;          /* ORC_ROD .. ORC_CUBE3D                                */
    int source;        /* ORC_SRC_FACE or ORC_SRC_VOLUME                       */
    int estimator;     /* ORC_EST_COLLISION or ORC_EST_TRACK                   */
    int nbins;         /* uniform x-mesh on [0, L], >= 1                       */
    double L;          /* box side                                             */
    double sigma[2];   /* total cross sections Sigma_0, Sigma_1                */
    double c[2];       /* scattering ratios c_i = Sigma_s,i / Sigma_i in [0,1] */
    double lambda[2];  /* mean chord lengths Lambda_0, Lambda_1                */
    uint64_t max_steps;/* flight cap per history; 0 selects 10^8              */
} orc_problem;

typedef struct {
    uint64_t histories, transmitted, reflected, absorbed, capped;
    uint64_t flights, collisions, scatters, interfaces, lateral;
    double score_sum;  /* sum over histories of the history's total flux score */
    double score_sq;   /* sum over histories of its square                     */
} orc_counts;

/* One Philox4x32-10 block (exposed for the generator pins). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The five uniforms of event step `step` of history `h` under key `seed`. */
void orc_step_uniforms(uint64_t seed, uint64_t h, uint32_t step, uint32_t lane, double u[5]);

/* Run histories h0 .. h0+n-1.
 *   bin_sum[k], bin_sq[k] (nbins each): sum over histories of the history's
 *   score in bin k, and of its square.
 *   trace_hash[i], trace_len[i] (n each, may be NULL): FNV-1a-64 hash of the
 *   event tuples of history h0+i and its number of flights.
 *   nthreads <= 0 uses every available core. Results are bitwise independent
 *   of nthreads. Returns 0, or -1 on an invalid argument. */
int orc_run(const orc_problem *p, uint64_t seed, uint64_t h0, uint64_t n, int nthreads,
            orc_counts *out, double *bin_sum, double *bin_sq,
            uint64_t *trace_hash, uint32_t *trace_len);

/* Number of OpenMP threads orc_run uses for nthreads <= 0. */
int orc_max_threads(void);

/* ---------------------------------------------------------------------- */
/* Quenched disorder in d = 1 (Section 3): reference solutions            */
/* ---------------------------------------------------------------------- */
/* A realization of the binary Markov slab (Sec. 3.1-3.2): the points of a
 * Poisson process of density rho = 1/Lambda on the line, 1/Lambda =
 * 1/Lambda_0 + 1/Lambda_1, cut [0, L] into cells, and each cell is given
 * material 0 with probability p_0 = Lambda_0 / (Lambda_0 + Lambda_1), 1
 * otherwise. Cell i of realization k spans a gap -ln(U_0)/rho and has
 * material 0 iff U_1 < p_0, with U_0, U_1 the first two uniforms of the
 * Philox block at counter (i, 3, lo32(k), hi32(k)) under the problem seed.
 * Neighbouring cells of one material are merged into one layer.
 * Writes at most cap layers: bounds[0..n] (bounds[0] = 0, bounds[n] = L) and
 * mat[0..n-1]; returns n, or -1 on an invalid argument (a layer count above
 * cap returns the count without writing beyond cap). */
int orc_quenched_layers(const orc_problem *p, uint64_t seed, uint64_t k,
                        double *bounds, int *mat, int cap);

typedef struct {
    uint64_t realizations, histories, transmitted, reflected, absorbed, capped;
    uint64_t flights, collisions, scatters, crossings, layers;
    /* Per-realization means of T, R, A, the total flux (track length per
     * history) and the leakage (T + R)/2: sum over realizations, and sum of
     * squares. */
    double sum[5], sq[5];
} orc_quenched;

/* Run realizations k0 .. k0+M-1 of problem p (geom ORC_ROD or ORC_SLAB), each
 * with N histories transported through its fixed layers (Sec. 3.3): history
 * h of realization k is global history g = k N + h, and its event step j
 * draws the Philox block at counter (j, 2, lo32(g), hi32(g)). Per
 * realization, the observables are history means; bin_sum[b] and bin_sq[b]
 * (nbins each) get the sum over realizations of the realization's mean flux
 * score in bin b (collision or track length, not divided by the bin width)
 * and of its square. Results are bitwise independent of nthreads. Returns
 * 0, or -1 on an invalid argument. */
int orc_run_quenched(const orc_problem *p, uint64_t seed, uint64_t k0, uint64_t M, uint64_t N,
                     int nthreads, orc_quenched *out, double *bin_sum, double *bin_sq);

#ifdef __cplusplus
}
#endif
#endif
