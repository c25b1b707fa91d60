/*
 * cls_oracle.c -- plain FP64 CPU reference for Chord Length Sampling (CLS).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may build, load or call this library;
 * the GPU library never does, and the two share no code.
 *
 * What is computed (Larmier et al., arXiv 1708.00765, Section 4, Algorithm A):
 * every history starts from the source with a material label drawn with the
 * volume fractions p_i = Lambda_i / (Lambda_0 + Lambda_1) (Section 2). Then,
 * until it leaks or is absorbed, it
 *   1. draws the distance to collision l_c, exponential with mean 1/Sigma_m,
 *   2. draws the distance to the next material interface l_i, exponential with
 *      mean Lambda_m projected for the dimension (Lambda/|mu| in the slab,
 *      Sec. 4.1; Lambda/sqrt(1-mu_z^2) in 2D extruded geometry, Sec. 4.2;
 *      Lambda in 3D, Sec. 4.3; Lambda on the rod),
 *   3. computes the distance to the box boundary l_b,
 *   4. moves by the smallest of the three and, for the interface, switches
 *      the label; for a collision, scatters isotropically with probability
 *      c_m or is absorbed; for a boundary, leaks through an x-face (x=L:
 *      transmission, x=0: reflection) or is mirrored by a lateral face
 *      (Section 2: reflective lateral faces),
 *   5. draws a fresh set of distances after every event (Section 4).
 * Scores: outgoing currents on the two x-faces, and the scalar flux on a
 * uniform x-mesh with the collision or the track-length estimator (Sec. 3.3),
 * normalized per source history.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - uniforms: one Philox4x32-10 block per event step, five 23-bit uniforms
 *     U = (k + 1/2) 2^-23 per block (exact in FP32 and FP64; open interval so
 *     that ln U and sqrt U are finite);
 *   - ties: boundary before collision before interface; x-faces before y
 *     before z;
 *   - half-open bins, x = L belongs to the last bin.
 *
 * Build: -O2 -fno-fast-math -ffp-contract=off, libm log/sqrt/sin/cos, FP64.
 */
#include "cls_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_CHUNK 4096u          /* histories per deterministic reduction chunk */
#define ORC_DEFAULT_CAP 100000000ull

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): ten rounds of the 4x32 S-box, key schedule by   */
/* the two Weyl increments.                                                  */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Step `step` of history h draws counter (step, lane, lo32(h), hi32(h)) under
 * key (lo32(seed), hi32(seed)); lane is 0 except for the second source block
 * of the 3D interior source. The 128 output bits give five 23-bit integers:
 * the top 23 bits of each word, and 9 + 9 + 5 low bits of words 0, 1, 2. */
void orc_step_uniforms(uint64_t seed, uint64_t h, uint32_t step, uint32_t lane, double u[5])
{
    uint32_t ctr[4] = { step, lane, (uint32_t)h, (uint32_t)(h >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    uint32_t k[5];
    k[0] = w[0] >> 9;
    k[1] = w[1] >> 9;
    k[2] = w[2] >> 9;
    k[3] = w[3] >> 9;
    k[4] = ((w[0] & 0x1FFu) << 14) | ((w[1] & 0x1FFu) << 5) | (w[2] & 0x1Fu);
    for (int i = 0; i < 5; ++i)
        u[i] = ((double)k[i] + 0.5) * 0x1p-23;
}

/* ------------------------------------------------------------------------ */
/* Per-history bookkeeping                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *score;      /* nbins: this history's score per bin   */
    int kmin, kmax;     /* touched bin range                     */
    double total;       /* this history's total score            */
    uint64_t hash;
    uint32_t flights;
} history_scratch;

static int bin_of(const orc_problem *p, double x)
{
    double dx = p->L / (double)p->nbins;
    double f = floor(x / dx);
    int k = (f < 0.0) ? 0 : (f >= (double)p->nbins ? p->nbins - 1 : (int)f);
    return k;
}

static void add_score(const orc_problem *p, history_scratch *hs, int k, double v)
{
    (void)p;
    hs->score[k] += v;
    hs->total += v;
    if (k < hs->kmin) hs->kmin = k;
    if (k > hs->kmax) hs->kmax = k;
}

/* FNV-1a over the four bytes (event, material, bin low, bin high). */
static void hash_event(history_scratch *hs, int ev, int m, int bin)
{
    const unsigned char bytes[4] = { (unsigned char)ev, (unsigned char)m,
                                     (unsigned char)(bin & 0xFF), (unsigned char)((bin >> 8) & 0xFF) };
    for (int i = 0; i < 4; ++i) {
        hs->hash ^= (uint64_t)bytes[i];
        hs->hash *= 0x100000001B3ull;
    }
}

/* Track-length estimator: the path inside bin k of a straight flight from
 * x_a to x_b with x-cosine ux is (overlap of [x_a, x_b] with bin k) / |ux|.
 * A flight with ux = 0 stays in one bin and scores its full length. */
static void score_track(const orc_problem *p, history_scratch *hs,
                        double xa, double xb, double ux, double len)
{
    if (len <= 0.0) return;
    double lo = xa < xb ? xa : xb;
    double hi = xa < xb ? xb : xa;
    int ka = bin_of(p, lo), kb = bin_of(p, hi);
    if (ux == 0.0 || ka == kb) {
        add_score(p, hs, ka, len);
        return;
    }
    double dx = p->L / (double)p->nbins;
    double aux = fabs(ux);
    for (int k = ka; k <= kb; ++k) {
        double e0 = (double)k * dx, e1 = (double)(k + 1) * dx;
        double a = lo > e0 ? lo : e0;
        double b = hi < e1 ? hi : e1;
        if (b > a) add_score(p, hs, k, (b - a) / aux);
    }
}

/* Number of position axes with faces: x for rod and slab, x,y for 2D, x,y,z
 * for 3D. Directions are 3-vectors except on the rod and slab (x only). */
static int n_axes(int geom)
{
    return geom == ORC_EXT2D ? 2 : (geom == ORC_CUBE3D ? 3 : 1);
}

/* Projection of the unit path onto the plane in which chords are measured:
 * the x-cosine in the slab (Sec. 4.1), the in-plane norm sqrt(ux^2+uy^2) =
 * sqrt(1-mu_z^2) in 2D (Sec. 4.2), 1 in 3D (Sec. 4.3) and on the rod. */
static double chord_factor(int geom, const double u[3])
{
    switch (geom) {
    case ORC_SLAB:  return fabs(u[0]);
    case ORC_EXT2D: return sqrt(u[0] * u[0] + u[1] * u[1]);
    default:        return 1.0;
    }
}

/* Isotropic direction from two uniforms: mu = 2U-1 is the cosine to the
 * polar axis z, phi = 2 pi U' the azimuth (Sec. 4.2, 4.3). */
static void isotropic_direction(double ua, double ub, double u[3])
{
    double mu = 2.0 * ua - 1.0;
    double phi = 2.0 * ORC_PI * ub;
    double st = sqrt(1.0 - mu * mu);
    u[0] = st * cos(phi);
    u[1] = st * sin(phi);
    u[2] = mu;
}

/* One history. Returns its outcome event (leak, absorb or cap). */
static int run_history(const orc_problem *p, uint64_t seed, uint64_t h,
                       history_scratch *hs, orc_counts *cnt)
{
    const double L = p->L;
    const int axes = n_axes(p->geom);
    const uint64_t cap = p->max_steps ? p->max_steps : ORC_DEFAULT_CAP;
    double U[5];
    double x[3] = { 0.0, 0.0, 0.0 };
    double u[3] = { 0.0, 0.0, 0.0 };
    int m;

    /* --- source (step 0) --------------------------------------------- */
    orc_step_uniforms(seed, h, 0, 0, U);
    double p0 = p->lambda[0] / (p->lambda[0] + p->lambda[1]);
    m = (U[0] < p0) ? 0 : 1;
    if (p->source == ORC_SRC_FACE) {
        /* Suite I: x = 0, inward cosine-weighted direction mu' = sqrt(U)
         * about +x (Sec. 4.1-4.3); the rod enters along +x. */
        if (p->geom == ORC_ROD) {
            u[0] = 1.0;
        } else if (p->geom == ORC_SLAB) {
            u[0] = sqrt(U[1]);
        } else {
            double mup = sqrt(U[1]);
            double phip = 2.0 * ORC_PI * U[2];
            double st = sqrt(1.0 - mup * mup);
            u[0] = mup;
            u[1] = st * cos(phip);
            u[2] = st * sin(phip);
            x[1] = L * U[3];
            if (p->geom == ORC_CUBE3D) x[2] = L * U[4];
        }
    } else {
        /* Suite II: position uniform in the box, direction isotropic. */
        x[0] = L * U[1];
        if (p->geom == ORC_ROD) {
            u[0] = (U[2] < 0.5) ? 1.0 : -1.0;
        } else if (p->geom == ORC_SLAB) {
            u[0] = 2.0 * U[2] - 1.0;
        } else if (p->geom == ORC_EXT2D) {
            x[1] = L * U[2];
            isotropic_direction(U[3], U[4], u);
        } else {
            isotropic_direction(U[2], U[3], u);
            x[1] = L * U[4];
            double V[5];
            orc_step_uniforms(seed, h, 0, 1, V);
            x[2] = L * V[0];
        }
    }
    hash_event(hs, ORC_EV_SOURCE, m, bin_of(p, x[0]));

    /* --- flights (steps 1, 2, ...) ------------------------------------ */
    for (uint64_t step = 1;; ++step) {
        if (step > cap) {
            hash_event(hs, ORC_EV_CAP, m, bin_of(p, x[0]));
            cnt->capped++;
            return ORC_EV_CAP;
        }
        orc_step_uniforms(seed, h, (uint32_t)step, 0, U);
        hs->flights++;
        cnt->flights++;

        double lc = -log(U[0]) / p->sigma[m];
        double g = chord_factor(p->geom, u);
        double li = (g > 0.0) ? -log(U[1]) * p->lambda[m] / g : INFINITY;
        double lb = INFINITY;
        int face = -1;            /* 2*axis + (1 for the face at L)     */
        for (int a = 0; a < axes; ++a) {
            double d;
            int f;
            if (u[a] > 0.0)      { d = (L - x[a]) / u[a];   f = 2 * a + 1; }
            else if (u[a] < 0.0) { d = (0.0 - x[a]) / u[a]; f = 2 * a; }
            else continue;
            if (d < lb) { lb = d; face = f; }
        }

        int event;                /* 0 boundary, 1 collision, 2 interface */
        double s;
        if (lb <= lc && lb <= li) { event = 0; s = lb; }
        else if (lc <= li)        { event = 1; s = lc; }
        else                      { event = 2; s = li; }

        double xa = x[0];
        for (int a = 0; a < axes; ++a) x[a] += s * u[a];
        if (event == 0) x[face / 2] = (face & 1) ? L : 0.0;
        if (p->estimator == ORC_EST_TRACK) score_track(p, hs, xa, x[0], u[0], s);

        const int mf = m;         /* material during this flight */
        if (event == 0) {
            if (face == 0) { hash_event(hs, ORC_EV_LEAK_XLO, mf, bin_of(p, x[0])); cnt->reflected++; return ORC_EV_LEAK_XLO; }
            if (face == 1) { hash_event(hs, ORC_EV_LEAK_XHI, mf, bin_of(p, x[0])); cnt->transmitted++; return ORC_EV_LEAK_XHI; }
            u[face / 2] = -u[face / 2];           /* mirror on a lateral face */
            cnt->lateral++;
            hash_event(hs, ORC_EV_REFL_YLO + (face - 2), mf, bin_of(p, x[0]));
        } else if (event == 2) {
            m = 1 - m;                            /* cross into the other material */
            cnt->interfaces++;
            hash_event(hs, ORC_EV_INTERFACE, mf, bin_of(p, x[0]));
        } else {
            cnt->collisions++;
            int k = bin_of(p, x[0]);
            if (p->estimator == ORC_EST_COLLISION) add_score(p, hs, k, 1.0 / p->sigma[m]);
            if (U[2] < p->c[m]) {
                cnt->scatters++;
                if (p->geom == ORC_ROD)       u[0] = (U[3] < 0.5) ? 1.0 : -1.0;
                else if (p->geom == ORC_SLAB) u[0] = 2.0 * U[3] - 1.0;
                else                          isotropic_direction(U[3], U[4], u);
                hash_event(hs, ORC_EV_SCATTER, mf, k);
            } else {
                cnt->absorbed++;
                hash_event(hs, ORC_EV_ABSORB, mf, k);
                return ORC_EV_ABSORB;
            }
        }
    }
}

static int valid_problem(const orc_problem *p)
{
    if (!p) return 0;
    if (p->geom < ORC_ROD || p->geom > ORC_CUBE3D) return 0;
    if (p->source != ORC_SRC_FACE && p->source != ORC_SRC_VOLUME) return 0;
    if (p->estimator != ORC_EST_COLLISION && p->estimator != ORC_EST_TRACK) return 0;
    if (p->nbins < 1 || p->nbins > 65535) return 0;
    if (!(p->L > 0.0) || !isfinite(p->L)) return 0;
    for (int i = 0; i < 2; ++i) {
        if (!(p->sigma[i] > 0.0) || !isfinite(p->sigma[i])) return 0;
        if (!(p->c[i] >= 0.0 && p->c[i] <= 1.0)) return 0;
        if (!(p->lambda[i] > 0.0) || !isfinite(p->lambda[i])) return 0;
    }
    return 1;
}

typedef struct {
    orc_counts cnt;
    double *bin_sum, *bin_sq;
} chunk_partial;

static void run_chunk(const orc_problem *p, uint64_t seed, uint64_t first, uint64_t count,
                      chunk_partial *cp, double *score, uint64_t *trace_hash, uint32_t *trace_len,
                      uint64_t h0)
{
    memset(&cp->cnt, 0, sizeof cp->cnt);
    memset(cp->bin_sum, 0, sizeof(double) * (size_t)p->nbins);
    memset(cp->bin_sq, 0, sizeof(double) * (size_t)p->nbins);
    for (uint64_t h = first; h < first + count; ++h) {
        history_scratch hs;
        hs.score = score;
        hs.kmin = p->nbins;
        hs.kmax = -1;
        hs.total = 0.0;
        hs.hash = 0xCBF29CE484222325ull;
        hs.flights = 0;
        run_history(p, seed, h, &hs, &cp->cnt);
        cp->cnt.histories++;
        for (int k = hs.kmin; k <= hs.kmax; ++k) {
            cp->bin_sum[k] += score[k];
            cp->bin_sq[k] += score[k] * score[k];
            score[k] = 0.0;
        }
        cp->cnt.score_sum += hs.total;
        cp->cnt.score_sq += hs.total * hs.total;
        if (trace_hash) trace_hash[h - h0] = hs.hash;
        if (trace_len) trace_len[h - h0] = hs.flights;
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_run(const orc_problem *p, uint64_t seed, uint64_t h0, uint64_t n, int nthreads,
            orc_counts *out, double *bin_sum, double *bin_sq,
            uint64_t *trace_hash, uint32_t *trace_len)
{
    if (!valid_problem(p) || !out || !bin_sum || !bin_sq) return -1;
    const int K = p->nbins;
    int nt = nthreads > 0 ? nthreads : orc_max_threads();
    memset(out, 0, sizeof *out);
    memset(bin_sum, 0, sizeof(double) * (size_t)K);
    memset(bin_sq, 0, sizeof(double) * (size_t)K);
    if (n == 0) return 0;

    /* Chunks of ORC_CHUNK histories are run in parallel in groups; partials
     * are then added in chunk order, so the result does not depend on the
     * thread count. */
    const uint64_t nchunks = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    const uint64_t group = (uint64_t)nt * 8u;
    chunk_partial *cps = (chunk_partial *)calloc((size_t)group, sizeof *cps);
    double *arena = (double *)calloc((size_t)group * 2u * (size_t)K, sizeof(double));
    double *scores = (double *)calloc((size_t)nt * (size_t)K, sizeof(double));
    if (!cps || !arena || !scores) { free(cps); free(arena); free(scores); return -1; }
    for (uint64_t i = 0; i < group; ++i) {
        cps[i].bin_sum = arena + (size_t)(2u * i) * (size_t)K;
        cps[i].bin_sq = arena + (size_t)(2u * i + 1u) * (size_t)K;
    }

    for (uint64_t g0 = 0; g0 < nchunks; g0 += group) {
        uint64_t gn = (nchunks - g0) < group ? (nchunks - g0) : group;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
        for (long long ci = 0; ci < (long long)gn; ++ci) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            uint64_t chunk = g0 + (uint64_t)ci;
            uint64_t first = h0 + chunk * ORC_CHUNK;
            uint64_t count = (chunk + 1 == nchunks) ? (n - chunk * ORC_CHUNK) : ORC_CHUNK;
            run_chunk(p, seed, first, count, &cps[ci], scores + (size_t)tid * (size_t)K,
                      trace_hash, trace_len, h0);
        }
        for (uint64_t ci = 0; ci < gn; ++ci) {
            const orc_counts *c = &cps[ci].cnt;
            out->histories += c->histories;
            out->transmitted += c->transmitted;
            out->reflected += c->reflected;
            out->absorbed += c->absorbed;
            out->capped += c->capped;
            out->flights += c->flights;
            out->collisions += c->collisions;
            out->scatters += c->scatters;
            out->interfaces += c->interfaces;
            out->lateral += c->lateral;
            out->score_sum += c->score_sum;
            out->score_sq += c->score_sq;
            for (int k = 0; k < K; ++k) {
                bin_sum[k] += cps[ci].bin_sum[k];
                bin_sq[k] += cps[ci].bin_sq[k];
            }
        }
    }
    free(cps);
    free(arena);
    free(scores);
    return 0;
}

/* ======================================================================== */
/* Quenched disorder in d = 1 (Section 3): reference solutions               */
/* ======================================================================== */
/*
 * Section 3 builds reference solutions by sampling realizations of the
 * stochastic medium and transporting particles through each one with the
 * geometry frozen, then averaging the observables over realizations. In
 * d = 1 a realization is the Poisson process on the line (Sec. 3.1): points
 * of density rho = 1/Lambda cut [0, L] into cells, and each cell is coloured
 * with material 0 with probability p_0 (Sec. 3.2), where
 *   1/Lambda = 1/Lambda_0 + 1/Lambda_1,   p_0 = Lambda_0 / (Lambda_0 + Lambda_1),
 * so that the clusters of material i have mean chord Lambda_i. Transport in
 * a realization is ordinary surface tracking: the distance to collision in
 * the current layer's material against the distance to the layer's face.
 * Per realization the observables are history means (Sec. 3.3); the
 * ensemble average is their mean over realizations.
 *
 * Readings (listed in the design notes): cells are generated from x = 0 by
 * exponential gaps (the Poisson process restricted to [0, L]); neighbouring
 * cells of one material form one layer (the medium is the same, and the
 * transport draws a fresh collision distance at every face); ties between
 * the face and the collision go to the face.
 */

typedef struct {
    double *b;          /* n + 1 bounds                    */
    int *m;             /* n materials                     */
    int n, cap;
} orc_layers;

static int layers_push(orc_layers *ly, double x, int mat)
{
    if (ly->n + 2 > ly->cap) {
        int nc = ly->cap ? 2 * ly->cap : 64;
        double *nb = (double *)realloc(ly->b, sizeof(double) * (size_t)nc);
        if (!nb) return -1;
        ly->b = nb;
        int *nm = (int *)realloc(ly->m, sizeof(int) * (size_t)nc);
        if (!nm) return -1;
        ly->m = nm;
        ly->cap = nc;
    }
    ly->b[ly->n] = x;
    ly->m[ly->n] = mat;
    ly->n++;
    return 0;
}

/* Realization k: cell i has gap -ln(U_0)/rho and material 0 iff U_1 < p_0,
 * from the block at counter (i, 3, lo32(k), hi32(k)). */
static int make_layers(const orc_problem *p, uint64_t seed, uint64_t k, orc_layers *ly)
{
    const double rho = 1.0 / p->lambda[0] + 1.0 / p->lambda[1];
    const double p0 = p->lambda[0] / (p->lambda[0] + p->lambda[1]);
    double x = 0.0;
    ly->n = 0;
    for (uint32_t i = 0;; ++i) {
        double U[5];
        orc_step_uniforms(seed, k, i, 3, U);
        int mat = (U[1] < p0) ? 0 : 1;
        double end = x + (-log(U[0]) / rho);
        if (ly->n == 0 || ly->m[ly->n - 1] != mat) {
            if (layers_push(ly, x, mat) != 0) return -1;
        }
        if (end >= p->L) break;
        x = end;
    }
    ly->b[ly->n] = p->L;
    return ly->n;
}

static int valid_quenched(const orc_problem *p)
{
    return valid_problem(p) && (p->geom == ORC_ROD || p->geom == ORC_SLAB);
}

int orc_quenched_layers(const orc_problem *p, uint64_t seed, uint64_t k,
                        double *bounds, int *mat, int cap)
{
    if (!valid_quenched(p) || !bounds || !mat || cap < 1) return -1;
    orc_layers ly = { NULL, NULL, 0, 0 };
    int n = make_layers(p, seed, k, &ly);
    if (n > 0) {
        int w = n < cap ? n : cap;
        for (int i = 0; i < w; ++i) {
            bounds[i] = ly.b[i];
            mat[i] = ly.m[i];
        }
        if (n <= cap) bounds[n] = ly.b[n];
    }
    free(ly.b);
    free(ly.m);
    return n;
}

typedef struct {
    uint64_t histories, transmitted, reflected, absorbed, capped;
    uint64_t flights, collisions, scatters, crossings;
} quenched_counts;

/* One history of global index g through the layers of its realization. */
static int run_quenched_history(const orc_problem *p, const orc_layers *ly, uint64_t seed, uint64_t g,
                                history_scratch *hs, quenched_counts *cnt)
{
    const double L = p->L;
    const uint64_t cap = p->max_steps ? p->max_steps : ORC_DEFAULT_CAP;
    double U[5];
    double x = 0.0, mu;
    int layer = 0;

    /* --- source (step 0): the same laws as the CLS source in d = 1 ------ */
    orc_step_uniforms(seed, g, 0, 2, U);
    if (p->source == ORC_SRC_FACE) {
        mu = (p->geom == ORC_ROD) ? 1.0 : sqrt(U[1]);
    } else {
        x = L * U[1];
        if (p->geom == ORC_ROD) mu = (U[2] < 0.5) ? 1.0 : -1.0;
        else                    mu = 2.0 * U[2] - 1.0;
        while (layer + 1 < ly->n && ly->b[layer + 1] <= x) ++layer;   /* x in [b_i, b_i+1) */
    }
    int m = ly->m[layer];

    for (uint64_t step = 1;; ++step) {
        if (step > cap) { cnt->capped++; return ORC_EV_CAP; }
        orc_step_uniforms(seed, g, (uint32_t)step, 2, U);
        hs->flights++;
        cnt->flights++;
        double lc = -log(U[0]) / p->sigma[m];
        double face = (mu > 0.0) ? ly->b[layer + 1] : ly->b[layer];
        double lb = (face - x) / mu;
        double xa = x;
        if (lb <= lc) {
            /* reach the layer's face: leak through x = 0 or x = L, or enter
             * the neighbouring layer */
            x = face;
            if (p->estimator == ORC_EST_TRACK) score_track(p, hs, xa, x, mu, lb);
            if (mu > 0.0 && layer + 1 == ly->n) { cnt->transmitted++; return ORC_EV_LEAK_XHI; }
            if (mu < 0.0 && layer == 0)         { cnt->reflected++;   return ORC_EV_LEAK_XLO; }
            layer += (mu > 0.0) ? 1 : -1;
            m = ly->m[layer];
            cnt->crossings++;
        } else {
            x += lc * mu;
            if (p->estimator == ORC_EST_TRACK) score_track(p, hs, xa, x, mu, lc);
            cnt->collisions++;
            if (p->estimator == ORC_EST_COLLISION) add_score(p, hs, bin_of(p, x), 1.0 / p->sigma[m]);
            if (U[2] < p->c[m]) {
                cnt->scatters++;
                if (p->geom == ORC_ROD) mu = (U[3] < 0.5) ? 1.0 : -1.0;
                else                    mu = 2.0 * U[3] - 1.0;
            } else {
                cnt->absorbed++;
                return ORC_EV_ABSORB;
            }
        }
    }
}

typedef struct {
    quenched_counts cnt;
    uint64_t layers;
    double obs[5];      /* T, R, A, total flux, leakage: this realization's history means */
    double *bin;        /* nbins: this realization's mean score per bin           */
    int failed;
} realization_partial;

static void run_realization(const orc_problem *p, uint64_t seed, uint64_t k, uint64_t N,
                            realization_partial *rp, double *score, orc_layers *ly)
{
    memset(&rp->cnt, 0, sizeof rp->cnt);
    memset(rp->bin, 0, sizeof(double) * (size_t)p->nbins);
    rp->failed = 0;
    int n = make_layers(p, seed, k, ly);
    if (n < 0) { rp->failed = 1; return; }
    rp->layers = (uint64_t)n;
    double total = 0.0;
    for (uint64_t h = 0; h < N; ++h) {
        history_scratch hs;
        hs.score = score;
        hs.kmin = p->nbins;
        hs.kmax = -1;
        hs.total = 0.0;
        hs.hash = 0xCBF29CE484222325ull;
        hs.flights = 0;
        run_quenched_history(p, ly, seed, k * N + h, &hs, &rp->cnt);
        rp->cnt.histories++;
        for (int b = hs.kmin; b <= hs.kmax; ++b) {
            rp->bin[b] += score[b];
            score[b] = 0.0;
        }
        total += hs.total;
    }
    const double inv = 1.0 / (double)N;
    rp->obs[0] = (double)rp->cnt.transmitted * inv;
    rp->obs[1] = (double)rp->cnt.reflected * inv;
    rp->obs[2] = (double)rp->cnt.absorbed * inv;
    rp->obs[3] = total * inv;
    rp->obs[4] = 0.5 * (rp->obs[0] + rp->obs[1]);
    for (int b = 0; b < p->nbins; ++b) rp->bin[b] *= inv;
}

int orc_run_quenched(const orc_problem *p, uint64_t seed, uint64_t k0, uint64_t M, uint64_t N,
                     int nthreads, orc_quenched *out, double *bin_sum, double *bin_sq)
{
    if (!valid_quenched(p) || !out || !bin_sum || !bin_sq || N == 0) return -1;
    const int K = p->nbins;
    int nt = nthreads > 0 ? nthreads : orc_max_threads();
    memset(out, 0, sizeof *out);
    memset(bin_sum, 0, sizeof(double) * (size_t)K);
    memset(bin_sq, 0, sizeof(double) * (size_t)K);
    if (M == 0) return 0;

    /* Realizations run in parallel in groups; their partials are added in
     * realization order, so the result does not depend on the thread count. */
    const uint64_t group = (uint64_t)nt * 8u;
    realization_partial *rps = (realization_partial *)calloc((size_t)group, sizeof *rps);
    double *arena = (double *)calloc((size_t)group * (size_t)K, sizeof(double));
    double *scores = (double *)calloc((size_t)nt * (size_t)K, sizeof(double));
    orc_layers *lys = (orc_layers *)calloc((size_t)nt, sizeof *lys);
    if (!rps || !arena || !scores || !lys) { free(rps); free(arena); free(scores); free(lys); return -1; }
    for (uint64_t i = 0; i < group; ++i) rps[i].bin = arena + (size_t)i * (size_t)K;

    int rc = 0;
    for (uint64_t g0 = 0; g0 < M && rc == 0; g0 += group) {
        uint64_t gn = (M - g0) < group ? (M - g0) : group;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
        for (long long ri = 0; ri < (long long)gn; ++ri) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            run_realization(p, seed, k0 + g0 + (uint64_t)ri, N, &rps[ri], scores + (size_t)tid * (size_t)K,
                            &lys[tid]);
        }
        for (uint64_t ri = 0; ri < gn; ++ri) {
            const realization_partial *rp = &rps[ri];
            if (rp->failed) { rc = -1; break; }
            out->realizations++;
            out->histories += rp->cnt.histories;
            out->transmitted += rp->cnt.transmitted;
            out->reflected += rp->cnt.reflected;
            out->absorbed += rp->cnt.absorbed;
            out->capped += rp->cnt.capped;
            out->flights += rp->cnt.flights;
            out->collisions += rp->cnt.collisions;
            out->scatters += rp->cnt.scatters;
            out->crossings += rp->cnt.crossings;
            out->layers += rp->layers;
            for (int j = 0; j < 5; ++j) {
                out->sum[j] += rp->obs[j];
                out->sq[j] += rp->obs[j] * rp->obs[j];
            }
            for (int b = 0; b < K; ++b) {
                bin_sum[b] += rp->bin[b];
                bin_sq[b] += rp->bin[b] * rp->bin[b];
            }
        }
    }
    for (int t = 0; t < nt; ++t) { free(lys[t].b); free(lys[t].m); }
    free(lys);
    free(rps);
    free(arena);
    free(scores);
    return rc;
}
