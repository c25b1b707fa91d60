// HIP kernels of the Chord Length Sampling library (gfx950).
//
// The tracking kernel runs Algorithm A of Chord Length Sampling (Larmier et
// al., arXiv 1708.00765, Section 4): from the source (position, direction and
// a material label drawn with the volume fractions p_i of Section 2), every
// history repeatedly draws the distance to collision l_c (mean 1/Sigma_m), the
// distance to the next material interface l_i (mean chord Lambda_m, projected
// per dimension: Sec. 4.1 slab, 4.2 extruded 2D, 4.3 3D), computes the distance
// to the box boundary l_b, moves by the smallest, and then switches material,
// scatters isotropically (probability c_m), is absorbed, leaks through an
// x-face or is mirrored by a lateral face (Section 2).
//
// Design (MI355X, wave64):
//  * one history per lane, all particle state in registers; a lane whose
//    history ends takes the next history of its wave's work chunk at the top
//    of the next step, so lanes stay busy until the chunk queue is empty; the
//    lanes in flight are a wave mask, which a lane reads with no vector
//    instruction (inverse ballot);
//  * every step consumes exactly one Philox block per lane (source step or
//    flight), so the random-number work never diverges;
//  * the source and the scattering direction share one direction sampler;
//  * each wave owns two LDS tally buffers ("slots"), one per batch of the
//    batch-means flux error in flight: histories of the batch being filled go
//    to one, stragglers of the previous batch finish in the other, and a
//    batch's buffer is flushed to HBM with FP64 atomics once its last history
//    ends (with fine meshes a launch may give each wave one buffer, which
//    then waits for its batch's last history before it starts the next);
//  * work comes in chunks of consecutive histories from one queue per
//    problem, and a wave keeps taking chunks of its problem: in a batch launch
//    the chunks a wave takes of one problem join the batch it is filling up
//    to the problem's batch size, so a launch flushes about one batch per wave
//    and problem instead of one per chunk (served rounds flush every chunk);
//  * a served round runs every kind of problem of one precision, each kind in
//    a tracking loop of its own (compiled as a batch kernel's is), entered for
//    the kind of the chunk the wave holds;
//  * track-length flux goes to the LDS buffer in difference form (four LDS
//    FP64 atomics per flight whatever the number of bins crossed); the flush
//    prefix-scans it across the wave;
//  * per-history scores and event counts are summed in each lane's registers
//    over its histories of one chunk and reach the slot's LDS counters when
//    the lane takes a history of another chunk or the slot is flushed;
//    collisions and lateral reflections are derived when the record is made.
#include <map>
#include <mutex>
#include <type_traits>

#include "cls_internal.hpp"
#include "philox.hpp"

namespace cls {

// ---------------------------------------------------------------------------
// precision-specific math
// ---------------------------------------------------------------------------
template <typename R>
struct Math;

template <>
struct Math<float> {
    // the logarithm a flight distance is scaled from: hardware log2 (the
    // distance scales carry the factor -ln 2)
    static __device__ __forceinline__ float dlog(float u) { return __builtin_amdgcn_logf(u); }
    static __device__ __forceinline__ float sqrt_(float v) { return __builtin_amdgcn_sqrtf(v); }
    static __device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
    static __device__ __forceinline__ float rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
    static __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float abs_(float v) { return __builtin_fabsf(v); }
    // sin and cos of 2 pi u: the hardware takes its argument in turns
    static __device__ __forceinline__ void sincos_turns(float u, float *s, float *c)
    {
        *s = __builtin_amdgcn_sinf(u);
        *c = __builtin_amdgcn_cosf(u);
    }
};

template <>
struct Math<double> {
    // -ln(u): the distance scales are 1/Sigma_i and Lambda_i themselves
    static __device__ __forceinline__ double dlog(double u) { return -log(u); }
    static __device__ __forceinline__ double sqrt_(double v) { return sqrt(v); }
    static __device__ __forceinline__ double rcp(double v) { return 1.0 / v; }
    static __device__ __forceinline__ double rsqrt(double v) { return 1.0 / sqrt(v); }
    static __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double abs_(double v) { return __builtin_fabs(v); }
    static __device__ __forceinline__ void sincos_turns(double u, double *s, double *c)
    {
        sincos(6.283185307179586476925286766559 * u, s, c);
    }
};

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t rank_in(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l)
{
    return ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), l) << 32) |
           (uint64_t)__builtin_amdgcn_readlane((uint32_t)v, l);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_inclusive_scan(double v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        double t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

__device__ __forceinline__ void lds_add(double *p, double v) { atomicAdd(p, v); }

__device__ __forceinline__ uint64_t fnv_event(uint64_t h, int ev, int m, int bin)
{
    const uint32_t bytes[4] = {(uint32_t)ev & 0xFFu, (uint32_t)m & 0xFFu, (uint32_t)bin & 0xFFu,
                               ((uint32_t)bin >> 8) & 0xFFu};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h ^= (uint64_t)bytes[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

// ---------------------------------------------------------------------------
// per-slot bookkeeping (wave-uniform values)
// ---------------------------------------------------------------------------
// Event counters of a slot, in the order of the global counters they are
// added to (slot_ctr_to_global); collisions and lateral reflections are
// derived in the record (record_into).
enum SlotCtr : int { S_T = 0, S_R, S_A, S_CAP, S_FLIGHTS, S_SCAT, S_INT, S_NCTR };
// Their 64-bit LDS words: transmitted and reflected share one (low and high
// half), absorbed and capped another (each half counts histories of the
// batch, below 2^31, so the halves never carry into each other); flights,
// scatters and interface crossings have one each, and the last word of the
// slot's area holds the histories of its batch.
enum SlotWord : int { W_TR = 0, W_AC, W_FLIGHTS, W_SCAT, W_INT, W_STORED };
constexpr int W_TOTAL = kSlotCounters - 1;
// Two words of slot 0's area that no counter uses hold, in a batch launch, the
// wave's problem and its pending chunk (see the kernel).
constexpr int W_HOME = W_STORED, W_PEND = W_STORED + 1;
static_assert(W_PEND < W_TOTAL, "slot counters do not fit their LDS area");
static_assert(EV_LEAK_XHI - EV_LEAK_XHI == S_T && EV_LEAK_XHI - EV_LEAK_XLO == S_R &&
                  EV_LEAK_XHI - EV_ABSORB == S_A,
              "outcome counters follow the leak and absorption event codes");

// Problem parameters used by an event step. Loaded each step: with scalar
// loads (SGPRs) when every live lane of the wave tracks the same problem, per
// lane otherwise (a wave straddling two work chunks of different problems).
template <typename R>
struct Prm {
    R Lr, dxr;
    double Ld, inv_dx, dx;
    int K;
    uint32_t p0thr;
    uint32_t key_lo, key_hi;
    uint64_t trace_n, max_steps;
    uint64_t *trace_hash;
    uint32_t *trace_len;
    int trace_bins;
};

// The problem records are written by the host before the launch and only read
// by the kernel: reading them through the constant address space lets the
// compiler use scalar loads (SGPRs) for a wave-uniform record.
typedef const __attribute__((address_space(4))) DevProblem ConstProblem;

template <typename R>
__device__ __forceinline__ Prm<R> load_prm(ConstProblem &P)
{
    Prm<R> q;
    if constexpr (std::is_same<R, float>::value) {
        q.Lr = P.Lf; q.dxr = P.dxf;
    } else {
        q.Lr = P.L; q.dxr = P.dx;
    }
    q.Ld = P.L; q.inv_dx = P.inv_dx; q.dx = P.dx; q.K = P.nbins;
    q.p0thr = P.p0thr;
    q.key_lo = (uint32_t)P.seed; q.key_hi = (uint32_t)(P.seed >> 32);
    q.trace_n = P.trace_n; q.max_steps = P.max_steps;
    q.trace_hash = P.trace_hash; q.trace_len = P.trace_len;
    q.trace_bins = P.trace_bins;
    return q;
}

// Flight parameters of one material of a problem, kept per chunk slot in LDS
// (written when the slot takes a chunk): the collision and interface distance
// scales (FP32: -ln2 / Sigma_i and -ln2 Lambda_i, applied to log2 U; FP64:
// 1 / Sigma_i and Lambda_i, applied to -ln U), 1 / Sigma_i and the integer
// threshold of the scattering decision (see DevProblem::cthr). A flight reads
// its material's row with one LDS load instead of selecting four values
// between the two materials.
template <typename R>
struct alignas(16) MatRow {
    R ds, dl;
    uint32_t cthr;
    R isig;
};
static_assert(sizeof(MatRow<float>) == 16 && sizeof(MatRow<double>) == 32, "material rows of 16 / 32 bytes");

template <typename R>
__device__ __forceinline__ MatRow<R> mat_row(ConstProblem &P, int m)
{
    MatRow<R> r;
    if constexpr (std::is_same<R, float>::value) {
        r.ds = P.dsigf[m]; r.dl = P.dlamf[m]; r.isig = P.isigf[m];
    } else {
        r.ds = P.isig[m]; r.dl = P.lam[m]; r.isig = P.isig[m];
    }
    r.cthr = P.cthr[m];
    return r;
}

// Per-lane particle state. The lateral coordinates are kept as the distance
// along each axis to the lateral face the particle is heading for (the face
// at y = L when u_y > 0, at y = 0 otherwise), which is all that the flight
// needs: the distance to that face is dy / |u_y|, a flight of length s takes
// s |u_y| off it, a mirror reflection resets it to L, and a new direction
// whose u_y has the other sign turns it into L - dy. Positions (x and these
// distances) are FP64 in both tracking precisions.
template <typename R>
struct Lane {
    double x;
    double dy, dz;           // distance along y / z to the face headed for
    R ux, uy, uz;
    R iux, aiuy, aiuz, ig;   // 1/u_x, |1/u_y|, |1/u_z|, 1/(chord factor)
    R fx;                    // x inside its flux bin, in bin widths (FP32 track-length)
    double tscore;           // this history's flux score
    // Sums over the lane's histories in chunk slot `slot` (the current one
    // included): flux score and its square per history, interface crossings,
    // scatters, lateral reflections and the outcomes. They move to the slot's
    // LDS counters only when the lane changes slot or the slot is flushed, so
    // that a history's end costs no LDS atomics (all ending lanes would hit
    // the same addresses).
    double ssum, ssq;
    uint64_t h;
    uint64_t hash;
    uint32_t step;
    uint32_t n_int, n_scat, n_fl;   // interface crossings, scatters, flights (of finished histories)
    uint32_t n_t, n_r, n_a, n_cap;
    int m, slot, kcur;       // material, chunk slot (its problem and LDS buffer), bin of x
};

// Flux bin of x and, in FP32, the position of x inside that bin in bin
// widths. Positions lie in [0, L] up to the rounding of a leaking FP32 move
// (never below -dx), and truncation maps t in (-1, 0) to bin 0, so only the
// upper end needs a clamp (x = L, or just beyond, is in bin K - 1).
template <typename R>
__device__ __forceinline__ int bin_of(double x, double inv_dx, int K, R *frac)
{
    const double t = x * inv_dx;
    const int k = min((int)t, K - 1);
    if (sizeof(R) == 4) *frac = (R)(t - (double)k);
    return k;
}

// U < 1/2 as an integer test on the uniform's bit pattern (see
// DevProblem::cthr): k < 2^22.
constexpr uint32_t kHalfThr = 0x3FC00000u;

// One event step of one lane: the source (step 0) or a flight. Returns the
// event code. `tal` is the lane's LDS tally buffer.
template <int G, int EST, int SRC, bool FP32, bool TRACE, typename R>
__device__ __forceinline__ int event_step(Lane<R> &L, const Prm<R> &P, double *tal, const MatRow<R> *mtab)
{
    using MM = Math<R>;
    constexpr int AXES = (G == GEOM_EXT2D) ? 2 : (G == GEOM_CUBE3D ? 3 : 1);
    constexpr bool DIR3 = (G == GEOM_EXT2D || G == GEOM_CUBE3D);

    const Block5 B = philox_u23(L.step, 0u, L.h, P.key_lo, P.key_hi);
    int ev;
    bool need_dir = false, src_dir = false;
    R cos_t = 0, turns = 0;
    if (L.step == 0) {
        // ---- source (Section 2; Sec. 4.1-4.3) ----
        // Lateral coordinates go into dy / dz with u_y = u_z = -1 standing for
        // "heading for the face at 0"; the direction sampler below converts
        // them to distances to the faces the sampled direction heads for.
        L.m = B.k[0] < P.p0thr ? 0 : 1;
        L.x = 0.0; L.dy = 0; L.dz = 0;
        L.uy = (R)-1; L.uz = (R)-1;
        // the chord factor is 1 on the rod and in the cube (the slab and the
        // extruded geometry set theirs below)
        if (G == GEOM_ROD || G == GEOM_CUBE3D) L.ig = (R)1;
        if (SRC == SRC_FACE) {
            if (G == GEOM_ROD) {
                L.ux = 1; L.iux = 1;
            } else if (G == GEOM_SLAB) {
                L.ux = MM::sqrt_(unit<R>(B.k[1]));
                L.iux = MM::rcp(L.ux);
                L.ig = L.iux;
            } else {
                need_dir = true; src_dir = true;
                cos_t = MM::sqrt_(unit<R>(B.k[1]));
                turns = unit<R>(B.k[2]);
                L.dy = P.Ld * unit<double>(B.k[3]);
                if (G == GEOM_CUBE3D) L.dz = P.Ld * unit<double>(B.k[4]);
            }
        } else {
            L.x = P.Ld * (double)unit<R>(B.k[1]);
            if (G == GEOM_ROD) {
                L.ux = B.k[2] < kHalfThr ? (R)1 : (R)-1;
                L.iux = L.ux;
            } else if (G == GEOM_SLAB) {
                L.ux = (R)2 * unit<R>(B.k[2]) - (R)1;
                L.iux = MM::rcp(L.ux);
                L.ig = MM::abs_(L.iux);
            } else if (G == GEOM_EXT2D) {
                L.dy = P.Ld * unit<double>(B.k[2]);
                need_dir = true;
                cos_t = (R)2 * unit<R>(B.k[3]) - (R)1;
                turns = unit<R>(B.k[4]);
            } else {
                need_dir = true;
                cos_t = (R)2 * unit<R>(B.k[2]) - (R)1;
                turns = unit<R>(B.k[3]);
                L.dy = P.Ld * unit<double>(B.k[4]);
                const Block5 B2 = philox_u23(0u, 1u, L.h, P.key_lo, P.key_hi);
                L.dz = P.Ld * unit<double>(B2.k[0]);
            }
        }
        if (SRC == SRC_FACE) {
            L.kcur = 0;      // x = 0: bin 0, offset 0
            L.fx = 0;
        } else {
            L.kcur = bin_of<R>(L.x, P.inv_dx, P.K, &L.fx);
        }
        ev = EV_SOURCE;
        if (TRACE) L.hash = fnv_event(L.hash, EV_SOURCE, L.m, P.trace_bins ? L.kcur : 0);
    } else if ((uint64_t)L.step > P.max_steps) {
        ev = EV_CAP;
        if (TRACE) L.hash = fnv_event(L.hash, EV_CAP, L.m, P.trace_bins ? L.kcur : 0);
    } else {
        // ---- flight: three distances, the smallest wins (Section 4) ----
        const int mf = L.m;
        const MatRow<R> mat = mtab[mf];
        const R lc = MM::dlog(unit<R>(B.k[0])) * mat.ds;
        const R li = MM::dlog(unit<R>(B.k[1])) * mat.dl * L.ig;
        // distance to the box: |distance to the face headed for| / |u| per
        // axis; a direction parallel to an axis gives +inf (or NaN for a
        // particle on that face), which never wins
        const double xh = L.ux > 0 ? P.Ld - L.x : L.x;
        R lb = (R)xh * MM::abs_(L.iux);
        // which face is nearest: y beats x, then z beats both (masks, not an
        // axis index: the event tests below use them directly)
        bool ny = false, nz = false;
        if (AXES >= 2) {
            const R l = (R)L.dy * L.aiuy;
            ny = l < lb;
            lb = ny ? l : lb;
        }
        if (AXES >= 3) {
            const R l = (R)L.dz * L.aiuz;
            nz = l < lb;
            lb = nz ? l : lb;
        }
        const bool bnd = (lb <= lc) && (lb <= li);
        const bool coll = !bnd && (lc <= li);
        R s = bnd ? lb : (coll ? lc : li);
        // a face already passed by rounding: cross at once. s is never NaN (a
        // NaN face distance never wins), so the FP32 clamp at 0 is an integer
        // max of the bit pattern (negative floats are negative integers)
        if (FP32) s = __int_as_float(max(__float_as_int(s), 0));
        const double sd = (double)s;
        const double xa = L.x;
        const int ka0 = L.kcur;
        const R fa = L.fx;
        if (FP32) L.x = __builtin_fma(sd, (double)L.ux, L.x);
        else L.x += s * L.ux;
        // FP32 tracking moves the FP64 positions by the exact FP64 product of
        // the FP32 flight length and direction (no rounding beyond the add):
        // lateral coordinates rounded to FP32 drifted by up to 3e-7 per
        // flight, enough to change which of a lateral face and a collision
        // comes first in about 2.6e-5 of the 98-flight histories of optically
        // thick cubes; in FP64 that is 2.4e-6
        if (AXES >= 2) L.dy = __builtin_fma(-sd, (double)MM::abs_(L.uy), L.dy);
        if (AXES >= 3) L.dz = __builtin_fma(-sd, (double)MM::abs_(L.uz), L.dz);
        // FP64 puts a leaking particle exactly on its face; in FP32 the
        // history ends there anyway and the snap would only move the last
        // track-length partial by a rounding error
        if (!FP32 && bnd && !ny && !nz) L.x = L.ux > 0 ? P.Ld : 0.0;
        // A lateral coordinate rounded past its face is harmless: the next
        // distance to that face is <= 0, so the particle reaches it at once.
        L.kcur = bin_of<R>(L.x, P.inv_dx, P.K, &L.fx);
        // ---- track-length score in difference form ----
        // A flight from bin ka up to bin kb adds its partial overlap pa to ka,
        // the full width to every bin strictly between and its partial
        // overlap pb to kb: in difference form D[ka] += pa, D[ka+1] += full -
        // pa, D[kb] += pb - full, D[kb+1] -= pb. A flight inside one bin is the
        // same update with pa = s and full = pb = 0, so every flight issues
        // the same four adds.
        if (EST == EST_TRACK) {
            L.tscore += sd;
            // s >= 0, so x moves with the sign of u_x (a move that rounds to
            // zero stays in its bin, where the orientation does not matter)
            const bool up = L.ux > 0;
            const int ka = up ? ka0 : L.kcur;
            const int kb = up ? L.kcur : ka0;
            const bool one = (ka == kb);
            if (FP32) {
                // overlaps from the in-bin positions: (1 - f) of the lower
                // end's bin and f of the upper end's, times the bin width
                // along the track. The differences are taken in FP64, where
                // they are exact for FP32 operands, so the four adds of a
                // flight cancel exactly beyond its last bin (FP32 differences
                // left a rounding residue in every bin past the track)
                const R dxw = P.dxr * MM::abs_(L.iux);
                const double pa = (double)(one ? s : ((R)1 - (up ? fa : L.fx)) * dxw);
                const double pb = one ? 0.0 : (double)((up ? L.fx : fa) * dxw);
                const double full = one ? 0.0 : (double)dxw;
                lds_add(tal + ka, pa);
                lds_add(tal + ka + 1, full - pa);
                lds_add(tal + kb, pb - full);
                lds_add(tal + kb + 1, -pb);
            } else {
                const double lo = up ? xa : L.x;
                const double hi = up ? L.x : xa;
                const double w = (double)MM::abs_(L.iux);
                const double pa = one ? sd : ((double)(ka + 1) * P.dx - lo) * w;
                const double pb = one ? 0.0 : (hi - (double)kb * P.dx) * w;
                const double full = one ? 0.0 : P.dx * w;
                lds_add(tal + ka, pa);
                lds_add(tal + ka + 1, full - pa);
                lds_add(tal + kb, pb - full);
                lds_add(tal + kb + 1, -pb);
            }
        }
        // ---- the event (Section 4), written as selects: every lane evaluates
        //      the same instructions whichever event it meets ----
        const bool leak = bnd && !ny && !nz;
        const bool refl_y = AXES >= 2 && bnd && ny && !nz;
        const bool refl_z = AXES >= 3 && bnd && nz;
        const bool intf = !bnd && !coll;
        const bool scat = coll && B.k[2] < mat.cthr;
        if (EST == EST_COLLISION) {
            if (coll) {
                lds_add(tal + L.kcur, (double)mat.isig);
                L.tscore += (double)mat.isig;
            }
        }
        int e = coll ? (scat ? EV_SCATTER : EV_ABSORB) : EV_INTERFACE;
        e = leak ? (L.ux > 0 ? EV_LEAK_XHI : EV_LEAK_XLO) : e;
        if (TRACE) {
            // the exact event enters the trace hash; without a trace only the
            // ends of a history (leaks, absorption) need telling apart
            if (AXES >= 2) e = refl_y ? (L.uy > 0 ? EV_REFL_YHI : EV_REFL_YLO) : e;
            if (AXES >= 3) e = refl_z ? (L.uz > 0 ? EV_REFL_ZHI : EV_REFL_ZLO) : e;
        }
        ev = e;
        L.m = mf ^ (int)intf;
        // a mirror reflection turns u_y (u_z) over and leaves the particle at
        // distance L from the face it now heads for
        if (AXES >= 2) {
            L.uy = refl_y ? -L.uy : L.uy;
            L.dy = refl_y ? P.Ld : L.dy;
        }
        if (AXES >= 3) {
            L.uz = refl_z ? -L.uz : L.uz;
            L.dz = refl_z ? P.Ld : L.dz;
        }
        // isotropic scattering: a new direction
        if (G == GEOM_ROD) {
            const R nu = B.k[3] < kHalfThr ? (R)1 : (R)-1;
            L.ux = scat ? nu : L.ux;
            L.iux = L.ux;
        } else if (G == GEOM_SLAB) {
            if (scat) {
                L.ux = (R)2 * unit<R>(B.k[3]) - (R)1;
                L.iux = MM::rcp(L.ux);
                L.ig = MM::abs_(L.iux);
            }
        } else {
            need_dir = scat;
            cos_t = (R)2 * unit<R>(B.k[3]) - (R)1;
            turns = unit<R>(B.k[4]);
        }
        L.n_int += (uint32_t)intf;
        L.n_scat += (uint32_t)scat;
        if (TRACE) L.hash = fnv_event(L.hash, ev, mf, P.trace_bins ? L.kcur : 0);
    }
    // ---- shared direction sampler: polar axis x for the inward cosine-law
    //      source, z for isotropic emission ----
    if (DIR3 && need_dir) {
        R sn, cs;
        MM::sincos_turns(turns, &sn, &cs);
        R st;
        if (FP32) st = MM::sqrt_(((R)1 - cos_t) * ((R)1 + cos_t));
        else st = MM::sqrt_((R)1 - cos_t * cos_t);
        const R a = st * cs, b = st * sn;
        R nx, ny, nz;
        if (src_dir) { nx = cos_t; ny = a; nz = b; }
        else { nx = a; ny = b; nz = cos_t; }
        if ((ny > 0) != (L.uy > 0)) L.dy = P.Ld - L.dy;
        L.ux = nx; L.uy = ny;
        L.iux = MM::rcp(nx);
        L.aiuy = MM::rcp(MM::abs_(ny));
        if (G == GEOM_CUBE3D) {
            if ((nz > 0) != (L.uz > 0)) L.dz = P.Ld - L.dz;
            L.aiuz = MM::rcp(MM::abs_(nz));
        }
        L.uz = nz;
        if (G == GEOM_EXT2D) L.ig = MM::rsqrt(nx * nx + ny * ny);
    }
    ++L.step;
    return ev;
}

// ---------------------------------------------------------------------------
// chunk slots
// ---------------------------------------------------------------------------
// Wave-uniform state of one chunk slot: first history, size, histories handed
// out, histories in flight, problem, open flag.
// s_waitcnt with vmcnt(0) and the other counters left at their maximum: the
// wave's vector memory operations, stores and atomics included, are complete.
constexpr int kWaitVmcnt0 = 0x0F70;

// (h0, cnt, next: the chunk being handed out; live: the slot's histories in
// flight; the histories of the slot's batch so far are an LDS word, W_TOTAL)
struct SlotState {
    uint64_t h0;
    uint32_t cnt, next, live;
    int32_t pid, open;
};

// ---------------------------------------------------------------------------
// finalize: means and one-sigma errors per source history
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mean_sigma(double sum, double sq, double n, double *mean, double *sig)
{
    const double mu = n > 0.0 ? sum / n : 0.0;
    double var = n > 1.0 ? (sq / n - mu * mu) * n / (n - 1.0) : 0.0;
    var = var > 0.0 ? var : 0.0;
    *mean = mu;
    *sig = n > 1.0 ? sqrt(var / n) : 0.0;
}

// Loads of the problem's tallies: plain in the finalize kernel (a later kernel
// than the tracking one), from L2 (device-scope atomic loads) when a tracking
// wave finalizes after the other waves' flush atomics.
template <bool L2>
__device__ __forceinline__ uint64_t tally_u(const uint64_t *p)
{
    if (L2) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}
template <bool L2>
__device__ __forceinline__ double tally_d(const double *p)
{
    if (L2) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

// The result record of a problem from its tallies, written by threads t of
// nt: the counters, T, R, A and the total flux with their binomial or
// per-history errors, and the per-bin flux with its batch-means error.
template <bool L2, typename PR>
__device__ __forceinline__ void record_into(PR &P, uint64_t *rec, int t, int nt)
{
    const int K = P.nbins;
    const uint64_t *C = P.counters;
    const double n = (double)tally_u<L2>(C + C_HISTORIES);
    const double B = (double)tally_u<L2>(C + C_BATCHES);
    double *out = (double *)(rec + C_COUNT);
    for (int i = t; i < C_COUNT; i += nt)
        if (i != C_COLLISIONS && i != C_LATERAL) rec[i] = tally_u<L2>(C + i);
    if (t == 0) {
        // derived counts: a collision is a scatter or an absorption; a flight
        // ends in a leak, an absorption, a scatter, an interface crossing or a
        // lateral mirror (a capped history's refused step is no flight)
        const uint64_t sc = tally_u<L2>(C + C_SCATTERS), ab = tally_u<L2>(C + C_ABSORBED);
        rec[C_COLLISIONS] = sc + ab;
        rec[C_LATERAL] = tally_u<L2>(C + C_FLIGHTS) - (tally_u<L2>(C + C_TRANSMITTED) + tally_u<L2>(C + C_REFLECTED) +
                                                       ab + sc + tally_u<L2>(C + C_INTERFACES));
        double mu, sg;
        const double nt_ = (double)tally_u<L2>(C + C_TRANSMITTED);
        const double nr_ = (double)tally_u<L2>(C + C_REFLECTED);
        const double na_ = (double)tally_u<L2>(C + C_ABSORBED);
        mean_sigma(nt_, nt_, n, &mu, &sg);
        out[R_T] = mu; out[R_SIGMA_T] = sg;
        mean_sigma(nr_, nr_, n, &mu, &sg);
        out[R_R] = mu; out[R_SIGMA_R] = sg;
        mean_sigma(na_, na_, n, &mu, &sg);
        out[R_A] = mu; out[R_SIGMA_A] = sg;
        mean_sigma(tally_d<L2>(P.sums), tally_d<L2>(P.sums + 1), n, &mu, &sg);
        out[R_TOTAL] = mu; out[R_SIGMA_TOTAL] = sg;
    }
    // batch means: batch b holds n_b histories with bin score s_b, and m is
    // the mean per history. sum (s_b - n_b m)^2 = P - 2 m R + m^2 M has the
    // expectation sigma^2 (N - M / N) (sigma^2 the per-history variance)
    // whatever the batch sizes; every history's squared score enters it with
    // weight one, and a batch mean that drifts with the batch size enters it
    // only squared (with equal batches it is the usual (B - 1) n times the
    // variance of the batch means). The error of the mean is sqrt(sigma^2 / N).
    const double M = tally_d<L2>(P.sums + 2 + 3 * K);
    const double den = n > 0.0 ? n - M / n : 0.0;
    for (int k = t; k < K; k += nt) {
        const double S = tally_d<L2>(P.sums + 2 + k);
        const double Pk = tally_d<L2>(P.sums + 2 + K + k);
        const double Rk = tally_d<L2>(P.sums + 2 + 2 * K + k);
        const double mu = n > 0.0 ? S / n : 0.0;
        double var = (B > 1.0 && den > 0.0) ? (Pk - mu * (2.0 * Rk - mu * M)) / den : 0.0;
        var = var > 0.0 ? var : 0.0;
        out[R_HEADER + k] = mu / P.dx;
        out[R_HEADER + K + k] = (n > 0.0 && B > 1.0) ? sqrt(var / n) / P.dx : 0.0;
    }
}

// Move a lane's sums to the LDS counters of its slot (a lane that finished no
// history there holds none) and clear them.
// A lane's sums are 32-bit and cover its histories of one chunk: the host caps
// a history's flights at (2^32 - 1) / (histories per chunk), so they cannot
// wrap; the slot's counters, over a whole batch, are 64-bit.
template <typename R>
__device__ __forceinline__ void lane_to_slot(Lane<R> &L, double *wsum, uint64_t *wctr)
{
    if ((L.n_t | L.n_r | L.n_a | L.n_cap) != 0u) {
        double *ss = wsum + 2 * L.slot;
        lds_add(ss, L.ssum);
        lds_add(ss + 1, L.ssq);
        unsigned long long *c = (unsigned long long *)(wctr + L.slot * kSlotCounters);
        atomicAdd(c + W_TR, (unsigned long long)L.n_t | ((unsigned long long)L.n_r << 32));
        atomicAdd(c + W_AC, (unsigned long long)L.n_a | ((unsigned long long)L.n_cap << 32));
        atomicAdd(c + W_FLIGHTS, (unsigned long long)L.n_fl);
        atomicAdd(c + W_SCAT, (unsigned long long)L.n_scat);
        atomicAdd(c + W_INT, (unsigned long long)L.n_int);
    }
    L.ssum = 0.0;
    L.ssq = 0.0;
    L.n_t = L.n_r = L.n_a = L.n_cap = 0u;
    L.n_int = L.n_scat = L.n_fl = 0u;
}

// Move a finished batch's tallies from its LDS slot to HBM: the flux bins
// (prefix-scanned first for the difference-form track-length tally) as the
// batch sum s_b into S, s_b^2 into P and n_b s_b into R, n_b^2 into M (the
// batch of n_b histories), the history score sums and the event counters.
// Leaves the LDS slot zeroed and the slot closed.
template <int EST, bool SERVED>
__device__ __forceinline__ void flush_slot(SlotState &S, const TrackArgs &A, double *b, double *ssum, uint64_t *c,
                                           int lane)
{
    ConstProblem &P = ((ConstProblem *)A.probs)[S.pid];
    const int KK = P.nbins;
    double *Sk = P.sums + 2;
    double *Pk = P.sums + 2 + KK;
    double *Rk = P.sums + 2 + 2 * KK;
    const uint64_t total = readlane64(c[W_TOTAL], 0);
    const double nb = (double)total;
    // Track length: the four entries of each flight sum to zero, so from the
    // last nonzero entry of the difference buffer on the exact running sum is
    // zero (no track reached those bins); the accumulated entries would leave
    // a rounding residue of ~1e-17 there, so those bins are not added at all.
    int kend = KK;
    if (EST == EST_TRACK) {
        kend = 0;
        for (int base = (KK / 64) * 64; base >= 0; base -= 64) {
            const int k = base + lane;
            const uint64_t nz = ballot(k <= KK && b[k] != 0.0);
            if (nz != 0) {
                kend = base + 63 - __builtin_clzll(nz);
                break;
            }
        }
    }
    double carry = 0.0;
    for (int base = 0; base <= KK; base += 64) {
        const int k = base + lane;
        double v = (k <= KK) ? b[k] : 0.0;
        if (EST == EST_TRACK) {
            v = wave_inclusive_scan(v, lane) + carry;
            carry = __shfl(v, 63, 64);
        }
        if (k < kend && v != 0.0) atomicAdd(Sk + k, v);
        if (k <= KK) b[k] = (k < kend) ? v : 0.0;
    }
    for (int k = lane; k < kend; k += 64) {
        const double v = b[k];
        if (v != 0.0) atomicAdd(Pk + k, v * v);
    }
    for (int k = lane; k < kend; k += 64) {
        const double v = b[k];
        if (v != 0.0) atomicAdd(Rk + k, v * nb);
        b[k] = 0.0;
    }
    const double st = ssum[0];
    const double st2 = ssum[1];
    // one counter per lane: lanes 0..S_NCTR-1 move them to HBM (the first four
    // are the halves of two words)
    static_assert(S_T == 0 && S_R == 1 && S_A == 2 && S_CAP == 3 && S_FLIGHTS == W_FLIGHTS + 2 &&
                      S_SCAT == W_SCAT + 2 && S_INT == W_INT + 2 && W_TR == 0 && W_AC == 1,
                  "slot counters map onto their LDS words");
    const int w = lane < 4 ? (lane >> 1) : lane - 2;
    const uint64_t v = lane < S_NCTR ? c[w] : 0u;
    const uint64_t cv = lane < 4 ? ((lane & 1) ? (v >> 32) : (v & 0xFFFFFFFFull)) : v;
    if (lane < W_STORED) c[lane] = 0u;
    const int slot_ctr_to_global[S_NCTR] = {C_TRANSMITTED, C_REFLECTED, C_ABSORBED, C_CAPPED, C_FLIGHTS,
                                            C_SCATTERS, C_INTERFACES};
    unsigned long long *Cg = (unsigned long long *)P.counters;
    if (lane < S_NCTR && cv != 0u) atomicAdd(Cg + slot_ctr_to_global[lane], (unsigned long long)cv);
    if (lane == 0) {
        ssum[0] = 0.0;
        ssum[1] = 0.0;
        atomicAdd(Cg + C_HISTORIES, (unsigned long long)total);
        atomicAdd(Cg + C_BATCHES, 1ull);
        atomicAdd(P.sums + 0, st);
        atomicAdd(P.sums + 1, st2);
        atomicAdd(P.sums + 2 + 3 * KK, nb * nb);
    }
    S.open = 0;
    if (SERVED) {
        // A served request: its flushed chunks are counted once this wave's
        // flush atomics have been performed (waited for; they need no cache
        // write-back, being performed where every later atomic on those words
        // is). The wave that counts the last chunk, in this launch or another,
        // does so after every other chunk's atomics were performed: it tells
        // the host through the request's done word, and the host launches the
        // finalize, which reads the tallies with atomic loads.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        uint64_t done = 0;
        if (lane == 0) done = atomicAdd(Cg + C_DONE_CHUNKS, 1ull) + 1ull;
        done = readlane64(done, 0);
        if (done == P.final_chunks && lane == 0)
            __hip_atomic_store(P.done_word, P.tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ---------------------------------------------------------------------------
// served rounds: work from the host's queues
// ---------------------------------------------------------------------------
// Outcomes of a claim other than a table entry: the wave's ticket is not
// published yet, the wave received kServedLeave, or an item was refused
// (reported in the feed's error word).
constexpr int kClaimWait = -1;
constexpr int kClaimLeave = -2;
constexpr int kClaimRefused = -3;
constexpr uint64_t kNoTicket = ~0ull;

// A served wave's claim state in its LDS words: its ticket (kNoTicket when it
// holds none), the last `published` it read, the loop passes until it looks
// again and the current gap, its idle passes since the ticket was taken, and
// the device clock when it started, when its idle stretch began and the idle
// ticks so far.
enum ServedWave { SV_TICKET, SV_PUB, SV_POLL_WAIT, SV_POLL_GAP, SV_WAITED, SV_BORN, SV_IDLE_FROM, SV_IDLE_TICKS };
static_assert(SV_IDLE_TICKS < kServedWaveWords, "served wave state exceeds its LDS words");

// A wave-uniform 64-bit value from LDS (every lane reads the same word).
__device__ __forceinline__ uint64_t lds_uniform(const uint64_t *p) { return readlane64(*p, 0); }

__device__ __forceinline__ void served_report(const TrackArgs &A, int lane, uint64_t code, uint64_t item)
{
    if (lane == 0) {
        __hip_atomic_store(&A.feed->error_item, item, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&A.feed->error, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// The next chunk of a served round (see ServedFeed): its table entry and chunk
// index. Called by the whole wave; lane 0 does the queue work. The wave's
// ticket (an item index from one fetch-add on the head) is kept across calls
// until the host has published that far; `pub` caches the last `published`
// the wave read. The item is read only once `published` has been seen to
// cover it, and both live in pinned host memory read past the caches (system
// scope), so no fence is needed. The entry's record, in pinned memory too, was
// written before its first item was published and is not changed while the
// round runs.
__device__ __forceinline__ int served_claim(const TrackArgs &A, int lane, uint64_t *wsrv, uint64_t *chunk)
{
    uint64_t ticket = lds_uniform(wsrv + SV_TICKET);
    if (ticket == kNoTicket) {
        uint64_t t = 0;
        if (lane == 0) {
            t = atomicAdd((unsigned long long *)&A.served->head, 1ull);
            if ((t & 31u) == 0u)
                __hip_atomic_store(&A.feed->seen, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        ticket = readlane64(t, 0);
        if (lane == 0) wsrv[SV_TICKET] = ticket;
    }
    if (ticket >= lds_uniform(wsrv + SV_PUB)) {
        uint64_t p = 0;
        if (lane == 0) {
            p = __hip_atomic_load(&A.feed->published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            wsrv[SV_PUB] = p;
        }
        if (ticket >= readlane64(p, 0)) return kClaimWait;
    }
    uint64_t item = 0;
    if (lane == 0) {
        item = __hip_atomic_load(A.items + ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        wsrv[SV_TICKET] = kNoTicket;
    }
    item = readlane64(item, 0);
    if (item == kServedLeave) return kClaimLeave;
    // The host writes only chunks of the entry's own range; the kernel refuses
    // an entry outside the table (which it could not read), and an entry of
    // an unknown kind ends its histories at once as capped (the loop of
    // kKindUnknown) instead of leaving its lanes stepping for ever.
    const uint64_t ent = item >> 32;
    if (ent >= (uint64_t)A.nprobs) {
        served_report(A, lane, kServedErrBadItem, item);
        return kClaimRefused;
    }
    *chunk = item & 0xFFFFFFFFull;
    return (int)ent;
}

// ---------------------------------------------------------------------------
// batch launches: one work queue per problem
// ---------------------------------------------------------------------------
// A problem's chunks are handed out by a counter of its own (C_QUEUE_HEAD), and
// a wave takes chunks of one problem for as long as that problem has any, so
// that the chunks it takes can join one error batch. A wave starts on the
// problem that holds its share of the launch (wave w of W: chunk w * total / W
// in the problems' order). Once its problem has none left it goes through the
// other problems in order, once: a problem whose counter was read at or beyond
// its chunk count (counters only grow), or whose fetch-add returned such a
// value, has none left, so every wave leaves after at most one pass.
constexpr uint64_t kNoChunk = ~0ull;

__device__ __forceinline__ uint64_t queue_fetch(const TrackArgs &A, int q, int lane)
{
    uint64_t got = 0;
    if (lane == 0) got = atomicAdd((unsigned long long *)(A.probs[q].counters + C_QUEUE_HEAD), 1ull);
    return readlane64(got, 0);
}

// The next chunk for a wave whose problem is *hp: its index among the chunks
// of problem *hp (updated), or kNoChunk when no problem has any left.
__device__ __forceinline__ uint64_t batch_claim(const TrackArgs &A, int lane, int *hp)
{
    const uint64_t *starts = A.item_start;
    const int n = A.nprobs;
    const int p = *hp;
    uint64_t got = queue_fetch(A, p, lane);
    if (got < starts[p + 1] - starts[p]) return ((ConstProblem *)A.probs)[p].chunk_base + got;
    // the others, 64 at a time: each lane reads one counter
    for (int base = 1; base < n; base += 64) {
        const int off = base + lane;
        int q = p + off;
        if (q >= n) q -= n;
        bool left = false;
        if (off < n) {
            const uint64_t head =
                __hip_atomic_load(A.probs[q].counters + C_QUEUE_HEAD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            left = head < starts[q + 1] - starts[q];
        }
        uint64_t m = ballot(left);
        while (m != 0) {
            int r = p + base + __builtin_ctzll(m);
            if (r >= n) r -= n;
            m &= m - 1;
            got = queue_fetch(A, r, lane);
            if (got < starts[r + 1] - starts[r]) {
                *hp = r;
                return ((ConstProblem *)A.probs)[r].chunk_base + got;
            }
        }
    }
    return kNoChunk;
}

// The flush of a slot: with the estimator of the kernel, or (served rounds)
// of the slot's problem.
template <int EST, bool SERVED>
__device__ __forceinline__ void flush_any(SlotState &S, const TrackArgs &A, double *b, double *ssum, uint64_t *c,
                                          int lane)
{
    if constexpr (EST >= 0) {
        flush_slot<EST, SERVED>(S, A, b, ssum, c, lane);
    } else {
        const int est = (((ConstProblem *)A.probs)[S.pid].kind >> 2) & 1;
        if (est == EST_TRACK) flush_slot<EST_TRACK, SERVED>(S, A, b, ssum, c, lane);
        else flush_slot<EST_COLLISION, SERVED>(S, A, b, ssum, c, lane);
    }
}

// ---------------------------------------------------------------------------
// the tracking kernel
// ---------------------------------------------------------------------------
// One event step of a lane with the loop's kind of problem; the loop for
// kinds outside [0, kKinds) ends the history at once as capped, with no flight
// (step 2: the capped-history accounting counts step - 2 flights).
template <int G, int EST, int SRC, bool FP32, bool TRACE, typename R>
__device__ __forceinline__ int lane_step(Lane<R> &L, const Prm<R> &P, double *tal, const MatRow<R> *mtab)
{
    if constexpr (G >= 0) {
        return event_step<G, EST, SRC, FP32, TRACE, R>(L, P, tal, mtab);
    } else {
        L.step = 2u;
        return EV_CAP;
    }
}

// A wave's LDS area: one or two tally buffers of KP doubles, then the score
// sum and score square sum of each slot, then kSlotCounters 64-bit counter
// words per slot, then the material rows of each slot, then (served rounds)
// the wave's claim state.
__device__ __forceinline__ double *wave_lds(const TrackArgs &A, int wid)
{
    extern __shared__ double lds[];
    return lds + (size_t)wid * ((size_t)A.slots * (size_t)A.lds_stride + kWaveExtraDoubles);
}
__device__ __forceinline__ double *wave_sums(const TrackArgs &A, double *wbuf) { return wbuf + A.slots * A.lds_stride; }
__device__ __forceinline__ uint64_t *wave_ctrs(const TrackArgs &A, double *wbuf)
{
    return (uint64_t *)(wave_sums(A, wbuf) + 4);                       // [slot][kSlotCounters]
}
__device__ __forceinline__ uint64_t *wave_served(const TrackArgs &A, double *wbuf)
{
    return (uint64_t *)(wave_sums(A, wbuf) + 4 + 2 * kSlotCounters + kMatTableDoubles);
}

// Kinds of problem a served round's kernel has a tracking loop for (every
// geometry, estimator and source); another value ends its histories at once.
constexpr int kKinds = 16;
constexpr int kKindUnknown = -2;   // the G of the loop for kinds outside [0, kKinds)
static_assert(problem_kind(GEOM_CUBE3D, EST_TRACK, SRC_VOLUME) == kKinds - 1, "kinds are 0 .. kKinds - 1");

// The tracking loop of a wave. A batch launch runs it once for the launch's
// kind of problem. A served round runs the loop of the kind of the chunk it
// holds: when the wave takes a chunk of another kind, the chunk waits in the
// wave's W_PEND word, the loop runs its histories out and returns true, and the
// round's kernel enters the loop of that kind (returns false once the wave
// leaves the round). Every kind has its own loop, so each is compiled and
// register-allocated for its geometry, estimator and source alone.
template <int G, int EST, int SRC, bool FP32, bool TRACE, bool SERVED>
__device__ __forceinline__ bool track_loop(const TrackArgs &A)
{
    using R = typename std::conditional<FP32, float, double>::type;

    const int lane = (int)(threadIdx.x & 63u);
    const int wid = (int)(threadIdx.x >> 6);
    const int KP = A.lds_stride;
    const int nslots = A.slots;
    double *const wbuf = wave_lds(A, wid);
    double *const wsum = wave_sums(A, wbuf);
    uint64_t *const wctr = wave_ctrs(A, wbuf);
    MatRow<R> *const wmat = (MatRow<R> *)(wsum + 4 + 2 * kSlotCounters);   // [slot][material]
    uint64_t *const wsrv = wave_served(A, wbuf);
    // (a served wave's area is cleared once, by its kernel: a loop starts and
    // ends with every slot flushed, which leaves the slots' words zero)
    if constexpr (!SERVED)
        for (int i = lane; i < nslots * KP + kWaveExtraDoubles; i += 64) wbuf[i] = 0.0;

    // Wave-uniform state of the two slots, kept as two named records (never
    // indexed by a run-time value, so that they stay in scalar registers): C
    // receives new histories and owns tally buffer cp, O is the other one
    // (buffer cp ^ 1) whose stragglers may still be in flight. With a single
    // buffer (large meshes) O stays closed and a new batch starts only once C
    // has been flushed.
    SlotState C = {0, 0, 0, 0, 0, 0}, O = {0, 0, 0, 0, 0, 0};
    int cp = 0;
    bool queue_empty = false;
    // batch launches: the wave's problem and a chunk of it taken but not yet
    // placed (kNoChunk: none, else it waits for a free slot), kept in the
    // wave's LDS words (touched only where chunks are taken)
    if (!SERVED) {
        const __attribute__((address_space(4))) uint64_t *starts =
            (const __attribute__((address_space(4))) uint64_t *)A.item_start;
        const uint64_t wpb = blockDim.x >> 6;
        const uint64_t w = (uint64_t)blockIdx.x * wpb + (uint64_t)__builtin_amdgcn_readfirstlane(wid);
        const uint64_t t = w * starts[A.nprobs] / ((uint64_t)gridDim.x * wpb);
        int l = 0, hi = A.nprobs;
        while (hi - l > 1) {
            const int mid = (l + hi) >> 1;
            if (starts[mid] <= t) l = mid; else hi = mid;
        }
        if (lane == 0) {
            wctr[W_HOME] = (uint64_t)l;
            wctr[W_PEND] = kNoChunk;
        }
    }
    // served rounds: the wave's claim state lives in its LDS words (wsrv,
    // ServedWave): it is touched only when the wave claims or has nothing to
    // run, and kept out of the scalar registers the tracking loop needs. While
    // the ticket is not published the wave looks again after SV_POLL_WAIT more
    // passes of this loop (the gap doubles from 1 to 32); a pass of a wave with
    // nothing to run sleeps (s_sleep 127, about 3.4 us at 2.4 GHz), and
    // SV_WAITED counts those passes since the ticket was taken. The device
    // clock is read only where an idle stretch begins and ends.
    bool idle_stretch = false;

    Lane<R> L;
    L.x = 0.0; L.dy = L.dz = L.ux = L.uy = L.uz = 0;
    L.iux = L.aiuy = L.aiuz = 0; L.ig = 1; L.fx = 0;
    L.tscore = 0.0; L.ssum = 0.0; L.ssq = 0.0; L.h = 0; L.hash = 0; L.step = 0;
    L.n_int = L.n_scat = L.n_fl = 0;
    L.n_t = L.n_r = L.n_a = L.n_cap = 0;
    L.m = 0; L.slot = 0; L.kcur = 0;
    // the lanes with a history in flight, as a wave mask (a lane reads its bit
    // with no VALU work)
    uint64_t live = 0;

    for (;;) {
        // ---------------- hand out histories to idle lanes ----------------
        // Idle lanes are refilled once at least refill_min of them wait (or the
        // whole wave is idle): fewer, fuller source steps against idle lanes.
        // At most one hand-out per step: when the current chunk runs out, a
        // new one is claimed first (if the other slot is free); idle lanes the
        // chunk cannot serve wait for the next step.
        uint64_t dead = ~live;
        if (dead != 0 && (dead == ~0ull || popc(dead) >= (uint32_t)A.refill_min)) {
            if constexpr (SERVED) {
                // a served round: every chunk is a batch of its own
                const bool slot_free = nslots == 2 ? ((!C.open || C.next == C.cnt) && !O.open) : !C.open;
                if (slot_free && !queue_empty) {
                    uint64_t chunk_index = 0;
                    int lo = kClaimWait;
                    const uint64_t pend = lds_uniform(wctr + W_PEND);
                    const uint64_t poll_wait = lds_uniform(wsrv + SV_POLL_WAIT);
                    if (pend != kNoChunk) {
                        // the chunk that made the wave enter this loop
                        lo = (int)(pend >> 32);
                        chunk_index = pend & 0xFFFFFFFFull;
                        if (lane == 0) wctr[W_PEND] = kNoChunk;
                    } else if (poll_wait == 0) {
                        lo = served_claim(A, lane, wsrv, &chunk_index);
                        const uint64_t gap = lds_uniform(wsrv + SV_POLL_GAP);
                        if (lane == 0) {
                            if (lo == kClaimWait) {
                                wsrv[SV_POLL_WAIT] = gap;
                                wsrv[SV_POLL_GAP] = gap < 32u ? gap * 2u : gap;
                            } else {
                                wsrv[SV_POLL_GAP] = 1;
                                wsrv[SV_WAITED] = 0;
                            }
                        }
                        if (lo == kClaimLeave || lo == kClaimRefused) queue_empty = true;
                    } else if (lane == 0) {
                        wsrv[SV_POLL_WAIT] = poll_wait - 1;
                    }
                    if (lo >= 0) {
                        const int kind = ((ConstProblem *)A.probs)[lo].kind;
                        const bool other = G == kKindUnknown ? (kind >= 0 && kind < kKinds)
                                                             : kind != problem_kind(G, EST, SRC);
                        // a chunk for another kind's loop waits in W_PEND, and
                        // the wave leaves this loop as if the round were over
                        // for it (written with selects: a branch here costs the
                        // loop ~27 more VGPRs)
                        if (lane == 0) wctr[W_PEND] = other ? ((uint64_t)lo << 32) | chunk_index : kNoChunk;
                        queue_empty = queue_empty || other;
                        lo = other ? kClaimWait : lo;
                    }
                    if (lo >= 0) {
                        ConstProblem &P = ((ConstProblem *)A.probs)[lo];
                        const uint64_t first = chunk_index * P.chunk;
                        const uint64_t rest = P.histories - first;
                        // the new chunk goes to the free slot, which becomes current
                        if (nslots == 2) {
                            O = C;
                            cp ^= 1;
                        }
                        C.h0 = first;
                        C.cnt = (uint32_t)(rest < P.chunk ? rest : P.chunk);
                        C.next = 0;
                        C.live = 0;
                        C.pid = lo;
                        C.open = 1;
                        if (lane == 0) wctr[cp * kSlotCounters + W_TOTAL] = C.cnt;
                        // the new slot's material rows; no lane of this wave reads
                        // them before its next event step, and a wave's LDS
                        // operations complete in order
                        if (lane < 2) wmat[2 * cp + lane] = mat_row<R>(P, lane);
                    }
                }
            } else {
                // a batch launch: the next chunk is taken once the current one
                // is handed out; it joins the batch of slot C when it is of the
                // same problem and fits, else it opens a batch in a free slot
                // (and waits while there is none)
                if (!C.open || C.next == C.cnt) {
                    uint64_t pend = lds_uniform(wctr + W_PEND);
                    int hp = (int)lds_uniform(wctr + W_HOME);
                    if (pend == kNoChunk && !queue_empty) {
                        pend = batch_claim(A, lane, &hp);
                        if (pend == kNoChunk) queue_empty = true;
                        if (lane == 0) wctr[W_HOME] = (uint64_t)hp;
                    }
                    if (pend != kNoChunk) {
                        ConstProblem &P = ((ConstProblem *)A.probs)[hp];
                        const uint64_t first = pend * P.chunk;
                        const uint64_t rest = P.histories - first;
                        const uint32_t cnt = (uint32_t)(rest < P.chunk ? rest : P.chunk);
                        uint64_t *const ctot = wctr + cp * kSlotCounters + W_TOTAL;
                        const uint64_t total = C.open ? lds_uniform(ctot) : 0;
                        if (C.open && C.pid == hp && total + cnt <= (uint64_t)P.batch_max) {
                            C.h0 = first;
                            C.cnt = cnt;
                            C.next = 0;
                            if (lane == 0) *ctot = total + cnt;
                            pend = kNoChunk;
                        } else if (!C.open || (nslots == 2 && !O.open)) {
                            if (C.open) {
                                O = C;
                                cp ^= 1;
                            }
                            C.h0 = first;
                            C.cnt = cnt;
                            C.next = 0;
                            C.live = 0;
                            C.pid = hp;
                            C.open = 1;
                            if (lane == 0) wctr[cp * kSlotCounters + W_TOTAL] = cnt;
                            if (lane < 2) wmat[2 * cp + lane] = mat_row<R>(P, lane);
                            pend = kNoChunk;
                        }
                    }
                    if (lane == 0) wctr[W_PEND] = pend;
                }
            }
            if (C.open && C.next < C.cnt) {
                const uint32_t avail = C.cnt - C.next;
                const uint32_t nd = popc(dead);
                const uint32_t take = avail < nd ? avail : nd;
                const uint32_t r = rank_in(dead);
                // the r-th idle lane takes history C.h0 + C.next + r (an
                // exec-masked block: scalar values move straight into the
                // lanes' registers, where selects would first copy them)
                const bool nw = __builtin_amdgcn_inverse_ballot_w64(dead) && r < take;
                if (nw) {
                    // sums of the lane's histories in the other slot, or of an
                    // earlier chunk of this slot's batch, go to the slot first
                    if (L.slot != cp || L.h - C.h0 >= (uint64_t)C.cnt) lane_to_slot(L, wsum, wctr);
                    L.slot = cp;
                    L.h = C.h0 + C.next + r;
                    L.step = 0u;
                    L.tscore = 0.0;
                    if (TRACE) L.hash = 0xCBF29CE484222325ull;
                }
                live |= ballot(nw);
                C.next += take;
                C.live += take;
                dead = ~live;
            }
        }

        // ---------------- exit when nothing is left --------------------------
        if (dead == ~0ull && !C.open && !O.open) {
            if (queue_empty) break;
            if (SERVED) {
                // nothing to run: the ticket is not published yet; pause
                // before looking again
                if (!idle_stretch) {
                    idle_stretch = true;
                    if (lane == 0) wsrv[SV_IDLE_FROM] = wall_clock64();
                }
                __builtin_amdgcn_s_sleep(127);
                const uint64_t waited = lds_uniform(wsrv + SV_WAITED) + 1;
                if (lane == 0) wsrv[SV_WAITED] = waited;
                if (waited > A.wait_passes) {
                    // the host never published this far: report it and leave
                    served_report(A, lane, kServedErrWait, lds_uniform(wsrv + SV_TICKET));
                    queue_empty = true;
                }
            }
        } else if (SERVED && idle_stretch) {
            idle_stretch = false;
            if (lane == 0) wsrv[SV_IDLE_TICKS] += (uint64_t)wall_clock64() - wsrv[SV_IDLE_FROM];
        }

        // ---------------- one event step per live lane -----------------------
        // A wave holds lanes of at most two problems (one per slot: a live lane
        // is in an open slot); each pass steps the lanes of one problem with
        // its parameters in scalars, both slots at once when they hold the
        // same problem.
        int ev = EV_NONE;
        uint64_t todo = live;
        const bool same = C.open && O.open && C.pid == O.pid;
        while (todo != 0) {
            const int sc = __builtin_amdgcn_readlane(L.slot, __builtin_ctzll(todo));
            const int pidc = sc == cp ? C.pid : O.pid;
            // this pass's lanes as a wave mask (a lane takes its bit of it
            // with no VALU work): the live lanes of slot sc, or of both slots
            // when they hold the same problem
            const uint64_t pass = same ? todo : todo & ballot(L.slot == sc);
            if (__builtin_amdgcn_inverse_ballot_w64(pass)) {
                ConstProblem *cprob = (ConstProblem *)A.probs;
                const Prm<R> P = load_prm<R>(cprob[pidc]);
                ev = lane_step<G, EST, SRC, FP32, TRACE, R>(L, P, wbuf + (L.slot ? KP : 0), wmat + 2 * L.slot);
            }
            todo &= ~pass;
        }

        // ---------------- histories that ended -------------------------------
        constexpr uint32_t kEnds = (1u << EV_LEAK_XLO) | (1u << EV_LEAK_XHI) | (1u << EV_ABSORB) | (1u << EV_CAP);
        const bool fin = ((kEnds >> ev) & 1u) != 0u;
        const uint64_t m_fin = ballot(fin);
        if (m_fin) {
            const uint64_t in_c = ballot(fin && L.slot == cp);
            C.live -= popc(in_c);
            O.live -= popc(m_fin & ~in_c);
            if (fin) {
                L.ssum += L.tscore;
                L.ssq = fma(L.tscore, L.tscore, L.ssq);
                L.n_t += ev == EV_LEAK_XHI ? 1u : 0u;
                L.n_r += ev == EV_LEAK_XLO ? 1u : 0u;
                L.n_a += ev == EV_ABSORB ? 1u : 0u;
                L.n_cap += ev == EV_CAP ? 1u : 0u;
                // steps = source + flights (+ the refused step of a capped history)
                L.n_fl += L.step - 1u - (ev == EV_CAP ? 1u : 0u);
                if (TRACE) {
                    const DevProblem &P = A.probs[L.slot == cp ? C.pid : O.pid];
                    if (L.h < P.trace_n) {
                        // steps = source + flights (+ the refused step of a capped history)
                        P.trace_hash[L.h] = L.hash;
                        P.trace_len[L.h] = L.step - 1u - (ev == EV_CAP ? 1u : 0u);
                    }
                }
            }
            live &= ~m_fin;

            // ------------- flush batches whose last history ended ------------
            // (every lane that ran histories of the batch is idle now and holds
            // their sums; they join the slot's counters first)
            if (C.open && C.next == C.cnt && C.live == 0) {
                if (L.slot == cp) lane_to_slot(L, wsum, wctr);
                flush_any<EST, SERVED>(C, A, wbuf + cp * KP, wsum + 2 * cp, wctr + cp * kSlotCounters, lane);
            }
            if (O.open && O.next == O.cnt && O.live == 0) {
                if (L.slot == (cp ^ 1)) lane_to_slot(L, wsum, wctr);
                flush_any<EST, SERVED>(O, A, wbuf + (cp ^ 1) * KP, wsum + 2 * (cp ^ 1), wctr + (cp ^ 1) * kSlotCounters,
                                       lane);
            }
        }
    }
    if (SERVED && idle_stretch && lane == 0) wsrv[SV_IDLE_TICKS] += (uint64_t)wall_clock64() - wsrv[SV_IDLE_FROM];
    return SERVED && lds_uniform(wctr + W_PEND) != kNoChunk;
}

// A batch launch: one kernel per kind of problem and precision.
template <int G, int EST, int SRC, bool FP32, bool TRACE>
__global__ void __launch_bounds__(512) track_kernel(TrackArgs A)
{
    track_loop<G, EST, SRC, FP32, TRACE, false>(A);
}

// A served round: every kind of problem of one precision, each in its own
// tracking loop (a wave starts in the cube's, the loop of the first chunk it
// takes if that is another kind).
template <bool FP32>
__global__ void __launch_bounds__(512) served_kernel(TrackArgs A)
{
    const int lane = (int)(threadIdx.x & 63u);
    double *const wbuf = wave_lds(A, (int)(threadIdx.x >> 6));
    uint64_t *const wctr = wave_ctrs(A, wbuf);
    uint64_t *const wsrv = wave_served(A, wbuf);
    for (int i = lane; i < A.slots * A.lds_stride + kWaveExtraDoubles; i += 64) wbuf[i] = 0.0;
    if (lane == 0) {
        wctr[W_PEND] = kNoChunk;
        wsrv[SV_TICKET] = kNoTicket;
        wsrv[SV_POLL_GAP] = 1;
        wsrv[SV_BORN] = wall_clock64();
    }
    int kind = problem_kind(GEOM_CUBE3D, EST_TRACK, SRC_FACE);
    for (;;) {
        bool more;
#define CLS_KIND_CASE(g, e, s) \
    case problem_kind(g, e, s): more = track_loop<g, e, s, FP32, false, true>(A); break;
#define CLS_KIND_CASES(g)                          \
    CLS_KIND_CASE(g, EST_COLLISION, SRC_FACE)      \
    CLS_KIND_CASE(g, EST_COLLISION, SRC_VOLUME)    \
    CLS_KIND_CASE(g, EST_TRACK, SRC_FACE)          \
    CLS_KIND_CASE(g, EST_TRACK, SRC_VOLUME)
        switch (kind) {
            CLS_KIND_CASES(GEOM_ROD)
            CLS_KIND_CASES(GEOM_SLAB)
            CLS_KIND_CASES(GEOM_EXT2D)
            CLS_KIND_CASES(GEOM_CUBE3D)
        default: more = track_loop<kKindUnknown, EST_COLLISION, SRC_FACE, FP32, false, true>(A); break;
        }
#undef CLS_KIND_CASES
#undef CLS_KIND_CASE
        if (!more) break;
        const uint64_t pend = lds_uniform(wctr + W_PEND);
        kind = ((ConstProblem *)A.probs)[pend >> 32].kind;
    }
    if (lane == 0) {
        const uint64_t now = wall_clock64();
        atomicAdd(&A.served->alive_ticks, (unsigned long long)(now - wsrv[SV_BORN]));
        atomicAdd(&A.served->idle_ticks, (unsigned long long)wsrv[SV_IDLE_TICKS]);
    }
}

// ---------------------------------------------------------------------------
// reset: zero the tallies of every problem and the work counter
// ---------------------------------------------------------------------------
__global__ void reset_kernel(const DevProblem *probs, uint64_t *queue_head)
{
    const DevProblem &P = probs[blockIdx.x];
    const int n = (int)sums_words(P.nbins);
    for (int i = threadIdx.x; i < n; i += blockDim.x) P.sums[i] = 0.0;
    for (int i = threadIdx.x; i < C_COUNT; i += blockDim.x) P.counters[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue_head = 0ull;
}

// ---------------------------------------------------------------------------
// finalize kernel: one workgroup per problem (record_into above)
// ---------------------------------------------------------------------------
__global__ void finalize_kernel(const DevProblem *probs)
{
    const DevProblem &P = probs[blockIdx.x];
    record_into<false>(P, P.record, (int)threadIdx.x, (int)blockDim.x);
}

// ---------------------------------------------------------------------------
// finalize of served requests: one wave per request; the record goes to
// P.record (the pinned host record or a device record), then the tallies are
// cleared for the next request of that memory. The records are read from
// pinned host memory.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) finalize_clear_kernel(const DevProblem *probs)
{
    // the tracking round that flushed these tallies may still be running:
    // they are read and cleared with device-scope atomic operations, which see
    // every flush atomic performed before
    const DevProblem &P = probs[blockIdx.x];
    record_into<true>(P, P.record, (int)threadIdx.x, (int)blockDim.x);
    __syncthreads();
    for (int i = threadIdx.x; i < (int)sums_words(P.nbins); i += blockDim.x)
        __hip_atomic_store(P.sums + i, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int i = threadIdx.x; i < C_COUNT; i += blockDim.x)
        __hip_atomic_store(P.counters + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_reset(const DevProblem *d_probs, int nprobs, uint64_t *queue_head,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(reset_kernel, dim3(nprobs), dim3(256), 0, stream, d_probs, queue_head);
    return hipGetLastError();
}

hipError_t launch_finalize_clear(const DevProblem *probs, int nprobs, hipStream_t stream)
{
    hipLaunchKernelGGL(finalize_clear_kernel, dim3(nprobs), dim3(64), 0, stream, probs);
    return hipGetLastError();
}

hipError_t launch_finalize(const DevProblem *d_probs, int nprobs, hipStream_t stream)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(nprobs), dim3(256), 0, stream, d_probs);
    return hipGetLastError();
}

// Kernel entry for a variant: geometry x estimator x source x precision x trace.
typedef void (*TrackFn)(TrackArgs);

template <int G, int EST, int SRC>
static TrackFn pick_prec(const Variant &v)
{
    if (v.fp32) return v.trace ? track_kernel<G, EST, SRC, true, true> : track_kernel<G, EST, SRC, true, false>;
    if (v.trace) return track_kernel<G, EST, SRC, false, true>;
    return track_kernel<G, EST, SRC, false, false>;
}

template <int G>
static TrackFn pick_geom(const Variant &v)
{
    if (v.est == EST_TRACK)
        return v.src == SRC_FACE ? pick_prec<G, EST_TRACK, SRC_FACE>(v) : pick_prec<G, EST_TRACK, SRC_VOLUME>(v);
    return v.src == SRC_FACE ? pick_prec<G, EST_COLLISION, SRC_FACE>(v) : pick_prec<G, EST_COLLISION, SRC_VOLUME>(v);
}

static TrackFn pick(const Variant &v)
{
    // served rounds: one kernel per precision for every kind of problem
    if (v.served) {
        if (v.trace || v.geom != GEOM_ANY) return nullptr;
        return v.fp32 ? served_kernel<true> : served_kernel<false>;
    }
    switch (v.geom) {
    case GEOM_ROD: return pick_geom<GEOM_ROD>(v);
    case GEOM_SLAB: return pick_geom<GEOM_SLAB>(v);
    case GEOM_EXT2D: return pick_geom<GEOM_EXT2D>(v);
    case GEOM_CUBE3D: return pick_geom<GEOM_CUBE3D>(v);
    default: return nullptr;
    }
}

// A workgroup above 64 KB of LDS (meshes beyond ~4050 bins take two-wave
// workgroups of more than that; gfx950 allows the CU's 160 KB) needs the
// kernel's attribute raised: once per kernel, to the CU's LDS, by the first
// occupancy query (before any launch, outside any graph capture) or launch.
// Smaller workgroups leave the attribute as it is.
static hipError_t allow_lds(TrackFn f, size_t lds)
{
    static std::mutex mu;
    static std::map<TrackFn, bool> raised;
    if (lds <= 65536) return hipSuccess;
    std::lock_guard<std::mutex> lk(mu);
    if (raised[f]) return hipSuccess;
    int dev = 0, lds_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (e == hipSuccess && (size_t)lds_cu < lds) e = hipErrorInvalidValue;
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize, lds_cu);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    raised[f] = true;
    return hipSuccess;
}

hipError_t track_occupancy(const Variant &v, int block, size_t lds, int *blocks_per_cu)
{
    const TrackFn f = pick(v);
    if (!f) return hipErrorInvalidValue;
    const hipError_t e = allow_lds(f, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void *>(f), block, lds);
}

hipError_t launch_track(const Variant &v, const TrackArgs &a, int grid, int block, size_t lds,
                        hipStream_t s)
{
    const TrackFn f = pick(v);
    if (!f || grid <= 0) return hipErrorInvalidValue;
    const hipError_t e = allow_lds(f, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(f, dim3(grid), dim3(block), lds, s, a);
    return hipGetLastError();
}

}  // namespace cls
