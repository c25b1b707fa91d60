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
//    of the next step, so lanes stay busy until the chunk queue is empty;
//  * every step consumes exactly one Philox block per lane (source step or
//    flight), so the random-number work never diverges;
//  * the source and the scattering direction share one direction sampler;
//  * each wave owns two LDS tally buffers ("slots"), one per work chunk in
//    flight: histories of the chunk being started go to one, stragglers of the
//    previous chunk finish in the other, and a chunk's buffer is flushed to
//    HBM with FP64 atomics once its last history ends, so a chunk is exactly
//    one batch of the batch-means flux error with no tail stall;
//  * track-length flux goes to the LDS buffer in difference form (at most four
//    LDS FP64 atomics per flight whatever the number of bins crossed); the
//    flush prefix-scans it across the wave;
//  * integer tallies are wave-level ballot counts kept in scalar registers.
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
    // -ln(u) for u in (0, 1): hardware log2 times ln 2
    static __device__ __forceinline__ float neglog(float u)
    {
        return __builtin_amdgcn_logf(u) * -0.693147180559945309f;
    }
    static __device__ __forceinline__ float sqrt_(float v) { return __builtin_amdgcn_sqrtf(v); }
    static __device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
    static __device__ __forceinline__ float rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
    // sin and cos of 2 pi u: the hardware takes its argument in turns
    static __device__ __forceinline__ void sincos_turns(float u, float *s, float *c)
    {
        *s = __builtin_amdgcn_sinf(u);
        *c = __builtin_amdgcn_cosf(u);
    }
};

template <>
struct Math<double> {
    static __device__ __forceinline__ double neglog(double u) { return -log(u); }
    static __device__ __forceinline__ double sqrt_(double v) { return sqrt(v); }
    static __device__ __forceinline__ double rcp(double v) { return 1.0 / v; }
    static __device__ __forceinline__ double rsqrt(double v) { return 1.0 / sqrt(v); }
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
enum SlotCtr : int { S_T = 0, S_R, S_A, S_CAP, S_FLIGHTS, S_COLL, S_SCAT, S_INT, S_LAT, S_NCTR };


// ---------------------------------------------------------------------------
// the tracking kernel
// ---------------------------------------------------------------------------
template <int G, int EST, int SRC, bool FP32, bool TRACE>
__global__ void __launch_bounds__(512) track_kernel(TrackArgs A)
{
    using R = typename std::conditional<FP32, float, double>::type;
    using MM = Math<R>;
    constexpr int AXES = (G == GEOM_EXT2D) ? 2 : (G == GEOM_CUBE3D ? 3 : 1);
    constexpr bool DIR3 = (G == GEOM_EXT2D || G == GEOM_CUBE3D);
    const R INF = (R)__builtin_huge_val();

    extern __shared__ double lds[];
    const int lane = (int)(threadIdx.x & 63u);
    const int wid = (int)(threadIdx.x >> 6);
    const int KP = A.lds_stride;
    double *const wbuf = lds + (size_t)wid * 2u * (size_t)KP;
    for (int i = lane; i < 2 * KP; i += 64) wbuf[i] = 0.0;

    // Wave-uniform state of the two chunk slots: first history, size,
    // histories handed out, histories in flight, problem, open flag, counters.
    uint64_t s_h0[2] = {0, 0};
    uint32_t s_cnt[2] = {0, 0}, s_next[2] = {0, 0}, s_live[2] = {0, 0};
    int32_t s_pid[2] = {0, 0}, s_open[2] = {0, 0};
    uint32_t ctr[2][S_NCTR];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < S_NCTR; ++i) ctr[s][i] = 0;
    int cur = 0;
    bool queue_empty = false;
    const uint64_t total_items = A.item_start[A.nprobs];

    // lane state
    bool alive = false;
    int slot = 0;
    uint64_t h = 0;
    uint32_t step = 0;
    int m = 0;
    double x = 0.0;
    R y = 0, z = 0, ux = 0, uy = 0, uz = 0;
    R iux = 0, iuy = 0, iuz = 0, ig = 1;   // cached 1/u components and 1/chord factor
    double tscore = 0.0;
    uint64_t hash = 0;
    // lane copy of its problem's parameters
    R sig0 = 1, sig1 = 1, isig0 = 1, isig1 = 1, c0 = 0, c1 = 0, lam0 = 1, lam1 = 1, p0 = 0;
    R Lr = 1;
    double Ld = 1.0, inv_dx = 1.0, dx = 1.0;
    int K = 1;
    uint32_t key_lo = 0, key_hi = 0;
    uint64_t trace_n = 0, max_steps = 0;
    uint64_t *trace_hash = nullptr;
    uint32_t *trace_len = nullptr;
    double acc_t[2] = {0.0, 0.0}, acc_t2[2] = {0.0, 0.0};

    auto bin_of = [&](double xx) -> int {
        int k = (int)floor(xx * inv_dx);
        k = k < 0 ? 0 : k;
        return k > K - 1 ? K - 1 : k;
    };

    for (;;) {
        // ---------------- hand out histories to idle lanes ----------------
        uint64_t dead = ballot(!alive);
        while (dead != 0) {
            if (!s_open[cur] || s_next[cur] == s_cnt[cur]) {
                const int o = cur ^ 1;
                if (s_open[o] || queue_empty) break;
                uint64_t item = 0;
                if (lane == 0) item = atomicAdd((unsigned long long *)A.queue_head, 1ull);
                item = __shfl(item, 0, 64);
                if (item >= total_items) {
                    queue_empty = true;
                    break;
                }
                int lo = 0, hi = A.nprobs;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (A.item_start[mid] <= item) lo = mid; else hi = mid;
                }
                const DevProblem &P = A.probs[lo];
                const uint64_t first = (item - A.item_start[lo]) * P.chunk;
                const uint64_t rest = P.histories - first;
                s_h0[o] = first;
                s_cnt[o] = (uint32_t)(rest < P.chunk ? rest : P.chunk);
                s_next[o] = 0;
                s_live[o] = 0;
                s_pid[o] = lo;
                s_open[o] = 1;
                if (o) {
#pragma unroll
                    for (int i = 0; i < S_NCTR; ++i) ctr[1][i] = 0;
                } else {
#pragma unroll
                    for (int i = 0; i < S_NCTR; ++i) ctr[0][i] = 0;
                }
                cur = o;
                continue;
            }
            const uint32_t avail = s_cnt[cur] - s_next[cur];
            const uint32_t nd = popc(dead);
            const uint32_t take = avail < nd ? avail : nd;
            const uint32_t r = rank_in(dead);
            if (!alive && r < take) {
                const DevProblem &P = A.probs[s_pid[cur]];
                alive = true;
                slot = cur;
                h = s_h0[cur] + s_next[cur] + r;
                step = 0;
                tscore = 0.0;
                hash = 0xCBF29CE484222325ull;
                sig0 = (R)P.sigma[0]; sig1 = (R)P.sigma[1];
                isig0 = MM::rcp(sig0); isig1 = MM::rcp(sig1);
                c0 = (R)P.c[0]; c1 = (R)P.c[1];
                lam0 = (R)P.lam[0]; lam1 = (R)P.lam[1];
                p0 = (R)P.p0;
                Ld = P.L; Lr = (R)P.L;
                inv_dx = P.inv_dx; dx = P.dx;
                K = P.nbins;
                key_lo = (uint32_t)P.seed; key_hi = (uint32_t)(P.seed >> 32);
                trace_n = P.trace_n; trace_hash = P.trace_hash; trace_len = P.trace_len;
                max_steps = P.max_steps;
            }
            s_next[cur] += take;
            s_live[cur] += take;
            dead = ballot(!alive);
        }

        // ---------------- exit when nothing is left --------------------------
        if (dead == ~0ull && queue_empty && !s_open[0] && !s_open[1]) break;

        // ---------------- one event step per live lane -----------------------
        int ev = EV_NONE;
        if (alive) {
            const Block5 B = philox_u23(step, 0u, h, key_lo, key_hi);
            bool need_dir = false;
            bool src_dir = false;
            R cos_t = 0, turns = 0;
            double xa = 0.0;
            if (step == 0) {
                // ---- source (Section 2, Sec. 4.1-4.3) ----
                m = (unit<R>(B.k[0]) < p0) ? 0 : 1;
                x = 0.0; y = 0; z = 0;
                if (SRC == SRC_FACE) {
                    if (G == GEOM_ROD) {
                        ux = 1; iux = 1;
                    } else if (G == GEOM_SLAB) {
                        ux = MM::sqrt_(unit<R>(B.k[1]));
                        iux = MM::rcp(ux);
                        ig = iux;
                    } else {
                        need_dir = true; src_dir = true;
                        cos_t = MM::sqrt_(unit<R>(B.k[1]));
                        turns = unit<R>(B.k[2]);
                        y = Lr * unit<R>(B.k[3]);
                        if (G == GEOM_CUBE3D) z = Lr * unit<R>(B.k[4]);
                    }
                } else {
                    x = Ld * (double)unit<R>(B.k[1]);
                    if (G == GEOM_ROD) {
                        ux = unit<R>(B.k[2]) < (R)0.5 ? (R)1 : (R)-1;
                        iux = ux;
                    } else if (G == GEOM_SLAB) {
                        ux = (R)2 * unit<R>(B.k[2]) - (R)1;
                        iux = MM::rcp(ux);
                        ig = iux < 0 ? -iux : iux;
                    } else if (G == GEOM_EXT2D) {
                        y = Lr * unit<R>(B.k[2]);
                        need_dir = true;
                        cos_t = (R)2 * unit<R>(B.k[3]) - (R)1;
                        turns = unit<R>(B.k[4]);
                    } else {
                        need_dir = true;
                        cos_t = (R)2 * unit<R>(B.k[2]) - (R)1;
                        turns = unit<R>(B.k[3]);
                        y = Lr * unit<R>(B.k[4]);
                        const Block5 B2 = philox_u23(0u, 1u, h, key_lo, key_hi);
                        z = Lr * unit<R>(B2.k[0]);
                    }
                }
                ev = EV_SOURCE;
                if (TRACE) hash = fnv_event(hash, EV_SOURCE, m, bin_of(x));
            } else if ((uint64_t)step > max_steps) {
                ev = EV_CAP;
                if (TRACE) hash = fnv_event(hash, EV_CAP, m, bin_of(x));
            } else {
                // ---- flight ----
                const R sig_m = m ? sig1 : sig0;
                const R isig_m = m ? isig1 : isig0;
                const R lam_m = m ? lam1 : lam0;
                const R lc = MM::neglog(unit<R>(B.k[0])) * isig_m;
                const R li = MM::neglog(unit<R>(B.k[1])) * lam_m * ig;
                // distance to the boundary; ties go to x, then y, then z
                R lb;
                int face;
                {
                    const double dxf = ux > 0 ? (Ld - x) : (0.0 - x);
                    lb = (ux == 0) ? INF : (R)dxf * iux;
                    face = ux > 0 ? 1 : 0;
                }
                if (AXES >= 2) {
                    const R d = uy > 0 ? (Lr - y) : (R)0 - y;
                    const R l = (uy == 0) ? INF : d * iuy;
                    if (l < lb) { lb = l; face = uy > 0 ? 3 : 2; }
                }
                if (AXES >= 3) {
                    const R d = uz > 0 ? (Lr - z) : (R)0 - z;
                    const R l = (uz == 0) ? INF : d * iuz;
                    if (l < lb) { lb = l; face = uz > 0 ? 5 : 4; }
                }
                const bool bnd = (lb <= lc) && (lb <= li);
                const bool coll = !bnd && (lc <= li);
                R s = bnd ? lb : (coll ? lc : li);
                if (FP32) s = s > (R)0 ? s : (R)0;   // l_b <= 0: cross at once
                xa = x;
                x += (double)(s * ux);
                if (AXES >= 2) y += s * uy;
                if (AXES >= 3) z += s * uz;
                if (bnd) {
                    const R fv = (face & 1) ? Lr : (R)0;
                    if (face < 2) x = (face & 1) ? Ld : 0.0;
                    else if (face < 4) y = fv;
                    else z = fv;
                }
                if (FP32) {
                    x = x < 0.0 ? 0.0 : (x > Ld ? Ld : x);
                    if (AXES >= 2) y = y < (R)0 ? (R)0 : (y > Lr ? Lr : y);
                    if (AXES >= 3) z = z < (R)0 ? (R)0 : (z > Lr ? Lr : z);
                }
                // ---- track-length score in difference form ----
                const double sd = (double)s;
                if (EST == EST_TRACK && sd > 0.0) {
                    double *b = wbuf + slot * KP;
                    const double lo = xa < x ? xa : x;
                    const double hi = xa < x ? x : xa;
                    const int ka = bin_of(lo);
                    const int kb = bin_of(hi);
                    tscore += sd;
                    if (ka == kb) {
                        lds_add(b + ka, sd);
                        lds_add(b + ka + 1, -sd);
                    } else {
                        const double w = (double)(iux < 0 ? -iux : iux);
                        const double pa = ((double)(ka + 1) * dx - lo) * w;
                        const double pb = (hi - (double)kb * dx) * w;
                        const double full = dx * w;
                        lds_add(b + ka, pa);
                        lds_add(b + ka + 1, full - pa);
                        lds_add(b + kb, pb - full);
                        lds_add(b + kb + 1, -pb);
                    }
                }
                const int mf = m;
                if (bnd) {
                    if (face == 0) ev = EV_LEAK_XLO;
                    else if (face == 1) ev = EV_LEAK_XHI;
                    else {
                        ev = EV_REFL_YLO + (face - 2);
                        if (face < 4) { uy = -uy; iuy = -iuy; }
                        else { uz = -uz; iuz = -iuz; }
                    }
                } else if (!coll) {
                    ev = EV_INTERFACE;
                    m = 1 - m;
                } else {
                    const int k = bin_of(x);
                    if (EST == EST_COLLISION) {
                        lds_add(wbuf + slot * KP + k, (double)isig_m);
                        tscore += (double)isig_m;
                    }
                    const R c_m = mf ? c1 : c0;
                    if (unit<R>(B.k[2]) < c_m) {
                        ev = EV_SCATTER;
                        if (G == GEOM_ROD) {
                            ux = unit<R>(B.k[3]) < (R)0.5 ? (R)1 : (R)-1;
                            iux = ux;
                        } else if (G == GEOM_SLAB) {
                            ux = (R)2 * unit<R>(B.k[3]) - (R)1;
                            iux = MM::rcp(ux);
                            ig = iux < 0 ? -iux : iux;
                        } else {
                            need_dir = true;
                            cos_t = (R)2 * unit<R>(B.k[3]) - (R)1;
                            turns = unit<R>(B.k[4]);
                        }
                    } else {
                        ev = EV_ABSORB;
                    }
                }
                (void)sig_m;
                if (TRACE) hash = fnv_event(hash, ev, mf, bin_of(x));
            }
            // ---- shared direction sampler: polar axis x for the inward
            //      cosine-law source, z for isotropic emission ----
            if (DIR3 && need_dir) {
                R sn, cs;
                MM::sincos_turns(turns, &sn, &cs);
                R st;
                if (FP32) st = MM::sqrt_(((R)1 - cos_t) * ((R)1 + cos_t));
                else st = MM::sqrt_((R)1 - cos_t * cos_t);
                const R a = st * cs, b = st * sn;
                if (src_dir) { ux = cos_t; uy = a; uz = b; }
                else { ux = a; uy = b; uz = cos_t; }
                iux = MM::rcp(ux);
                iuy = MM::rcp(uy);
                iuz = MM::rcp(uz);
                if (G == GEOM_EXT2D) ig = MM::rsqrt(ux * ux + uy * uy);
            }
            ++step;
        }

        // ---------------- wave-level tallies ---------------------------------
        const bool fin = (ev == EV_LEAK_XLO) || (ev == EV_LEAK_XHI) || (ev == EV_ABSORB) || (ev == EV_CAP);
        const uint64_t in1 = ballot(alive && slot == 1);      // lanes of slot 1 (before retiring)
        const uint64_t flights = ballot(ev != EV_NONE && ev != EV_SOURCE && ev != EV_CAP);
        const uint64_t m_int = ballot(ev == EV_INTERFACE);
        const uint64_t m_coll = ballot(ev == EV_SCATTER || ev == EV_ABSORB);
        const uint64_t m_scat = ballot(ev == EV_SCATTER);
        const uint64_t m_lat = ballot(ev >= EV_REFL_YLO && ev <= EV_REFL_ZHI);
        const uint64_t m_fin = ballot(fin);
        ctr[0][S_FLIGHTS] += popc(flights & ~in1);  ctr[1][S_FLIGHTS] += popc(flights & in1);
        ctr[0][S_INT] += popc(m_int & ~in1);        ctr[1][S_INT] += popc(m_int & in1);
        ctr[0][S_COLL] += popc(m_coll & ~in1);      ctr[1][S_COLL] += popc(m_coll & in1);
        ctr[0][S_SCAT] += popc(m_scat & ~in1);      ctr[1][S_SCAT] += popc(m_scat & in1);
        ctr[0][S_LAT] += popc(m_lat & ~in1);        ctr[1][S_LAT] += popc(m_lat & in1);
        if (m_fin) {
            const uint64_t mT = ballot(ev == EV_LEAK_XHI);
            const uint64_t mR = ballot(ev == EV_LEAK_XLO);
            const uint64_t mA = ballot(ev == EV_ABSORB);
            const uint64_t mC = ballot(ev == EV_CAP);
            ctr[0][S_T] += popc(mT & ~in1);  ctr[1][S_T] += popc(mT & in1);
            ctr[0][S_R] += popc(mR & ~in1);  ctr[1][S_R] += popc(mR & in1);
            ctr[0][S_A] += popc(mA & ~in1);  ctr[1][S_A] += popc(mA & in1);
            ctr[0][S_CAP] += popc(mC & ~in1); ctr[1][S_CAP] += popc(mC & in1);
            s_live[0] -= popc(m_fin & ~in1);
            s_live[1] -= popc(m_fin & in1);
            if (fin) {
                if (slot) { acc_t[1] += tscore; acc_t2[1] += tscore * tscore; }
                else { acc_t[0] += tscore; acc_t2[0] += tscore * tscore; }
                if (TRACE && h < trace_n) {
                    trace_hash[h] = hash;
                    trace_len[h] = step - 1u;
                }
                alive = false;
            }

            // ------------- flush chunks whose last history ended -------------
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (s_open[s] && s_next[s] == s_cnt[s] && s_live[s] == 0) {
                    const DevProblem &P = A.probs[s_pid[s]];
                    const int KK = P.nbins;
                    double *b = wbuf + s * KP;
                    double *Sk = P.sums + 2;
                    double *Qk = P.sums + 2 + KK;
                    const double inv_n = 1.0 / (double)s_cnt[s];
                    double carry = 0.0;
                    for (int base = 0; base <= KK; base += 64) {
                        const int k = base + lane;
                        double v = (k <= KK) ? b[k] : 0.0;
                        if (EST == EST_TRACK) {
                            v = wave_inclusive_scan(v, lane) + carry;
                            carry = __shfl(v, 63, 64);
                        }
                        if (k < KK && v != 0.0) {
                            atomicAdd(Sk + k, v);
                            atomicAdd(Qk + k, v * v * inv_n);
                        }
                        if (k <= KK) b[k] = 0.0;
                    }
                    const double st = wave_sum(acc_t[s]);
                    const double st2 = wave_sum(acc_t2[s]);
                    acc_t[s] = 0.0;
                    acc_t2[s] = 0.0;
                    if (lane == 0) {
                        unsigned long long *C = (unsigned long long *)P.counters;
                        atomicAdd(C + C_HISTORIES, (unsigned long long)s_cnt[s]);
                        atomicAdd(C + C_TRANSMITTED, (unsigned long long)ctr[s][S_T]);
                        atomicAdd(C + C_REFLECTED, (unsigned long long)ctr[s][S_R]);
                        atomicAdd(C + C_ABSORBED, (unsigned long long)ctr[s][S_A]);
                        atomicAdd(C + C_CAPPED, (unsigned long long)ctr[s][S_CAP]);
                        atomicAdd(C + C_FLIGHTS, (unsigned long long)ctr[s][S_FLIGHTS]);
                        atomicAdd(C + C_COLLISIONS, (unsigned long long)ctr[s][S_COLL]);
                        atomicAdd(C + C_SCATTERS, (unsigned long long)ctr[s][S_SCAT]);
                        atomicAdd(C + C_INTERFACES, (unsigned long long)ctr[s][S_INT]);
                        atomicAdd(C + C_LATERAL, (unsigned long long)ctr[s][S_LAT]);
                        atomicAdd(C + C_BATCHES, 1ull);
                        atomicAdd(P.sums + 0, st);
                        atomicAdd(P.sums + 1, st2);
                    }
                    s_open[s] = 0;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// reset: zero the tallies of every problem and the work counter
// ---------------------------------------------------------------------------
__global__ void reset_kernel(const DevProblem *probs, uint64_t *queue_head)
{
    const DevProblem &P = probs[blockIdx.x];
    const int n = 2 + 2 * P.nbins;
    for (int i = threadIdx.x; i < n; i += blockDim.x) P.sums[i] = 0.0;
    for (int i = threadIdx.x; i < C_COUNT; i += blockDim.x) P.counters[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue_head = 0ull;
}

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

__global__ void finalize_kernel(const DevProblem *probs)
{
    const DevProblem &P = probs[blockIdx.x];
    const int K = P.nbins;
    const uint64_t *C = P.counters;
    const double n = (double)C[C_HISTORIES];
    const double B = (double)C[C_BATCHES];
    uint64_t *rec = P.record;
    double *out = (double *)(rec + C_COUNT);
    for (int i = threadIdx.x; i < C_COUNT; i += blockDim.x) rec[i] = C[i];
    if (threadIdx.x == 0) {
        double mu, sg;
        mean_sigma((double)C[C_TRANSMITTED], (double)C[C_TRANSMITTED], n, &mu, &sg);
        out[R_T] = mu; out[R_SIGMA_T] = sg;
        mean_sigma((double)C[C_REFLECTED], (double)C[C_REFLECTED], n, &mu, &sg);
        out[R_R] = mu; out[R_SIGMA_R] = sg;
        mean_sigma((double)C[C_ABSORBED], (double)C[C_ABSORBED], n, &mu, &sg);
        out[R_A] = mu; out[R_SIGMA_A] = sg;
        mean_sigma(P.sums[0], P.sums[1], n, &mu, &sg);
        out[R_TOTAL] = mu; out[R_SIGMA_TOTAL] = sg;
    }
    // batch means: chunk b holds n_b histories with bin score s_b; with
    // S = sum s_b and Q = sum s_b^2 / n_b the per-history variance is
    // (Q - S^2/N) / (B - 1) and the error of the mean its square root over N.
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double S = P.sums[2 + k];
        const double Q = P.sums[2 + K + k];
        const double mu = n > 0.0 ? S / n : 0.0;
        double var = B > 1.0 ? (Q - S * mu) / (B - 1.0) : 0.0;
        var = var > 0.0 ? var : 0.0;
        out[R_HEADER + k] = mu / P.dx;
        out[R_HEADER + K + k] = (n > 0.0 && B > 1.0) ? sqrt(var / n) / P.dx : 0.0;
    }
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

hipError_t launch_finalize(const DevProblem *d_probs, int nprobs, hipStream_t stream)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(nprobs), dim3(256), 0, stream, d_probs);
    return hipGetLastError();
}

template <int G, int EST, int SRC, bool FP32, bool TRACE>
static hipError_t launch_one(const TrackArgs &a, int grid, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((track_kernel<G, EST, SRC, FP32, TRACE>), dim3(grid), dim3(block), lds, s, a);
    return hipGetLastError();
}

template <int G, int EST, int SRC>
static hipError_t launch_prec(const Variant &v, const TrackArgs &a, int grid, int block, size_t lds,
                              hipStream_t s)
{
    if (v.fp32) return launch_one<G, EST, SRC, true, false>(a, grid, block, lds, s);
    if (v.trace) return launch_one<G, EST, SRC, false, true>(a, grid, block, lds, s);
    return launch_one<G, EST, SRC, false, false>(a, grid, block, lds, s);
}

template <int G>
static hipError_t launch_geom(const Variant &v, const TrackArgs &a, int grid, int block, size_t lds,
                              hipStream_t s)
{
    if (v.est == EST_TRACK) {
        if (v.src == SRC_FACE) return launch_prec<G, EST_TRACK, SRC_FACE>(v, a, grid, block, lds, s);
        return launch_prec<G, EST_TRACK, SRC_VOLUME>(v, a, grid, block, lds, s);
    }
    if (v.src == SRC_FACE) return launch_prec<G, EST_COLLISION, SRC_FACE>(v, a, grid, block, lds, s);
    return launch_prec<G, EST_COLLISION, SRC_VOLUME>(v, a, grid, block, lds, s);
}

hipError_t launch_track(const Variant &v, const TrackArgs &a, int grid, int block, size_t lds,
                        hipStream_t s)
{
    switch (v.geom) {
    case GEOM_ROD: return launch_geom<GEOM_ROD>(v, a, grid, block, lds, s);
    case GEOM_SLAB: return launch_geom<GEOM_SLAB>(v, a, grid, block, lds, s);
    case GEOM_EXT2D: return launch_geom<GEOM_EXT2D>(v, a, grid, block, lds, s);
    case GEOM_CUBE3D: return launch_geom<GEOM_CUBE3D>(v, a, grid, block, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace cls
