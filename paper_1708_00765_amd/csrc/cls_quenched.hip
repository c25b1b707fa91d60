// Quenched-disorder reference solutions in d = 1 (Section 3 of Larmier et al.,
// arXiv 1708.00765) on gfx950.
//
// A reference solution averages an observable over realizations of the
// stochastic medium, each one transported with its geometry frozen (Sec. 3.3).
// In d = 1 a realization of the binary Markov mixture is the Poisson process on
// the line (Sec. 3.1): points of density rho = 1/Lambda, 1/Lambda = 1/Lambda_0 +
// 1/Lambda_1, cut [0, L] into cells, each of material 0 with probability p_0 =
// Lambda_0 / (Lambda_0 + Lambda_1) (Sec. 3.2). Neighbouring cells of one
// material form one layer, so the layers alternate and only the first layer's
// material is stored.
//
// Design (MI355X, wave64):
//  * a wave claims one realization at a time from a device counter, builds its
//    layers in LDS (cell gaps and colours drawn 64 at a time, one cell per lane,
//    then summed in cell order exactly like a sequential walk from x = 0), and
//    transports the realization's N histories with one history per lane and
//    lane refill once at least kQRefillMin lanes are idle;
//  * the slab needs FP64 here: the run reproduces the FP64 oracle's streams
//    (cell i of realization k: Philox block (i, 3, k); step j of history
//    g = kN + h: block (j, 2, g)); distances are taken as products with 1 /
//    Sigma_m and 1 / mu (kept per lane, recomputed when mu changes) where the
//    oracle divides: the same values to rounding, and an event decided by
//    the last bit is rare beyond what a test could meet;
//  * flux goes to an LDS difference-form buffer (four FP64 adds per flight);
//    when the realization is done the wave turns its counts and the buffer into
//    the realization's history means and adds them and their squares to HBM
//    with FP64 atomics (ensemble mean and spread over realizations).
#include "cls_quenched.hpp"
#include "philox.hpp"

namespace cls {

typedef const __attribute__((address_space(4))) DevQuenched ConstQuenched;

__device__ __forceinline__ uint64_t q_ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t q_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ double q_wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint64_t q_wave_sum_u(uint64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double q_scan(double v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

__device__ __forceinline__ double q_readlane(double v, int j)
{
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, j);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), j);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ int q_bin(double x, double inv_dx, int K)
{
    const int k = (int)(x * inv_dx);
    return min(max(k, 0), K - 1);
}

// Track-length score of a straight flight from xa to xb with |1/mu| = w and
// length len, in difference form: the partial overlaps of the end bins and
// the full widths in between (a one-bin flight scores len).
__device__ __forceinline__ void q_track(double *tal, double xa, double xb, double w, double len, double inv_dx,
                                        double dx, int K)
{
    const bool up = xb >= xa;
    const double lo = up ? xa : xb;
    const double hi = up ? xb : xa;
    const int ka = q_bin(lo, inv_dx, K), kb = q_bin(hi, inv_dx, K);
    const bool one = ka == kb;
    const double pa = one ? len : ((double)(ka + 1) * dx - lo) * w;
    const double pb = one ? 0.0 : (hi - (double)kb * dx) * w;
    const double full = one ? 0.0 : dx * w;
    atomicAdd(tal + ka, pa);
    atomicAdd(tal + ka + 1, full - pa);
    atomicAdd(tal + kb, pb - full);
    atomicAdd(tal + kb + 1, -pb);
}

// Idle lanes a wave waits for before it hands out new histories (or the whole
// wave idle): a history's first step (the source) is a branch beside the
// flights, which a refill of a single lane runs with one lane active.
constexpr uint32_t kQRefillMin = 8;

template <bool SLAB, int SRC, int EST>
__global__ void __launch_bounds__(256) quenched_kernel(const DevQuenched *rec)
{
    ConstQuenched &P = *(ConstQuenched *)rec;
    extern __shared__ double lds[];
    const int lane = (int)(threadIdx.x & 63u);
    const int wid = (int)(threadIdx.x >> 6);
    const int K = P.nbins;
    const int cap = P.layer_cap;
    double *const bnd = lds + (size_t)wid * (size_t)P.lds_stride;   // cap + 1 layer bounds
    double *const tal = bnd + cap + 1;                                 // K + 1 difference bins
    for (int i = lane; i <= K; i += 64) tal[i] = 0.0;
    const uint32_t key_lo = (uint32_t)P.seed, key_hi = (uint32_t)(P.seed >> 32);
    const uint64_t N = P.histories;
    const double L = P.L, inv_dx = P.inv_dx, dx = P.dx;
    // 1 / Sigma_m: a collision distance is -ln U / Sigma_m, taken as a product
    const double isig0 = 1.0 / P.sigma[0], isig1 = 1.0 / P.sigma[1];

    for (;;) {
        // ---------------- claim a realization --------------------------------
        uint64_t got = 0;
        if (lane == 0) got = atomicAdd((unsigned long long *)P.queue, 1ull);
        const uint64_t k = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(got >> 32), 0) << 32) |
                           (uint64_t)__builtin_amdgcn_readlane((uint32_t)got, 0);
        if (k >= P.realizations) break;

        // ---------------- its layers (Sec. 3.1-3.2) ---------------------------
        // 64 cells per round, one per lane; the walk from x = 0 adds the gaps in
        // cell order and starts a new layer where the material changes.
        int n = 0, m0 = 0, curm = -1;
        double x = 0.0;
        bool done = false;
        for (uint32_t base = 0; !done; base += 64) {
            const Block5 B = philox_u23(base + (uint32_t)lane, 3u, k, key_lo, key_hi);
            const double gap = -log(unit<double>(B.k[0])) / P.rho;
            const int mat = unit<double>(B.k[1]) < P.p0 ? 0 : 1;
            for (int j = 0; j < 64 && !done; ++j) {
                const double gj = q_readlane(gap, j);
                const int mj = __builtin_amdgcn_readlane(mat, j);
                if (mj != curm) {
                    if (n < cap && lane == 0) bnd[n] = x;
                    if (n == 0) m0 = mj;
                    ++n;
                    curm = mj;
                }
                const double end = x + gj;
                if (end >= L) done = true;
                else x = end;
            }
        }
        if (n > cap) {
            // more layers than the LDS holds: report and skip the realization
            if (lane == 0) atomicOr(P.overflow, 1u);
            continue;
        }
        if (lane == 0) bnd[n] = L;

        // ---------------- transport its N histories (Sec. 3.3) ---------------
        bool alive = false;
        uint64_t g = 0;
        uint32_t step = 0;
        // position, direction cosine and its reciprocal (set with mu, which
        // changes only at the source and at a scattering)
        double px = 0.0, mu = 0.0, imu = 0.0;
        int layer = 0;
        double tscore = 0.0;        // track length of the lane's histories in this realization
        // the lane's counts in this realization: outcomes (at most the N
        // histories, below 2^32), scatters and layer crossings; a flight ends in
        // a crossing, a leak, a scatter or an absorption, so flights and
        // collisions follow from these
        uint32_t nT = 0, nR = 0, nA = 0, nC = 0;
        uint64_t nSc = 0, nX = 0;
        uint64_t next = 0;          // histories handed out (wave-uniform)

        for (;;) {
            uint64_t dead = q_ballot(!alive);
            if (dead != 0 && next < N && (dead == ~0ull || (uint32_t)__popcll(dead) >= kQRefillMin)) {
                const uint64_t avail = N - next;
                const uint32_t nd = (uint32_t)__popcll(dead);
                const uint32_t take = avail < nd ? (uint32_t)avail : nd;
                const uint32_t r = q_rank(dead);
                const bool nw = !alive && r < take;
                g = nw ? k * N + next + r : g;
                step = nw ? 0u : step;
                alive = alive || nw;
                next += take;
                dead = q_ballot(!alive);
            }
            if (dead == ~0ull && next >= N) break;
            if (alive) {
                const Block5 B = philox_u23(step, 2u, g, key_lo, key_hi);
                if (step == 0) {
                    // source: the d = 1 laws of suite I (x = 0, cosine law about
                    // +x; the rod enters along +x) and suite II (uniform x,
                    // isotropic)
                    if (SRC == 0) {
                        px = 0.0;
                        mu = SLAB ? sqrt(unit<double>(B.k[1])) : 1.0;
                        imu = SLAB ? 1.0 / mu : 1.0;
                        layer = 0;
                    } else {
                        px = L * unit<double>(B.k[1]);
                        mu = SLAB ? 2.0 * unit<double>(B.k[2]) - 1.0 : (unit<double>(B.k[2]) < 0.5 ? 1.0 : -1.0);
                        imu = SLAB ? 1.0 / mu : mu;
                        // the layer containing x: the last bound <= x
                        int lo = 0, hi = n;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (bnd[mid] <= px) lo = mid; else hi = mid;
                        }
                        layer = lo;
                    }
                } else if ((uint64_t)step > P.max_steps) {
                    ++nC;
                    alive = false;
                } else {
                    const int m = m0 ^ (layer & 1);
                    const double isig = m ? isig1 : isig0;
                    const double lc = -log(unit<double>(B.k[0])) * isig;
                    const double face = mu > 0.0 ? bnd[layer + 1] : bnd[layer];
                    const double lb = (face - px) * imu;
                    const double xa = px;
                    const double w = fabs(imu);
                    if (lb <= lc) {
                        // the layer's face: leak, or enter the neighbouring layer
                        px = face;
                        if (EST == 1) {
                            tscore += lb;
                            q_track(tal, xa, px, w, lb, inv_dx, dx, K);
                        }
                        if (mu > 0.0 && layer + 1 == n) { ++nT; alive = false; }
                        else if (mu < 0.0 && layer == 0) { ++nR; alive = false; }
                        else { layer += mu > 0.0 ? 1 : -1; ++nX; }
                    } else {
                        px += lc * mu;
                        if (EST == 1) {
                            tscore += lc;
                            q_track(tal, xa, px, w, lc, inv_dx, dx, K);
                        }
                        if (EST == 0) {
                            atomicAdd(tal + q_bin(px, inv_dx, K), isig);
                            tscore += isig;
                        }
                        if (unit<double>(B.k[2]) < P.c[m]) {
                            ++nSc;
                            mu = SLAB ? 2.0 * unit<double>(B.k[3]) - 1.0 : (unit<double>(B.k[3]) < 0.5 ? 1.0 : -1.0);
                            imu = SLAB ? 1.0 / mu : mu;
                        } else {
                            ++nA;
                            alive = false;
                        }
                    }
                }
                ++step;
            }
        }

        // ---------------- the realization's history means -> HBM ------------
        const double inv_n = 1.0 / (double)N;
        const double sT = (double)q_wave_sum_u(nT), sR = (double)q_wave_sum_u(nR);
        const double sA = (double)q_wave_sum_u(nA);
        const double sTot = q_wave_sum(tscore);
        const uint64_t cC = q_wave_sum_u(nC);
        const uint64_t cSc = q_wave_sum_u(nSc), cX = q_wave_sum_u(nX);
        const uint64_t cCol = cSc + (uint64_t)sA;
        const uint64_t cF = cX + (uint64_t)sT + (uint64_t)sR + cCol;
        double o = 0.0;
        if (lane == QO_T) o = sT * inv_n;
        if (lane == QO_R) o = sR * inv_n;
        if (lane == QO_A) o = sA * inv_n;
        if (lane == QO_TOTAL) o = sTot * inv_n;
        if (lane == QO_LEAK) o = 0.5 * (sT + sR) * inv_n;
        if (lane < QO_COUNT) {
            atomicAdd(P.sums + lane, o);
            atomicAdd(P.sums + QO_COUNT + lane, o * o);
        }
        if (lane == 0) {
            unsigned long long *C = (unsigned long long *)P.counters;
            atomicAdd(C + Q_REALIZATIONS, 1ull);
            atomicAdd(C + Q_HISTORIES, (unsigned long long)N);
            atomicAdd(C + Q_TRANSMITTED, (unsigned long long)sT);
            atomicAdd(C + Q_REFLECTED, (unsigned long long)sR);
            atomicAdd(C + Q_ABSORBED, (unsigned long long)sA);
            atomicAdd(C + Q_CAPPED, (unsigned long long)cC);
            atomicAdd(C + Q_FLIGHTS, (unsigned long long)cF);
            atomicAdd(C + Q_COLLISIONS, (unsigned long long)cCol);
            atomicAdd(C + Q_SCATTERS, (unsigned long long)cSc);
            atomicAdd(C + Q_CROSSINGS, (unsigned long long)cX);
            atomicAdd(C + Q_LAYERS, (unsigned long long)n);
        }
        double *Sb = P.sums + 2 * QO_COUNT;
        double *Qb = Sb + K;
        double carry = 0.0;
        for (int b0 = 0; b0 <= K; b0 += 64) {
            const int b = b0 + lane;
            double v = b <= K ? tal[b] : 0.0;
            if (EST == 1) {
                v = q_scan(v, lane) + carry;
                carry = __shfl(v, 63, 64);
            }
            if (b < K) {
                const double ob = v * inv_n;
                if (ob != 0.0) {
                    atomicAdd(Sb + b, ob);
                    atomicAdd(Qb + b, ob * ob);
                }
            }
            if (b <= K) tal[b] = 0.0;
        }
    }
}

__global__ void quenched_reset_kernel(const DevQuenched *rec, int nbins)
{
    const DevQuenched &P = *rec;
    const int n = 2 * QO_COUNT + 2 * nbins;
    for (int i = threadIdx.x; i < n; i += blockDim.x) P.sums[i] = 0.0;
    for (int i = threadIdx.x; i < Q_COUNT; i += blockDim.x) P.counters[i] = 0ull;
    if (threadIdx.x == 0) {
        *P.queue = 0ull;
        *P.overflow = 0u;
    }
}

// Ensemble mean, standard error of the mean and spread of M per-realization values.
__device__ __forceinline__ void q_ensemble(double s, double q, double M, double *mean, double *se, double *spread)
{
    const double mu = M > 0.0 ? s / M : 0.0;
    double var = M > 1.0 ? (q / M - mu * mu) * M / (M - 1.0) : 0.0;
    var = var > 0.0 ? var : 0.0;
    *mean = mu;
    *spread = sqrt(var);
    *se = M > 1.0 ? sqrt(var / M) : 0.0;
}

__global__ void quenched_finalize_kernel(const DevQuenched *rec)
{
    const DevQuenched &P = *rec;
    const int K = P.nbins;
    const double M = (double)P.counters[Q_REALIZATIONS];
    uint64_t *out = P.record;
    double *d = (double *)(out + Q_COUNT);
    for (int i = threadIdx.x; i < Q_COUNT; i += blockDim.x) out[i] = P.counters[i];
    if (threadIdx.x < QO_COUNT) {
        const int j = threadIdx.x;
        double mu, se, sp;
        q_ensemble(P.sums[j], P.sums[QO_COUNT + j], M, &mu, &se, &sp);
        d[j] = mu;
        d[QO_COUNT + j] = se;
        d[2 * QO_COUNT + j] = sp;
    }
    const double *Sb = P.sums + 2 * QO_COUNT;
    const double *Qb = Sb + K;
    double *fl = d + 3 * QO_COUNT;
    for (int b = threadIdx.x; b < K; b += blockDim.x) {
        double mu, se, sp;
        q_ensemble(Sb[b], Qb[b], M, &mu, &se, &sp);
        fl[b] = mu / P.dx;
        fl[K + b] = se / P.dx;
    }
}

typedef void (*QFn)(const DevQuenched *);

template <bool SLAB>
static QFn q_pick(const QVariant &v)
{
    if (v.src == 0) return v.est == 1 ? quenched_kernel<SLAB, 0, 1> : quenched_kernel<SLAB, 0, 0>;
    return v.est == 1 ? quenched_kernel<SLAB, 1, 1> : quenched_kernel<SLAB, 1, 0>;
}

static QFn q_pick(const QVariant &v) { return v.slab ? q_pick<true>(v) : q_pick<false>(v); }

hipError_t launch_quenched(const QVariant &v, const DevQuenched *d_rec, int grid, int block, size_t lds,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(q_pick(v), dim3(grid), dim3(block), lds, stream, d_rec);
    return hipGetLastError();
}

hipError_t launch_quenched_reset(const DevQuenched *d_rec, int nbins, hipStream_t stream)
{
    hipLaunchKernelGGL(quenched_reset_kernel, dim3(1), dim3(256), 0, stream, d_rec, nbins);
    return hipGetLastError();
}

hipError_t launch_quenched_finalize(const DevQuenched *d_rec, hipStream_t stream)
{
    hipLaunchKernelGGL(quenched_finalize_kernel, dim3(1), dim3(256), 0, stream, d_rec);
    return hipGetLastError();
}

hipError_t quenched_occupancy(const QVariant &v, int block, size_t lds, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, q_pick(v), block, lds);
}

}  // namespace cls
