// Work-division rules of the CLS runtime: how a run is cut into chunks (work
// items of consecutive histories), how many of a problem's histories one
// batch of the batch-means flux error may gather, and how a server round
// shares its budget between requests. Plain host C++ with no HIP dependency, so that the CPU tests can
// compile and check it on its own.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace cls {
namespace sched {

// Batches of the flux error a problem keeps at least, when its history count
// allows.
constexpr uint64_t kMinErrorBatches = 256;

// Flights after which a history is cut (and the run reports it), at most.
constexpr uint64_t kMaxFlightsPerHistory = 100000000;

// Flight cap of the histories of a problem cut into chunks of `chunk`
// histories: the kernels sum a chunk's event counts in 32-bit counters, so a
// chunk may hold at most 2^32 - 1 flights. The cap is the smaller of
// kMaxFlightsPerHistory and floor((2^32 - 1) / chunk): 65535 flights per
// history at the largest chunk of 65536 histories, 2.6e5 at the default 16384.
inline uint64_t flight_cap(uint64_t chunk)
{
    return std::min<uint64_t>(kMaxFlightsPerHistory, 0xFFFFFFFFull / std::max<uint64_t>(chunk, 1));
}

// Chunk of a problem of n histories that runs alone on a grid of waves_total
// waves: about four chunks per wave (at least 256 histories each), but never
// fewer chunks than waves while chunks of 64 histories allow it (then
// floor(n / waves) histories each, so that every wave gets one), at most
// max_chunk.
inline uint64_t chunk_size(uint64_t n, uint64_t waves_total, uint64_t max_chunk)
{
    uint64_t c = (n + 4 * waves_total - 1) / (4 * waves_total);
    c = std::max<uint64_t>(c, 256);
    if (n / c < waves_total) c = std::max<uint64_t>(64, n / waves_total);
    c = std::min<uint64_t>(c, max_chunk);
    return std::max<uint64_t>(c, 1);
}

// Run together with other problems, a small problem need not be cut into a
// chunk per wave (which, with fine meshes, makes the chunk flushes the
// dominant cost): its chunks grow up to `cap`, while it keeps at least
// kMinErrorBatches chunks when its history count allows; never below
// chunk_size.
inline uint64_t grouped_chunk_size(uint64_t n, uint64_t waves_total, uint64_t max_chunk, uint64_t cap)
{
    const uint64_t c = chunk_size(n, waves_total, max_chunk);
    // rounded down, so that n histories make at least kMinErrorBatches chunks
    const uint64_t c_err = std::max<uint64_t>(1, n / kMinErrorBatches);
    return std::max(c, std::min(std::min(cap, c_err), max_chunk));
}

// A served request's chunk: the rule above with chunks up to one wave's share
// of a round; a request with at least that share for every wave of the round
// is cut into a whole number of chunks per wave (the count nearest to n /
// (waves x share), more if max_chunk needs it; chunks of 64 histories or
// more, and at least kMinErrorBatches of them), so that run alone it ends on
// every wave at about the same time instead of leaving most waves idle while
// some run one chunk more.
inline uint64_t served_chunk_size(uint64_t n, uint64_t waves_total, uint64_t max_chunk, uint64_t share)
{
    const uint64_t c = grouped_chunk_size(n, waves_total, max_chunk, share);
    const uint64_t w = std::max<uint64_t>(waves_total, 1);
    const uint64_t per = std::min(share, max_chunk);
    if (per < 64 || n / w < per) return c;
    uint64_t k = (n + w * per / 2) / (w * per);                       // nearest whole number
    k = std::max<uint64_t>(k, (n + w * max_chunk - 1) / (w * max_chunk));
    k = std::max<uint64_t>(k, 1);
    const uint64_t b = std::min<uint64_t>((n + k * w - 1) / (k * w), max_chunk);
    // (the error batches: a request keeps kMinErrorBatches chunks)
    return (n + b - 1) / b >= std::min<uint64_t>(kMinErrorBatches, n) ? b : c;
}

// Histories of a problem of n histories, cut into chunks of `chunk`, that
// one error batch may gather (a wave adds the chunks it takes of the problem
// to its batch while they fit): n / kMinErrorBatches, so that the problem
// keeps at least kMinErrorBatches batches, but never less than one chunk, and
// below 2^31 (the kernel counts a batch's histories in 32 bits).
inline uint64_t batch_histories(uint64_t n, uint64_t chunk)
{
    const uint64_t b = std::max<uint64_t>(chunk, n / kMinErrorBatches);
    return std::min<uint64_t>(b, 1ull << 31);
}

// A batch whose problems hold `total` histories: chunks up to the size that
// gives the whole batch about 32 chunks per wave (the density a single large
// problem gets).
inline uint64_t batch_chunk_size(uint64_t n, uint64_t total, uint64_t waves_total, uint64_t max_chunk)
{
    return grouped_chunk_size(n, waves_total, max_chunk, (total + 32 * waves_total - 1) / (32 * waves_total));
}

// Chunks of a problem's `items` that a calibration part of a batch runs: the
// first ceil(fraction x items), at least one, all of them for fraction >= 1.
inline uint64_t part_items(uint64_t items, double fraction)
{
    if (!(fraction < 1.0)) return items;
    const double want = std::ceil(std::max(0.0, fraction) * (double)items);
    return std::min(items, std::max<uint64_t>(1, (uint64_t)want));
}

// Chunks of the largest size per wave that a server round holds at least: a
// persistent launch lasts at least as long as one wave takes for its largest
// chunk, so a round with fewer leaves most waves idle (measured on the served
// mix at saturation: 3 -> 6 gained 3% at equal latency).
constexpr double kRoundChunksPerWave = 6.0;

// Histories a server round aims at: at least round_histories and at least
// kRoundChunksPerWave of its largest chunks per wave.
inline double round_budget(double round_histories, uint64_t waves, uint64_t largest_chunk)
{
    return std::max(round_histories, kRoundChunksPerWave * (double)waves * (double)largest_chunk);
}

// A request's part of a round: its chunk size and the chunks it has left.
struct RoundClaim {
    uint64_t chunk;
    uint64_t chunks_left;   // >= 1
};

// Water-filling of a round budget (histories) over requests: a request with
// less left than an equal share of what remains takes all of it; the others
// take the equal share of the rest, rounded down to whole chunks but at
// least one. Returns the chunks each request takes, in the input order.
inline std::vector<uint64_t> water_fill(const std::vector<RoundClaim> &claims, double budget)
{
    const size_t n = claims.size();
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    auto left = [&](size_t i) { return (double)claims[i].chunks_left * (double)claims[i].chunk; };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return left(a) < left(b); });
    double rest = budget, level = 0.0;
    size_t full = 0;
    for (; full < n; ++full) {
        const double share = rest / (double)(n - full);
        if (left(order[full]) > share) {
            level = share;
            break;
        }
        rest -= left(order[full]);
    }
    std::vector<uint64_t> take(n);
    for (size_t k = 0; k < n; ++k) {
        const size_t i = order[k];
        const uint64_t rem = claims[i].chunks_left;
        take[i] = k < full ? rem
                           : std::min(rem, std::max<uint64_t>(1, (uint64_t)std::floor(level / (double)claims[i].chunk)));
    }
    return take;
}

}  // namespace sched
}  // namespace cls
