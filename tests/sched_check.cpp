// Property checks of the runtime's work-division rules (csrc/cls_sched.hpp),
// compiled with the host C++ compiler by test_host_sched.py. Prints one line
// per failed property and exits with status 1 if any failed.
#include <stdint.h>
#include <stdio.h>

#include <random>
#include <vector>

#include "cls_sched.hpp"

using namespace cls::sched;

static int failures = 0;

#define CHECK(cond, ...)                                        \
    do {                                                        \
        if (!(cond)) {                                          \
            if (failures < 20) {                                \
                printf("FAIL %s: ", #cond);                     \
                printf(__VA_ARGS__);                            \
                printf("\n");                                   \
            }                                                   \
            ++failures;                                         \
        }                                                       \
    } while (0)

static uint64_t chunks_of(uint64_t n, uint64_t c) { return (n + c - 1) / c; }

int main()
{
    std::mt19937_64 rng(20170802);
    auto log_uniform = [&](double lo, double hi) {
        std::uniform_real_distribution<double> u(std::log(lo), std::log(hi));
        return (uint64_t)std::exp(u(rng));
    };
    const uint64_t max_chunks[] = {64, 1024, 16384, 65536};
    long cases = 0;

    // a lone problem
    for (int t = 0; t < 200000; ++t) {
        const uint64_t n = std::max<uint64_t>(1, log_uniform(1, 1e10));
        const uint64_t w = log_uniform(1, 20000) + 1;
        const uint64_t mc = max_chunks[t & 3];
        const uint64_t c = chunk_size(n, w, mc);
        CHECK(c >= 1 && c <= mc, "n=%llu w=%llu mc=%llu c=%llu", (unsigned long long)n, (unsigned long long)w,
              (unsigned long long)mc, (unsigned long long)c);
        // at least one chunk per wave whenever chunks of 64 histories allow it
        if (n >= 64 * w && mc >= 64)
            CHECK(chunks_of(n, c) >= w, "n=%llu w=%llu c=%llu chunks=%llu", (unsigned long long)n,
                  (unsigned long long)w, (unsigned long long)c, (unsigned long long)chunks_of(n, c));
        // no more than ~4 chunks per wave unless the floor of 256 histories or max_chunk binds
        if (c > 256 && c < mc)
            CHECK(chunks_of(n, c) <= 4 * w, "n=%llu w=%llu c=%llu", (unsigned long long)n, (unsigned long long)w,
                  (unsigned long long)c);
        ++cases;
    }

    // a problem in a batch
    for (int t = 0; t < 200000; ++t) {
        const uint64_t n = std::max<uint64_t>(1, log_uniform(1, 1e9));
        const uint64_t others = log_uniform(1, 1e11);
        const uint64_t total = n + others;
        const uint64_t w = log_uniform(64, 20000);
        const uint64_t mc = max_chunks[t & 3];
        const uint64_t alone = chunk_size(n, w, mc);
        const uint64_t c = batch_chunk_size(n, total, w, mc);
        CHECK(c >= alone, "batch chunk %llu below the lone chunk %llu", (unsigned long long)c,
              (unsigned long long)alone);
        CHECK(c <= std::max(alone, mc), "c=%llu mc=%llu", (unsigned long long)c, (unsigned long long)mc);
        // keeps at least kMinErrorBatches chunks unless its lone chunks are already larger
        if (c > alone)
            CHECK(chunks_of(n, c) >= std::min<uint64_t>(kMinErrorBatches, n),
                  "n=%llu c=%llu chunks=%llu", (unsigned long long)n, (unsigned long long)c,
                  (unsigned long long)chunks_of(n, c));
        // grows only up to ~32 chunks per wave for the whole batch
        const uint64_t cap = (total + 32 * w - 1) / (32 * w);
        if (c > alone) CHECK(c <= cap, "c=%llu cap=%llu", (unsigned long long)c, (unsigned long long)cap);
        // the histories an error batch may gather: at least one chunk, below 2^31, and
        // few enough that the problem keeps kMinErrorBatches batches when its chunks allow
        const uint64_t b = batch_histories(n, c);
        CHECK(b >= std::min<uint64_t>(c, 1ull << 31) && b <= (1ull << 31), "n=%llu c=%llu b=%llu",
              (unsigned long long)n, (unsigned long long)c, (unsigned long long)b);
        if (n / kMinErrorBatches >= c && n / kMinErrorBatches <= (1ull << 31))
            CHECK(chunks_of(n, b) >= kMinErrorBatches, "n=%llu c=%llu b=%llu batches=%llu", (unsigned long long)n,
                  (unsigned long long)c, (unsigned long long)b, (unsigned long long)chunks_of(n, b));
        ++cases;
    }

    // a served request: a whole number of chunks per wave of the round once it
    // has a wave's share for every wave
    for (int t = 0; t < 100000; ++t) {
        const uint64_t n = std::max<uint64_t>(1, log_uniform(1, 1e10));
        const uint64_t w = log_uniform(1, 20000) + 1;
        const uint64_t mc = max_chunks[t & 3];
        const uint64_t share = log_uniform(1, 1e6) + 1;
        const uint64_t c = served_chunk_size(n, w, mc, share);
        CHECK(c >= 1 && c <= mc, "served n=%llu w=%llu mc=%llu share=%llu c=%llu", (unsigned long long)n,
              (unsigned long long)w, (unsigned long long)mc, (unsigned long long)share, (unsigned long long)c);
        const uint64_t chunks = chunks_of(n, c);
        const uint64_t g = grouped_chunk_size(n, w, mc, share);
        if (c != g) {
            // the rule applied (a wave's share of at least 64 histories for every
            // wave): the waves' last chunks end together, the chunk count filling
            // the waves' turns (ceil(chunks / w) each) to within 1 / c (the
            // rounding of the chunk), and the request keeps kMinErrorBatches chunks
            const uint64_t per = std::min(share, mc);
            CHECK(per >= 64 && n / w >= per, "served rule outside its range n=%llu w=%llu", (unsigned long long)n,
                  (unsigned long long)w);
            const uint64_t turns = (chunks + w - 1) / w;
            CHECK(chunks * c >= turns * w * (c - 1), "served n=%llu w=%llu c=%llu chunks=%llu turns=%llu",
                  (unsigned long long)n, (unsigned long long)w, (unsigned long long)c, (unsigned long long)chunks,
                  (unsigned long long)turns);
            CHECK(chunks >= std::min<uint64_t>(kMinErrorBatches, n), "served n=%llu c=%llu chunks=%llu",
                  (unsigned long long)n, (unsigned long long)c, (unsigned long long)chunks);
        }
        ++cases;
    }

    // round budget and water-filling
    for (int t = 0; t < 20000; ++t) {
        std::uniform_int_distribution<int> nreq(1, 60);
        const int m = nreq(rng);
        std::vector<RoundClaim> claims(m);
        uint64_t largest = 1;
        double all = 0.0;
        for (auto &cl : claims) {
            cl.chunk = log_uniform(1, 20000) + 1;
            cl.chunks_left = log_uniform(1, 50000) + 1;
            largest = std::max(largest, cl.chunk);
            all += (double)cl.chunk * (double)cl.chunks_left;
        }
        const uint64_t waves = log_uniform(64, 9000);
        const double budget = round_budget(3e7, waves, largest);
        CHECK(budget >= 3e7 && budget >= kRoundChunksPerWave * (double)waves * (double)largest, "budget %g", budget);
        const std::vector<uint64_t> take = water_fill(claims, budget);
        // the level lies in [h_i, h_i + chunk_i) for every request cut to more than one chunk
        double got = 0.0, level_lo = 0.0, level_hi = 1e300;
        bool any_partial = false;
        for (int i = 0; i < m; ++i) {
            CHECK(take[i] >= 1 && take[i] <= claims[i].chunks_left, "take %llu of %llu",
                  (unsigned long long)take[i], (unsigned long long)claims[i].chunks_left);
            const double h = (double)take[i] * (double)claims[i].chunk;
            got += h;
            if (take[i] < claims[i].chunks_left) {
                any_partial = true;
                if (take[i] > 1) {
                    level_lo = std::max(level_lo, h);
                    level_hi = std::min(level_hi, h + (double)claims[i].chunk);
                }
            }
        }
        if (all <= budget) {
            CHECK(!any_partial, "everything fits (%g <= %g) but a request was cut", all, budget);
        } else {
            // at most the budget plus one chunk per request (the at-least-one rule)
            CHECK(got <= budget + (double)m * (double)largest, "took %g of budget %g", got, budget);
            CHECK(got >= budget - (double)m * (double)largest, "took %g of budget %g", got, budget);
            // the requests cut to several chunks share one level
            CHECK(level_lo < level_hi, "no common level: [%g, %g)", level_lo, level_hi);
            // a request taken whole had no more left than that level
            for (int i = 0; i < m; ++i)
                if (take[i] == claims[i].chunks_left)
                    CHECK((double)claims[i].chunk * (double)claims[i].chunks_left <= level_hi,
                          "a whole request (%g) above the level (< %g)",
                          (double)claims[i].chunk * (double)claims[i].chunks_left, level_hi);
        }
        ++cases;
    }
    // calibration parts of a batch
    for (int t = 0; t < 100000; ++t) {
        const uint64_t items = log_uniform(1, 1e7);
        std::uniform_real_distribution<double> uf(-0.5, 1.5);
        const double f = uf(rng);
        const uint64_t k = part_items(items, f);
        CHECK(k >= 1 && k <= items, "items %llu f %g -> %llu", (unsigned long long)items, f, (unsigned long long)k);
        if (f >= 1.0) CHECK(k == items, "whole run cut: %llu of %llu", (unsigned long long)k, (unsigned long long)items);
        if (f > 0.0 && f < 1.0)
            CHECK((double)k >= f * (double)items && (double)(k - 1) < f * (double)items,
                  "items %llu f %g -> %llu", (unsigned long long)items, f, (unsigned long long)k);
        ++cases;
    }
    // flight cap: a chunk's flights fit a 32-bit counter, and the cap is as
    // large as that allows (never above the global cap)
    for (int t = 0; t < 100000; ++t) {
        const uint64_t c = t < 70000 ? (uint64_t)(t + 1) : log_uniform(1, 4.0e9);
        const uint64_t cap = flight_cap(c);
        CHECK(cap >= 1 && cap <= kMaxFlightsPerHistory, "chunk=%llu cap=%llu", (unsigned long long)c,
              (unsigned long long)cap);
        CHECK(c * cap <= 0xFFFFFFFFull, "chunk=%llu cap=%llu", (unsigned long long)c, (unsigned long long)cap);
        CHECK(cap == kMaxFlightsPerHistory || c * (cap + 1) > 0xFFFFFFFFull, "chunk=%llu cap=%llu",
              (unsigned long long)c, (unsigned long long)cap);
        ++cases;
    }
    printf("%s %ld cases, %d failures\n", failures ? "FAILED" : "OK", cases, failures);
    return failures ? 1 : 0;
}
