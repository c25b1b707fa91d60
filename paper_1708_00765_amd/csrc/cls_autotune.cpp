// Launch-shape autotuner. Candidate shapes are timed on a calibration sample
// of the caller's problems run as one batched launch, in two stages: the LDS
// tally buffers per wave (one or two, or the automatic choice) with the
// workgroup size, then, for the fastest of those, the histories per chunk
// with the idle-lane refill threshold. The fastest becomes the process-wide
// launch configuration (chunk_batches, not a performance choice, stays as the
// caller set it). Results are cached in a text file (one line per key: device,
// kernel variant and flux-mesh size class, then the first five fields of
// cls_launch_config) named by the CLS_AUTOTUNE_CACHE environment variable,
// when it is set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "cls_runtime.hpp"

using namespace cls;
using namespace cls::rt;

namespace {

std::string cache_key(const Variant &v, int max_bins)
{
    int kc = 64;
    while (kc < max_bins) kc *= 2;
    char buf[128];
    std::snprintf(buf, sizeof buf, "gfx950/g%d/e%d/s%d/%s/k%d", v.geom, v.est, v.src, v.fp32 ? "fp32" : "fp64", kc);
    return buf;
}

bool cache_lookup(const std::string &key, cls_launch_config *cfg)
{
    const char *path = std::getenv("CLS_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[160];
        cls_launch_config c = {0, 0, 0, 0, 0, 0};
        // four fields (without the buffer count, read as automatic) or five
        const int got = std::sscanf(line, "%159s %d %d %d %d %d", k, &c.waves_per_block, &c.blocks_per_cu,
                                    &c.max_chunk, &c.refill_min, &c.slots);
        if (got >= 5 && key == k) {
            c.chunk_batches = cfg->chunk_batches;
            *cfg = c;       // the last line for a key wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string &key, const cls_launch_config &c)
{
    const char *path = std::getenv("CLS_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), c.waves_per_block, c.blocks_per_cu, c.max_chunk, c.refill_min,
                 c.slots);
    std::fclose(f);
}

}  // namespace

extern "C" cls_status cls_autotune(cls_problem *const *problems, const uint64_t *histories, int n,
                                   uint64_t sample_histories, cls_launch_config *best, double *best_rate)
{
    if (!histories || !best) return fail(CLS_ERR_INVALID_ARG, "NULL argument");
    uint64_t total = 0;
    const cls_status chk = check_problem_set(problems, n, histories, &total, "autotune");
    if (chk != CLS_OK) return chk;
    int max_bins = 1;
    for (int i = 0; i < n; ++i) max_bins = std::max(max_bins, problems[i]->nbins);
    const std::string key = cache_key(variant_of(problems[0]), max_bins);
    cls_launch_config saved;
    cls_status st = cls_get_launch_config(&saved);
    if (st != CLS_OK) return st;
    *best = saved;
    if (cache_lookup(key, best)) {
        if (best_rate) *best_rate = 0.0;
        return cls_set_launch_config(best);
    }
    // Calibration: a part of the real batch, the first chunks of every problem
    // cut exactly as the whole batch would be (same launch shape, chunk sizes and
    // one-or-two LDS buffer choice; a batch of scaled-down history counts has
    // smaller chunks and can favour shapes that the whole run does not). By
    // default a quarter of the work, at least 2e7 histories.
    if (sample_histories == 0) sample_histories = std::max<uint64_t>(20000000ull, total / 4);
    const double fraction = std::min(1.0, (double)sample_histories / (double)total);
    std::vector<uint64_t> seeds(n);
    for (int i = 0; i < n; ++i) seeds[i] = 0x5DEECE66Dull * (uint64_t)(i + 1);
    double best_r = -1.0;
    cls_launch_config best_c = saved;
    // one candidate: two timed runs of the calibration part, the faster kept
    auto try_cfg = [&](const cls_launch_config &cfg) -> cls_status {
        cls_status r = cls_set_launch_config(&cfg);
        if (r != CLS_OK) return r;
        double ms = 1e30;
        uint64_t processed = 0;
        for (int rep = 0; rep < 2; ++rep) {
            r = run_batch_part(problems, histories, seeds.data(), n, fraction, &processed);
            if (r != CLS_OK && r != CLS_ERR_EVENT_CAP) return r;
            cls_tallies t;
            (void)cls_read_tallies(problems[0], &t, nullptr, nullptr, 0);
            ms = std::min(ms, t.track_ms);
        }
        const double rate = (double)processed / (ms * 1e-3);
        if (rate > best_r) {
            best_r = rate;
            best_c = cfg;
        }
        return CLS_OK;
    };
    // stage 1: LDS buffers per wave x workgroup size, default chunk and refill
    const int slot_choices[] = {0, 1, 2};
    const int waves[] = {0, 2, 4, 8};
    for (int sl : slot_choices)
        for (int w : waves) {
            st = try_cfg({w, 0, 0, 0, sl, saved.chunk_batches});
            if (st != CLS_OK) {
                (void)cls_set_launch_config(&saved);
                return st;
            }
        }
    // stage 2: chunk size x refill threshold for the stage-1 winner
    const cls_launch_config shape = best_c;
    const int chunks[] = {4096, 16384, 65536};
    const int refills[] = {1, 4, 16};
    for (int c : chunks)
        for (int r : refills) {
            st = try_cfg({shape.waves_per_block, 0, c, r, shape.slots, saved.chunk_batches});
            if (st != CLS_OK) {
                (void)cls_set_launch_config(&saved);
                return st;
            }
        }
    *best = best_c;
    if (best_rate) *best_rate = best_r;
    cache_store(key, best_c);
    return cls_set_launch_config(&best_c);
}
