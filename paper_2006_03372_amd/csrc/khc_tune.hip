// Autotuner for the BFS source-block width and the wavefronts per CU of the
// decomposition drivers: times trials of every candidate (the decomposition
// cut after a few peeling rounds), keeps the candidate with the smallest
// median and remembers it for graphs of the same size class.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "khc_internal.h"

using namespace khc;

namespace {

// Smallest e with 2^e >= x.
uint64_t ceil_log2(uint64_t x) {
    uint64_t e = 0;
    while (e < 63 && (1ull << e) < x) ++e;
    return e;
}

// Size class of a tuning problem: driver, h, trial rounds, and the powers
// of two at or above the vertex and arc counts.
uint64_t tune_key(bool persistent, uint32_t h, uint32_t rounds, const khc_graph *g) {
    const uint64_t hr = std::min<uint64_t>(h, 1023), rr = std::min<uint64_t>(rounds, (1u << 20) - 1);
    return (persistent ? 1ull : 0ull) | hr << 1 | rr << 11 | ceil_log2(g->n) << 31 | ceil_log2(g->nnz) << 37;
}

}  // namespace

extern "C" int khc_autotune(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t rounds, khc_tune *out) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g) return set_error(ctx, KHC_EINVAL, "graph is null");
    if (h == 0) return set_error(ctx, KHC_EINVAL, "h must be >= 1");
    if (rounds == 0) return set_error(ctx, KHC_EINVAL, "rounds must be >= 1");
    (void)hipSetDevice(ctx->device);
    const bool persistent = ctx->driver == 1 || g->ngraphs > 1;
    khc_tune t;
    std::memset(&t, 0, sizeof(t));
    t.persistent = persistent ? 1u : 0u;
    auto apply = [&](int w, int wv) {
        if (persistent)
            ctx->persist_width = w;
        else
            ctx->max_width = w;
        ctx->waves_per_cu = wv;
    };
    if (g->n == 0) {
        t.width_words = (uint32_t)(persistent ? ctx->persist_width : ctx->max_width);
        t.waves_per_cu = (uint32_t)ctx->waves_per_cu;
        if (out) *out = t;
        return KHC_OK;
    }
    const uint64_t key = tune_key(persistent, h, rounds, g);
    if (ctx->tune_cache_on) {
        const auto it = ctx->tune_cache.find(key);
        if (it != ctx->tune_cache.end()) {
            apply(it->second.first, it->second.second);
            t.width_words = (uint32_t)it->second.first;
            t.waves_per_cu = (uint32_t)it->second.second;
            t.cached = 1;
            if (out) *out = t;
            return KHC_OK;
        }
    }
    uint32_t *core = nullptr;
    if (hipMalloc(&core, (size_t)g->n * 4) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, KHC_ENOMEM, "autotune output allocation failed");
    }
    const int widths[3] = {32, 16, 8};  // widest first: the workspace grows once
    const int waves[3] = {16, 8, 4};
    const int reps = ctx->tune_repeats;
    t.repeats = (uint32_t)reps;
    const uint32_t saved_limit = ctx->round_limit;
    const int saved_w = ctx->max_width, saved_pw = ctx->persist_width, saved_waves = ctx->waves_per_cu;
    ctx->round_limit = rounds;
    int rc = KHC_OK;
    double best = 0.0;
    int best_w = 0, best_wv = 0;
    // warm-up: workspace at the widest width, code paths loaded
    apply(widths[0], waves[0]);
    rc = khcore_decompose(ctx, g, h, core, nullptr, nullptr);
    std::vector<double> ms(reps);
    for (int i = 0; i < 3 && rc == KHC_OK; ++i) {
        for (int j = 0; j < 3 && rc == KHC_OK; ++j) {
            apply(widths[i], waves[j]);
            for (int k = 0; k < reps && rc == KHC_OK; ++k) {
                const auto t0 = std::chrono::steady_clock::now();
                rc = khcore_decompose(ctx, g, h, core, nullptr, nullptr);
                ms[k] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            }
            if (rc != KHC_OK) break;
            std::sort(ms.begin(), ms.end());
            const double med = (reps & 1) ? ms[reps / 2] : 0.5 * (ms[reps / 2 - 1] + ms[reps / 2]);
            const uint32_t c = t.candidates++;
            t.cand_width[c] = (uint32_t)widths[i];
            t.cand_waves[c] = (uint32_t)waves[j];
            t.trial_ms[c] = med;
            if (best_w == 0 || med < best) {
                best = med;
                best_w = widths[i];
                best_wv = waves[j];
            }
        }
    }
    ctx->round_limit = saved_limit;
    (void)hipFree(core);
    ctx->max_width = saved_w;
    ctx->persist_width = saved_pw;
    ctx->waves_per_cu = saved_waves;
    if (rc != KHC_OK) return rc;
    apply(best_w, best_wv);
    if (ctx->tune_cache_on) ctx->tune_cache[key] = {best_w, best_wv};
    t.width_words = (uint32_t)best_w;
    t.waves_per_cu = (uint32_t)best_wv;
    if (out) *out = t;
    return KHC_OK;
}
