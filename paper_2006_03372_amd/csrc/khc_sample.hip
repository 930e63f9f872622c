// Sampling-based approximate (k,h)-core decomposition (gfx950): the
// paper's KHCoreSamp / UpdateHNbrSamp (Section IV-C) in level-synchronous
// form.
//
// The caller passes the vertex sample S as a mask.  Every vertex v keeps
//   d0[v]  its exact initial h-degree,
//   sel0[v] the number of sampled vertices within h hops at the start,
//   est[v] = floor(sel[v] * d0[v] / sel0[v]) (d0[v] when sel0[v] = 0),
// where sel[v] is the number of sampled vertices within h hops in the
// current graph: the paper's estimator sel / rate with the initial rate
// sel0 / d0, in integer arithmetic.  Peeling runs on est as the exact
// driver runs on the h-degree (level k = max(k, min est), remove every
// est <= k), and after each round the live vertices within h hops of the
// removed set P recount their sampled vertices with the masked multi-source
// BFS (a reached row counts only if it is sampled).  sel never grows under
// removal, so est does not either and the result does not depend on the
// removal order; the CPU oracle computes the same numbers one by one.
//
// Only part of that set can lose a sampled vertex.  A vertex x leaves the
// h-ball of u, at distance j from P, only if every path of at most h hops
// from u to x runs through P, so x lies within h - j hops of P.  If no
// sampled vertex lies within h - j hops of P, sel(u) is unchanged.  With r0
// the smallest distance from P of a sampled vertex (r0 < h), the vertices
// at distance 1 .. h - r0 are recounted and the rest keep their counts; no
// vertex is recounted when no sampled vertex lies within h - 1 hops.
#include <chrono>
#include <cstring>

#include "khc_round.h"

namespace khc {
namespace {

using namespace rnd;

__global__ void sinit_kernel(uint32_t n, uint8_t *alive, uint32_t *mark, uint32_t *core, uint32_t *s, int nscal) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        alive[v] = 1;
        mark[v] = 0;
        core[v] = 0;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < nscal; i += blockDim.x) s[i] = i == R_LIVE ? n : 0u;
}

// est of list[i] (all vertices when list is null) from its sampled count.
__global__ void sample_estimate_kernel(const uint32_t *list, uint32_t count, const uint32_t *sel,
                                       const uint32_t *sel0, const uint32_t *d0, uint32_t *est) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint32_t v = list ? list[i] : i;
        est[v] = sel0[v] ? (uint32_t)(((uint64_t)sel[v] * d0[v]) / sel0[v]) : d0[v];
    }
}

// s[R_SMIN] = min(s[R_SMIN], level) over the sampled vertices of queue levels
// 0 .. h-1 (level boundaries from the round counters).
__global__ void sample_ring_kernel(const uint32_t *queue, uint32_t *s, int h, const uint8_t *sampled) {
    uint32_t end = 0;
    for (int j = 0; j < h; ++j) end += s[R_CNT + j];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < end; i += gridDim.x * blockDim.x) {
        if (!sampled[queue[i]]) continue;
        uint32_t j = 0, at = s[R_CNT];
        while (i >= at) at += s[R_CNT + ++j];
        atomicMin(&s[R_SMIN], j);
    }
}

// Record the estimate of the vertices removed this round (queue[0, |P|)).
__global__ void record_estimate_kernel(const uint32_t *queue, const uint32_t *s, const uint32_t *est,
                                       uint32_t *out) {
    const uint32_t np = s[R_CNT];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x)
        out[queue[i]] = est[queue[i]];
}

int sgrid(khc_ctx *ctx, uint64_t count) {
    uint64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > (uint64_t)ctx->num_cu * 8) g = (uint64_t)ctx->num_cu * 8;
    return (int)g;
}

}  // namespace
}  // namespace khc

using namespace khc;

extern "C" int khcore_decompose_sampled(khc_ctx *ctx, const khc_graph *g, uint32_t h, const uint8_t *sampled,
                                        uint32_t *core, uint32_t *estimate, khc_stats *stats) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !core || !sampled) return set_error(ctx, KHC_EINVAL, "graph, sample or output is null");
    if (h == 0 || h > kMaxRoundH) return set_error(ctx, KHC_EINVAL, "h must be in 1..1024");
    if (g->ngraphs > 1) return set_error(ctx, KHC_EINVAL, "the sampling mode takes one graph");
    (void)hipSetDevice(ctx->device);
    const auto t0 = std::chrono::steady_clock::now();
    const uint32_t n = g->n;
    khc_stats sl;
    std::memset(&sl, 0, sizeof(sl));
    if (n == 0) {
        if (stats) *stats = sl;
        return KHC_OK;
    }
    hipStream_t st = ctx->stream;
    const int nscal = round_nscal(h);
    int rc;
    void *alive_v, *mark_v, *queue_v, *scal_v, *est_v, *d0_v, *sel0_v, *sel_v, *part_v, *items_v;
    if ((rc = ws_get(ctx, WS_ALIVE, (size_t)n + 8, &alive_v)) ||
        (rc = ws_get(ctx, WS_MARK, (size_t)n * 4 + 8, &mark_v)) ||
        (rc = ws_get(ctx, WS_QUEUE0, (size_t)n * 4 + 8, &queue_v)) ||
        (rc = ws_get(ctx, WS_SCRATCH, round_scalar_bytes(h), &scal_v)) ||
        (rc = ws_get(ctx, WS_DEG, (size_t)n * 4 + 8, &est_v)) ||
        (rc = ws_get(ctx, WS_DHM1, (size_t)n * 4 + 8, &d0_v)) ||
        (rc = ws_get(ctx, WS_LB, (size_t)n * 4 + 8, &sel0_v)) ||
        (rc = ws_get(ctx, WS_LBX, (size_t)n * 4 + 8, &sel_v)) ||
        (rc = ws_get(ctx, WS_MINPART, (size_t)kMinBlocks * 4, &part_v)) ||
        (rc = ws_get(ctx, WS_ITEMS, round_item_capacity(n, g->nnz) * sizeof(uint2), &items_v)))
        return rc;
    uint8_t *alive = (uint8_t *)alive_v;
    uint32_t *mark = (uint32_t *)mark_v, *queue = (uint32_t *)queue_v, *scal = (uint32_t *)scal_v;
    uint32_t *est = (uint32_t *)est_v, *d0 = (uint32_t *)d0_v, *sel0 = (uint32_t *)sel0_v, *sel = (uint32_t *)sel_v;
    unsigned long long *s64 = round_s64(scal_v, h);
    uint2 *items = (uint2 *)items_v;
    uint32_t *part = (uint32_t *)part_v;
    const RoundGraph rg = round_graph(g);
    const int gn = sgrid(ctx, n);
    const int wgrid = ctx->num_cu * 4;

    hipLaunchKernelGGL(sinit_kernel, dim3(gn), dim3(256), 0, st, n, alive, mark, core, scal, nscal);
    // exact initial degrees, then the sampled counts of every vertex with a live neighbour
    if ((rc = khdeg_compute(ctx, g, alive, h, d0))) return rc;
    fill_u32(ctx, sel0, 0u, n);
    uint32_t *srcs, nsrc;
    if ((rc = compact_sources(ctx, g, alive, &srcs, &nsrc))) return rc;
    if ((rc = msbfs_masked_counts(ctx, g, alive, h, srcs, nsrc, sampled, sel0))) return rc;
    sl.h_recomputes += 2ull * nsrc;
    hipLaunchKernelGGL(sample_estimate_kernel, dim3(gn), dim3(256), 0, st, (const uint32_t *)nullptr, n,
                       (const uint32_t *)sel0, (const uint32_t *)sel0, (const uint32_t *)d0, est);

    uint64_t left = n;
    uint32_t r = 0;
    uint32_t *hs = ctx->host_scalars;
    auto last_report = std::chrono::steady_clock::now();
    while (left > 0) {
        if ((uint64_t)r > (uint64_t)n) return set_error(ctx, KHC_ELIMIT, "more rounds than vertices");
        hipLaunchKernelGGL(keymin_kernel, dim3(kMinBlocks), dim3(256), 0, st, n, alive, (const uint8_t *)nullptr,
                           est, (const uint32_t *)nullptr, part, scal, s64, (int)h);
        hipLaunchKernelGGL(select_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, g->row_ptr, alive,
                           (const uint8_t *)nullptr, est, part, mark, core, (uint32_t *)nullptr, r, queue, scal, s64,
                           items, (int)h);
        if (estimate)
            hipLaunchKernelGGL(record_estimate_kernel, dim3(gn), dim3(256), 0, st, (const uint32_t *)queue,
                               (const uint32_t *)scal, (const uint32_t *)est, estimate);
        for (uint32_t lev = 1; lev <= h; ++lev)
            hipLaunchKernelGGL(affected_kernel, dim3(wgrid), dim3(256), 0, st, rg, alive, mark, queue, scal, s64,
                               items, (int)lev, (int)h);
        fill_u32(ctx, scal + R_SMIN, h, 1);
        hipLaunchKernelGGL(sample_ring_kernel, dim3(gn), dim3(256), 0, st, (const uint32_t *)queue, scal, (int)h,
                           sampled);
        hipLaunchKernelGGL(kill_kernel, dim3(gn), dim3(256), 0, st, queue, scal, alive, (uint32_t *)nullptr, 0);
        hipError_t e = hipMemcpyAsync(hs, scal, (size_t)nscal * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return check_hip(ctx, e, "sampled round readback");
        const uint32_t np = hs[R_CNT];
        if (np == 0) return set_error(ctx, KHC_ELIMIT, "round removed no vertex");
        uint32_t tot = 0;
        for (uint32_t j = 0; j <= h; ++j) tot += hs[R_CNT + j];
        const uint32_t na = tot - np;
        // levels 1 .. h - r0 can lose a sampled vertex (r0 = hs[R_SMIN])
        const uint32_t r0 = hs[R_SMIN];
        uint32_t nr = 0;
        for (uint32_t j = 1; r0 < h && j <= h - r0; ++j) nr += hs[R_CNT + j];
        if (nr) {
            // recount the sampled vertices of those balls, then rescale
            if ((rc = msbfs_masked_counts(ctx, g, alive, h, queue + np, nr, sampled, sel))) return rc;
            hipLaunchKernelGGL(sample_estimate_kernel, dim3(sgrid(ctx, nr)), dim3(256), 0, st,
                               (const uint32_t *)(queue + np), nr, (const uint32_t *)sel, (const uint32_t *)sel0,
                               (const uint32_t *)d0, est);
            sl.h_recomputes += nr;
        }
        hipLaunchKernelGGL(finish_kernel, dim3(gn), dim3(256), 0, st, queue, scal, (int)h, mark, (uint8_t *)nullptr,
                           (uint8_t)0);
        sl.affected_total += na;
        left -= np;
        ++r;
        report_progress(ctx, &last_report, r, (uint64_t)n - left, hs[R_KNEW]);
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "sampled end");
    if ((e = hipGetLastError()) != hipSuccess) return check_hip(ctx, e, "sampled launch");
    sl.rounds = r;
    sl.max_level = hs[R_K];
    sl.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = sl;
    return KHC_OK;
}
