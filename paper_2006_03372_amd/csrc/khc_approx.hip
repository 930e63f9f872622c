// Learned approximate (k,h)-core decomposition (gfx950).
//
// The peeling loop is the level-synchronous one of the exact driver, but a
// vertex's h-degree is never recomputed: its estimate comes from the MLP of
// khc_mlp.hip applied to eight cheap features built from exact j-hop
// degrees for j < h, which are maintained exactly (they change only within
// h-1 hops of the removed set).  The paper's own approximate variant
// estimates updated h-degrees from a vertex sample (Section IV-C); this
// mode stands beside it, and its error is measured against the exact
// peeling.
//
// Features of a live vertex v (all log1p of exact counts in the current
// graph, divided by kFeatScale), with a = max(1, h-3), b = max(1, h-2):
//   d^a(v), d^b(v), d^{h-1}(v),
//   min, mean, max over live neighbours w of d^{h-1}(w),
//   mean over live neighbours of d^a(w), mean over live neighbours of d^b(w).
// The network predicts y ~ log1p(d^h(v)) / kFeatScale.  The estimate is
//   clamp(round(expm1(kFeatScale * y)), LB, UB), then min with the previous
// estimate (h-degrees never grow under removal), where for h >= 2
//   LB = max(d^{h-1}(v), max_w d^{h-1}(w))       (a neighbour's closed
//        (h-1)-ball lies in v's h-ball)
//   UB = min(live - 1, sum_w d^{h-1}(w))          (v's h-ball is the union of
//        its neighbours' closed (h-1)-balls minus v)
// are exact bounds.  Without a network the estimate is LB (the ablation).
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "khc_round.h"

namespace khc {
float *mlp_params(khc_mlp *m);
}

extern "C" int khc_mlp_forward(khc_ctx *ctx, const khc_mlp *m, const float *X, uint32_t n, float *y);

namespace khc {
namespace {

using namespace rnd;

constexpr float kFeatScale = 8.f;
constexpr int kFeat = 8;

// Features and exact bounds of list[i] (list null: vertex i), one wavefront
// per vertex.  Row i of X; lb/ub indexed by vertex.
__global__ void features_kernel(const uint32_t *list, uint32_t count, const uint64_t *row_ptr,
                                const uint32_t *col, const uint8_t *alive, const uint32_t *da,
                                const uint32_t *db, const uint32_t *dc, const uint32_t *live_count,
                                float *X, uint32_t *lb, uint32_t *ub) {
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t i = wave; i < count; i += nwaves) {
        const uint32_t v = list ? list[i] : i;
        const bool live = !alive || alive[v];
        uint32_t mn = 0xFFFFFFFFu, mx = 0, deg = 0;
        uint64_t sa = 0, sb = 0, sc = 0;
        if (live) {
            for (uint64_t a = row_ptr[v] + lane; a < row_ptr[v + 1]; a += 64) {
                const uint32_t w = col[a];
                if (alive && !alive[w]) continue;
                const uint32_t c = dc[w];
                mn = c < mn ? c : mn;
                mx = c > mx ? c : mx;
                sa += da[w];
                sb += db[w];
                sc += c;
                deg++;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t omn = __shfl_xor(mn, off, 64), omx = __shfl_xor(mx, off, 64);
            mn = omn < mn ? omn : mn;
            mx = omx > mx ? omx : mx;
            sa += __shfl_xor(sa, off, 64);
            sb += __shfl_xor(sb, off, 64);
            sc += __shfl_xor(sc, off, 64);
            deg += __shfl_xor(deg, off, 64);
        }
        if (lane == 0) {
            float f[kFeat] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            uint32_t l = 0, u = 0;
            if (live) {
                f[0] = log1pf((float)da[v]);
                f[1] = log1pf((float)db[v]);
                f[2] = log1pf((float)dc[v]);
                if (deg) {
                    f[3] = log1pf((float)mn);
                    f[4] = log1pf((float)sc / (float)deg);
                    f[5] = log1pf((float)mx);
                    f[6] = log1pf((float)sa / (float)deg);
                    f[7] = log1pf((float)sb / (float)deg);
                }
                l = dc[v] > mx ? dc[v] : mx;
                const uint64_t cap = *live_count ? (uint64_t)*live_count - 1 : 0;
                u = (uint32_t)(sc < cap ? sc : cap);
                if (u < l) u = l;
            }
            for (int k = 0; k < kFeat; ++k) X[(size_t)i * kFeat + k] = f[k] / kFeatScale;
            if (lb) lb[v] = l;
            if (ub) ub[v] = u;
        }
    }
}

// Estimate from the network output (or LB when y is null), clamped to the
// exact bounds and never above the previous estimate.
__global__ void estimate_kernel(const uint32_t *list, uint32_t count, const float *y, const uint32_t *lb,
                                const uint32_t *ub, uint32_t *dhat, int keep_min) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint32_t v = list ? list[i] : i;
        uint32_t e = lb[v];
        if (y) {
            const float z = expm1f(kFeatScale * y[i]);
            const float rz = floorf(z + 0.5f);
            uint32_t p = rz <= 0.f ? 0u : (rz >= 4294967040.f ? 0xFFFFFF00u : (uint32_t)rz);
            e = p < lb[v] ? lb[v] : (p > ub[v] ? ub[v] : p);
        }
        if (keep_min && dhat[v] < e) e = dhat[v];
        dhat[v] = e;
    }
}

__global__ void live_count_kernel(uint32_t n, const uint8_t *alive, uint32_t *out) {
    uint32_t c = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        c += (!alive || alive[v]) ? 1u : 0u;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__global__ void ainit_kernel(uint32_t n, uint8_t *alive, uint32_t *mark, uint32_t *core, uint32_t *s, int nscal) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        alive[v] = 1;
        mark[v] = 0;
        core[v] = 0;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < nscal; i += blockDim.x) s[i] = i == R_LIVE ? n : 0u;
}

int grid_of(khc_ctx *ctx, uint64_t count, int threads) {
    uint64_t g = (count + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > (uint64_t)ctx->num_cu * 8) g = (uint64_t)ctx->num_cu * 8;
    return (int)g;
}

// j-hop degrees (j = 1..h-1) of the listed vertices into dj[0..h-2].
int hop_degrees(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, const uint32_t *srcs,
                uint32_t nsrc, uint32_t *const *dj) {
    if (nsrc == 0) return KHC_OK;
    return msbfs_all_levels(ctx, g, alive, h - 1, srcs, nsrc, dj);
}

}  // namespace
}  // namespace khc

using namespace khc;

extern "C" {

int khc_features(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, float *X, uint32_t *lb,
                 uint32_t *ub) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !X) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h < 2 || h > 64) return set_error(ctx, KHC_EINVAL, "features need 2 <= h <= 64");
    (void)hipSetDevice(ctx->device);
    const uint32_t n = g->n;
    if (n == 0) return KHC_OK;
    hipStream_t st = ctx->stream;
    int rc;
    void *djv, *cnt;
    if ((rc = ws_get(ctx, WS_APPROX_DJ, (size_t)(h - 1) * n * 4 + 4, &djv)) ||
        (rc = ws_get(ctx, WS_APPROX_SCAL, 64, &cnt)))
        return rc;
    uint32_t *djb = (uint32_t *)djv;
    std::vector<uint32_t *> dj(h - 1);
    for (uint32_t j = 0; j + 1 < h; ++j) dj[j] = djb + (size_t)j * n;
    fill_u32(ctx, djb, 0u, (uint64_t)(h - 1) * n);
    uint32_t *srcs, nsrc;
    if ((rc = compact_sources(ctx, g, alive, &srcs, &nsrc))) return rc;
    if ((rc = hop_degrees(ctx, g, alive, h, srcs, nsrc, dj.data()))) return rc;
    uint32_t *live = (uint32_t *)cnt;
    fill_u32(ctx, live, 0u, 1);
    hipLaunchKernelGGL(live_count_kernel, dim3(grid_of(ctx, n, 256)), dim3(256), 0, st, n, alive, live);
    const uint32_t a = h >= 4 ? h - 3 : 1, b = h >= 3 ? h - 2 : 1;
    hipLaunchKernelGGL(features_kernel, dim3(ctx->num_cu * 4), dim3(256), 0, st, (const uint32_t *)nullptr, n,
                       g->row_ptr, g->col, alive, dj[a - 1], dj[b - 1], dj[h - 2], (const uint32_t *)live, X, lb,
                       ub);
    return check_hip(ctx, hipGetLastError(), "features");
}

int khcore_decompose_approx(khc_ctx *ctx, const khc_graph *g, uint32_t h, const khc_mlp *mlp, uint32_t *core,
                            uint32_t *estimate, khc_stats *stats) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !core) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h < 2 || h > 64) return set_error(ctx, KHC_EINVAL, "the approximate mode needs 2 <= h <= 64");
    if (g->ngraphs > 1) return set_error(ctx, KHC_EINVAL, "the approximate mode takes one graph");
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
    void *alive_v, *mark_v, *queue_v, *scal_v, *dhat_v, *lb_v, *ub_v, *x_v, *y_v, *dj_v, *part_v, *items_v;
    if ((rc = ws_get(ctx, WS_ALIVE, (size_t)n + 8, &alive_v)) || (rc = ws_get(ctx, WS_MARK, (size_t)n * 4 + 8, &mark_v)) ||
        (rc = ws_get(ctx, WS_QUEUE0, (size_t)n * 4 + 8, &queue_v)) ||
        (rc = ws_get(ctx, WS_SCRATCH, round_scalar_bytes(h), &scal_v)) ||
        (rc = ws_get(ctx, WS_DEG, (size_t)n * 4 + 8, &dhat_v)) || (rc = ws_get(ctx, WS_LB, (size_t)n * 4 + 8, &lb_v)) ||
        (rc = ws_get(ctx, WS_DHM1, (size_t)n * 4 + 8, &ub_v)) ||
        (rc = ws_get(ctx, WS_APPROX_X, (size_t)n * kFeat * 4 + 32, &x_v)) ||
        (rc = ws_get(ctx, WS_APPROX_Y, (size_t)n * 4 + 8, &y_v)) ||
        (rc = ws_get(ctx, WS_APPROX_DJ, (size_t)(h - 1) * n * 4 + 4, &dj_v)) ||
        (rc = ws_get(ctx, WS_MINPART, (size_t)kMinBlocks * 4, &part_v)) ||
        (rc = ws_get(ctx, WS_ITEMS, round_item_capacity(n, g->nnz) * sizeof(uint2), &items_v)))
        return rc;
    uint8_t *alive = (uint8_t *)alive_v;
    uint32_t *mark = (uint32_t *)mark_v, *queue = (uint32_t *)queue_v, *scal = (uint32_t *)scal_v;
    unsigned long long *s64 = round_s64(scal_v, h);
    uint2 *items = (uint2 *)items_v;
    const RoundGraph rg = round_graph(g);
    uint32_t *part = (uint32_t *)part_v;
    uint32_t *dhat = estimate ? estimate : (uint32_t *)dhat_v;
    uint32_t *lb = (uint32_t *)lb_v, *ub = (uint32_t *)ub_v;
    float *X = (float *)x_v, *Y = (float *)y_v;
    std::vector<uint32_t *> dj(h - 1);
    for (uint32_t j = 0; j + 1 < h; ++j) dj[j] = (uint32_t *)dj_v + (size_t)j * n;
    const uint32_t a = h >= 4 ? h - 3 : 1, b = h >= 3 ? h - 2 : 1;
    const int gn = grid_of(ctx, n, 256);
    const int wgrid = ctx->num_cu * 4;

    hipLaunchKernelGGL(ainit_kernel, dim3(gn), dim3(256), 0, st, n, alive, mark, core, scal, nscal);
    fill_u32(ctx, (uint32_t *)dj_v, 0u, (uint64_t)(h - 1) * n);
    uint32_t *srcs, nsrc;
    if ((rc = compact_sources(ctx, g, alive, &srcs, &nsrc))) return rc;
    if ((rc = hop_degrees(ctx, g, alive, h, srcs, nsrc, dj.data()))) return rc;
    sl.hm1_recomputes += n;
    // initial estimates of every vertex
    hipLaunchKernelGGL(features_kernel, dim3(wgrid), dim3(256), 0, st, (const uint32_t *)nullptr, n, g->row_ptr,
                       g->col, alive, dj[a - 1], dj[b - 1], dj[h - 2], (const uint32_t *)(scal + R_LIVE), X, lb, ub);
    if (mlp && (rc = khc_mlp_forward(ctx, mlp, X, n, Y))) return rc;
    hipLaunchKernelGGL(estimate_kernel, dim3(gn), dim3(256), 0, st, (const uint32_t *)nullptr, n,
                       mlp ? (const float *)Y : (const float *)nullptr, lb, ub, dhat, 0);

    uint64_t left = n;
    uint32_t r = 0;
    uint32_t *hs = ctx->host_scalars;
    auto last_report = std::chrono::steady_clock::now();
    while (left > 0) {
        if ((uint64_t)r > (uint64_t)n) return set_error(ctx, KHC_ELIMIT, "more rounds than vertices");
        hipLaunchKernelGGL(keymin_kernel, dim3(kMinBlocks), dim3(256), 0, st, n, alive, (const uint8_t *)nullptr,
                           dhat, (const uint32_t *)nullptr, part, scal, s64, (int)h);
        hipLaunchKernelGGL(select_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, g->row_ptr, alive,
                           (const uint8_t *)nullptr, dhat, part, mark, core, (uint32_t *)nullptr, r, queue, scal, s64,
                           items, (int)h);
        for (uint32_t lev = 1; lev <= h; ++lev)
            hipLaunchKernelGGL(affected_kernel, dim3(wgrid), dim3(256), 0, st, rg, alive, mark, queue, scal, s64,
                               items, (int)lev, (int)h);
        hipLaunchKernelGGL(kill_kernel, dim3(gn), dim3(256), 0, st, queue, scal, alive, (uint32_t *)nullptr, 0);
        hipError_t e = hipMemcpyAsync(hs, scal, (size_t)nscal * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return check_hip(ctx, e, "approx round readback");
        const uint32_t np = hs[R_CNT];
        uint32_t nm = 0, tot = 0;
        for (uint32_t j = 0; j <= h; ++j) {
            if (j < h) nm += hs[R_CNT + j];
            tot += hs[R_CNT + j];
        }
        if (np == 0) return set_error(ctx, KHC_ELIMIT, "round removed no vertex");
        // exact j-hop degrees change only within h-1 hops of P
        if (nm > np) {
            if ((rc = hop_degrees(ctx, g, alive, h, queue + np, nm - np, dj.data()))) return rc;
            sl.hm1_recomputes += nm - np;
        }
        // features and estimates of everything within h hops of P
        const uint32_t na = tot - np;
        if (na) {
            hipLaunchKernelGGL(features_kernel, dim3(wgrid), dim3(256), 0, st, (const uint32_t *)(queue + np), na,
                               g->row_ptr, g->col, alive, dj[a - 1], dj[b - 1], dj[h - 2],
                               (const uint32_t *)(scal + R_LIVE), X, lb, ub);
            if (mlp && (rc = khc_mlp_forward(ctx, mlp, X, na, Y))) return rc;
            hipLaunchKernelGGL(estimate_kernel, dim3(grid_of(ctx, na, 256)), dim3(256), 0, st,
                               (const uint32_t *)(queue + np), na, mlp ? (const float *)Y : (const float *)nullptr,
                               lb, ub, dhat, 1);
        }
        hipLaunchKernelGGL(finish_kernel, dim3(gn), dim3(256), 0, st, queue, scal, (int)h, mark, (uint8_t *)nullptr,
                           (uint8_t)0);
        sl.affected_total += na;
        left -= np;
        ++r;
        report_progress(ctx, &last_report, r, (uint64_t)n - left, hs[R_KNEW]);
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "approx end");
    sl.rounds = r;
    sl.max_level = hs[R_K];
    sl.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = sl;
    return KHC_OK;
}

}  // extern "C"
