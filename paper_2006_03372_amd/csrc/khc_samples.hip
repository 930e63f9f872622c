// Training samples of the learned modes, built on the device (gfx950).
//
// For a peeling state G(alive) the network's inputs are the features of
// every live vertex (khc_features for the estimating mode, khc_gate_features
// for the recompute gate) and its target is log1p(d^h(v)) / 8 with d^h the
// exact h-degree (khdeg_compute).  The live rows are compacted in vertex
// order by a block count, a scan and a scatter, so the sample order, and
// with it a seeded training run, does not depend on scheduling.  States
// come from an exact decomposition's removal rounds: the vertices still
// present after round r0 are those removed in round r0 or later.
#include <cmath>

#include "khc_internal.h"

extern "C" int khc_features(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, float *X,
                            uint32_t *lb, uint32_t *ub);
extern "C" int khc_gate_features(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                                 const uint32_t *dm, float *X);

namespace khc {
namespace {

constexpr int kTile = 1024;  // vertices per compaction block (one thread each)

// cnt[b] = live vertices among [b * kTile, (b + 1) * kTile).
__global__ __launch_bounds__(kTile) void tile_count_kernel(uint32_t n, const uint8_t *alive, uint32_t *cnt) {
    const uint32_t v = blockIdx.x * kTile + threadIdx.x;
    const int live = v < n && (!alive || alive[v]);
    const int c = __syncthreads_count(live);
    if (threadIdx.x == 0) cnt[blockIdx.x] = (uint32_t)c;
}

// Exclusive scan of cnt[0, nb) in place (one block); total into cnt[nb].
__global__ __launch_bounds__(1024) void tile_scan_kernel(uint32_t nb, uint32_t *cnt) {
    __shared__ uint32_t part[1024];
    const uint32_t per = (nb + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
    uint32_t s = 0;
    for (uint32_t b = b0; b < b1; ++b) s += cnt[b];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread sums
    for (uint32_t off = 1; off < blockDim.x; off <<= 1) {
        const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t c = cnt[b];
        cnt[b] = run;
        run += c;
    }
    if (threadIdx.x == blockDim.x - 1) cnt[nb] = part[threadIdx.x];
}

// Row i of X / target for the i-th live vertex in vertex order.
__global__ __launch_bounds__(kTile) void tile_scatter_kernel(uint32_t n, const uint8_t *alive, const uint32_t *offs,
                                                             const float *Xall, const uint32_t *d, float *X,
                                                             float *target) {
    __shared__ uint32_t wsum[kTile / 64];
    const uint32_t v = blockIdx.x * kTile + threadIdx.x;
    const bool live = v < n && (!alive || alive[v]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t m = __ballot(live);
    if (lane == 0) wsum[wave] = (uint32_t)__builtin_popcountll(m);
    __syncthreads();
    uint32_t at = offs[blockIdx.x];
    for (int w = 0; w < wave; ++w) at += wsum[w];
    at += (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
    if (!live) return;
    for (int k = 0; k < 8; ++k) X[(size_t)at * 8 + k] = Xall[(size_t)v * 8 + k];
    target[at] = (float)log1p((double)d[v]) / 8.f;
}

__global__ void alive_after_kernel(uint32_t n, const uint32_t *round, uint32_t r0, uint8_t *alive) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        alive[v] = round[v] >= r0 ? 1 : 0;
}

}  // namespace
}  // namespace khc

using namespace khc;

extern "C" int khc_mlp_samples(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, int kind,
                               float *X, float *target, uint32_t *count) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !X || !target || !count) return set_error(ctx, KHC_EINVAL, "graph, output or count is null");
    if (kind != 0 && kind != 1) return set_error(ctx, KHC_EINVAL, "kind must be 0 (estimate) or 1 (gate)");
    if (h < 2 || h > 64) return set_error(ctx, KHC_EINVAL, "samples need 2 <= h <= 64");
    (void)hipSetDevice(ctx->device);
    const uint32_t n = g->n;
    *count = 0;
    if (n == 0) return KHC_OK;
    hipStream_t st = ctx->stream;
    const uint32_t nb = (n + kTile - 1) / kTile;
    int rc;
    void *xall_v, *d_v, *dm_v, *cnt_v;
    if ((rc = ws_get(ctx, WS_APPROX_X, (size_t)n * 8 * 4 + 32, &xall_v)) ||
        (rc = ws_get(ctx, WS_DEG, (size_t)n * 4 + 8, &d_v)) || (rc = ws_get(ctx, WS_DHM1, (size_t)n * 4 + 8, &dm_v)) ||
        (rc = ws_get(ctx, WS_APPROX_Y, ((size_t)nb + 2) * 4 > (size_t)n * 4 + 8 ? ((size_t)nb + 2) * 4 : (size_t)n * 4 + 8,
                     &cnt_v)))
        return rc;
    float *Xall = (float *)xall_v;
    uint32_t *d = (uint32_t *)d_v, *dm = (uint32_t *)dm_v, *cnt = (uint32_t *)cnt_v;
    if (kind == 0) {
        if ((rc = khc_features(ctx, g, alive, h, Xall, nullptr, nullptr))) return rc;
    } else {
        if ((rc = khdeg_compute(ctx, g, alive, h - 1, dm))) return rc;
        if ((rc = khc_gate_features(ctx, g, alive, h, dm, Xall))) return rc;
    }
    if ((rc = khdeg_compute(ctx, g, alive, h, d))) return rc;
    hipLaunchKernelGGL(tile_count_kernel, dim3(nb), dim3(kTile), 0, st, n, alive, cnt);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(1024), 0, st, nb, cnt);
    hipLaunchKernelGGL(tile_scatter_kernel, dim3(nb), dim3(kTile), 0, st, n, alive, (const uint32_t *)cnt,
                       (const float *)Xall, (const uint32_t *)d, X, target);
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, cnt + nb, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "samples readback");
    *count = ctx->host_scalars[0];
    return KHC_OK;
}

extern "C" int khc_alive_after(khc_ctx *ctx, uint32_t n, const uint32_t *round, uint32_t r0, uint8_t *alive) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (n && (!round || !alive)) return set_error(ctx, KHC_EINVAL, "round or output is null");
    if (n == 0) return KHC_OK;
    (void)hipSetDevice(ctx->device);
    uint64_t blocks = ((uint64_t)n + 255) / 256;
    if (blocks > (uint64_t)ctx->num_cu * 8) blocks = (uint64_t)ctx->num_cu * 8;
    hipLaunchKernelGGL(alive_after_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, round, r0, alive);
    return check_hip(ctx, hipGetLastError(), "alive after");
}
