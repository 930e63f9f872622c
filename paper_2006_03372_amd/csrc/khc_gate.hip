// Learned recompute gate for the bounded peeling schedule (gfx950).
//
// The bounded schedule (khc_peel.hip) keeps an affected vertex dirty with
// its stale h-degree d (an upper bound) and an exact lower bound lb, and
// recomputes it by MS-BFS as soon as lb <= k < d at the current level k.
// Most of those recomputes find d^h well above k: the lower bound was
// loose.  The gate asks the network first.  For a dirty vertex u with
// lb <= k < d the estimate
//     e = clamp(expm1(8 y), lb, d),   y = net(features(u)),
// gives the soft key s = lb + floor((e - lb) * (1 - margin)); if s > k the
// recompute is deferred and s replaces lb as u's key, so u comes back when
// the level reaches s (then it is recomputed without asking again) or when
// a later removal affects it (then its exact lower bound is rebuilt and the
// gate may be asked again).  A vertex still leaves only when its exact or
// stale h-degree is at most k, so every core number the gated run returns
// is at least the exact one; it is larger exactly when a deferral passed
// over the level the vertex belonged to.  Without a network, or with
// margin 1, nothing is deferred and the run is the exact bounded schedule.
//
// Features of a live vertex u (log1p of the count, divided by 8), from
// quantities the bounded schedule keeps anyway (dm: lower bounds on the
// (h-1)-degrees, exact where recently recomputed) and the CSR:
//   0 live degree of u            4 max over live neighbours w of dm(w)
//   1 dm(u)                       5 mean over live w of the full degree of w
//   2 min over live w of dm(w)    6 min(live - 1, sum over live w of dm(w))
//   3 mean over live w of dm(w)   7 live - 1
// (the h-ball of u is the union of the closed (h-1)-balls of its live
// neighbours, minus u).
#include <chrono>
#include <cmath>

#include "khc_round.h"

extern "C" int khc_mlp_forward(khc_ctx *ctx, const khc_mlp *m, const float *X, uint32_t n, float *y);

namespace khc {
namespace {

using namespace rnd;

constexpr float kGateScale = 8.f;
constexpr int kGateFeat = 8;

// Features of list[i] (list null: vertex i) into row i of X, one wavefront
// per vertex; dead vertices get zeros.
__global__ void gate_features_kernel(const uint32_t *list, uint32_t count, const uint64_t *row_ptr,
                                     const uint32_t *col, const uint8_t *alive, const uint32_t *dm,
                                     const uint32_t *live_count, float *X) {
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t live_all = *live_count;
    for (uint32_t i = wave; i < count; i += nwaves) {
        const uint32_t u = list ? list[i] : i;
        const bool live = !alive || alive[u];
        uint32_t mn = 0xFFFFFFFFu, mx = 0, deg = 0;
        uint64_t sd = 0, sf = 0;
        if (live) {
            for (uint64_t a = row_ptr[u] + lane; a < row_ptr[u + 1]; a += 64) {
                const uint32_t w = col[a];
                if (alive && !alive[w]) continue;
                const uint32_t c = dm[w];
                mn = c < mn ? c : mn;
                mx = c > mx ? c : mx;
                sd += c;
                sf += row_ptr[w + 1] - row_ptr[w];
                deg++;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const uint32_t omn = __shfl_xor(mn, off, 64), omx = __shfl_xor(mx, off, 64);
            mn = omn < mn ? omn : mn;
            mx = omx > mx ? omx : mx;
            sd += __shfl_xor(sd, off, 64);
            sf += __shfl_xor(sf, off, 64);
            deg += __shfl_xor(deg, off, 64);
        }
        if (lane == 0) {
            float f[kGateFeat] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (live) {
                const uint64_t cap = live_all ? (uint64_t)live_all - 1 : 0;
                f[0] = log1pf((float)deg);
                f[1] = log1pf((float)dm[u]);
                if (deg) {
                    f[2] = log1pf((float)mn);
                    f[3] = log1pf((float)((double)sd / (double)deg));
                    f[4] = log1pf((float)mx);
                    f[5] = log1pf((float)((double)sf / (double)deg));
                }
                f[6] = log1pf((float)(sd < cap ? sd : cap));
                f[7] = log1pf((float)cap);
            }
            for (int k = 0; k < kGateFeat; ++k) X[(size_t)i * kGateFeat + k] = f[k] / kGateScale;
        }
    }
}

__global__ void gate_live_kernel(uint32_t n, const uint8_t *alive, uint32_t *out) {
    uint32_t c = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        c += (!alive || alive[v]) ? 1u : 0u;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

// The gate over the collected list (count s[R_RN], level from the partial
// minima as collect saw them).  A vertex asked before (dirty == 2) is kept
// for the recompute; a vertex whose soft key exceeds k is deferred (lb <- s,
// dirty <- 2); the kept ones are appended to out (count s[R_GKEEP], which
// keymin clears).  Every lane runs the same trip count (wave_reserve).
__global__ void gate_kernel(const uint32_t *list, const float *y, uint32_t *lb, const uint32_t *d, uint8_t *dirty,
                            const uint32_t *part, uint32_t *s, float keep, uint32_t *out) {
    const uint32_t k = block_level(part, s);
    const uint32_t cnt = s[R_RN];
    const uint32_t trips = (cnt + gridDim.x * blockDim.x - 1) / (gridDim.x * blockDim.x);
    for (uint32_t t = 0; t < trips; ++t) {
        const uint32_t i = (t * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
        bool take = false;
        if (i < cnt) {
            const uint32_t u = list[i];
            take = true;
            if (dirty[u] == 1) {
                const uint32_t lo = lb[u], hi = d[u];
                const float z = floorf(expm1f(kGateScale * y[i]) + 0.5f);
                uint32_t e = z <= 0.f ? 0u : (z >= 4294967040.f ? 0xFFFFFF00u : (uint32_t)z);
                e = e > hi ? hi : e;
                e = e < lo ? lo : e;
                const uint32_t soft = lo + (uint32_t)floorf((float)(e - lo) * keep);
                if (soft > k) {
                    lb[u] = soft;
                    dirty[u] = 2;
                    take = false;
                }
            }
        }
        const uint32_t at = wave_reserve(take, &s[R_GKEEP]);
        if (take) out[at] = list[i];
    }
}

}  // namespace

int gate_features(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, const uint32_t *dm, const uint32_t *list,
                  uint32_t count, const uint32_t *live_count, float *X) {
    if (count == 0) return KHC_OK;
    uint64_t waves = (uint64_t)count;
    uint64_t blocks = (waves + 3) / 4;
    if (blocks > (uint64_t)ctx->num_cu * 8) blocks = (uint64_t)ctx->num_cu * 8;
    hipLaunchKernelGGL(gate_features_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, list, count,
                       g->row_ptr, g->col, alive, dm, live_count, X);
    return check_hip(ctx, hipGetLastError(), "gate features");
}

int gate_pass(khc_ctx *ctx, const khc_graph *g, const khc_mlp *mlp, float margin, const uint8_t *alive,
              const uint32_t *dm, const uint32_t *list, uint32_t rn, uint32_t *lb, const uint32_t *d, uint8_t *dirty,
              const uint32_t *part, uint32_t *s, float *X, float *Y, uint32_t *out) {
    int rc;
    if ((rc = gate_features(ctx, g, alive, dm, list, rn, s + R_LIVE, X))) return rc;
    if ((rc = khc_mlp_forward(ctx, mlp, X, rn, Y))) return rc;
    uint64_t blocks = ((uint64_t)rn + 255) / 256;
    if (blocks > (uint64_t)ctx->num_cu * 8) blocks = (uint64_t)ctx->num_cu * 8;
    hipLaunchKernelGGL(gate_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, list, (const float *)Y, lb, d,
                       dirty, part, s, 1.f - margin, out);
    return check_hip(ctx, hipGetLastError(), "gate");
}

}  // namespace khc

using namespace khc;

extern "C" int khc_gate_features(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                                 const uint32_t *dm, float *X) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !dm || !X) return set_error(ctx, KHC_EINVAL, "graph, dm or output is null");
    if (h < 2 || h > kMaxRoundH) return set_error(ctx, KHC_EINVAL, "gate features need 2 <= h <= 1024");
    (void)hipSetDevice(ctx->device);
    const uint32_t n = g->n;
    if (n == 0) return KHC_OK;
    void *cnt;
    int rc;
    if ((rc = ws_get(ctx, WS_APPROX_SCAL, 64, &cnt))) return rc;
    uint32_t *live = (uint32_t *)cnt;
    fill_u32(ctx, live, 0u, 1);
    uint64_t blocks = ((uint64_t)n + 255) / 256;
    if (blocks > (uint64_t)ctx->num_cu * 8) blocks = (uint64_t)ctx->num_cu * 8;
    hipLaunchKernelGGL(gate_live_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, alive, live);
    return gate_features(ctx, g, alive, dm, nullptr, n, live, X);
}

extern "C" int khcore_decompose_gated(khc_ctx *ctx, const khc_graph *g, uint32_t h, const khc_mlp *mlp, float margin,
                                      uint32_t *core, uint32_t *peel_round, khc_stats *stats) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !core) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h < 2 || h > kMaxRoundH) return set_error(ctx, KHC_EINVAL, "the gated mode needs 2 <= h <= 1024");
    if (g->ngraphs > 1) return set_error(ctx, KHC_EINVAL, "the gated mode takes one graph");
    if (!(margin >= 0.f && margin <= 1.f)) return set_error(ctx, KHC_EINVAL, "margin must be in [0, 1]");
    (void)hipSetDevice(ctx->device);
    // the gate sits in the bounded schedules (1, or 3 with decremented (h-1)-bounds)
    const int saved = ctx->schedule;
    ctx->schedule = saved == 3 ? 3 : 1;
    const GateArgs gate{mlp, margin};
    const int rc = host_decompose(ctx, g, h, core, peel_round, stats, &gate);
    ctx->schedule = saved;
    return rc;
}
