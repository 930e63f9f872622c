// Level-synchronous (k,h)-core peeling driver (gfx950).
//
// Peeling follows Algorithms 1-2 of the paper in level-synchronous form:
// each round sets the level k <- max(k, min live h-degree), removes every
// live vertex whose h-degree is at most k (all of them get core k), and
// recomputes the h-degree of the live vertices within h hops of the removed
// set, measured in the graph before removal (Observations 1-2 of Section
// IV-A, which for a removed set say that no other vertex can lose a
// neighbour within h hops).  The recomputation runs the multi-source
// bounded BFS on the graph after removal.
//
// Device state: alive u8[n], d u32[n], mark u32[n] and one queue u32[n]
// whose prefix [0, |P|) is the removed set P of the round and whose
// remainder collects the affected set A level by level (a depth-h push
// BFS from P).  One small readback per round returns (k, |P|, |P|+|A|).
#include <chrono>
#include <cstring>

#include "khc_internal.h"

namespace khc {
namespace {

enum : int { SC_MIN = 0, SC_K = 1, SC_TOT = 2, SC_ENDS = 3 };

__global__ void peel_init_kernel(uint32_t n, uint8_t *alive, uint32_t *mark, uint32_t *core,
                                 uint32_t *round, uint32_t *scal, int nscal) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        alive[v] = 1;
        mark[v] = 0;
        core[v] = 0;
        if (round) round[v] = 0;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < nscal; i += blockDim.x) scal[i] = (i == SC_MIN) ? 0xFFFFFFFFu : 0u;
}

// min over live vertices of d, into scal[SC_MIN] (reset to ~0 each round).
__global__ void reduce_min_kernel(uint32_t n, const uint8_t *alive, const uint32_t *d, uint32_t *scal) {
    uint32_t m = 0xFFFFFFFFu;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (alive[v] && d[v] < m) m = d[v];
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t o = __shfl_down(m, off, 64);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m != 0xFFFFFFFFu) atomicMin(&scal[SC_MIN], m);
}

// k <- max(k, min d); reset the per-round counters.
__global__ void round_begin_kernel(uint32_t *scal) {
    const uint32_t m = scal[SC_MIN];
    if (m != 0xFFFFFFFFu && m > scal[SC_K]) scal[SC_K] = m;
    scal[SC_MIN] = 0xFFFFFFFFu;
    scal[SC_TOT] = 0;
}

// P = live vertices with d <= k: core k, removal round r, marked, queued.
__global__ void select_kernel(uint32_t n, const uint8_t *alive, const uint32_t *d, uint32_t *mark,
                              uint32_t *core, uint32_t *round, uint32_t r, uint32_t *queue,
                              uint32_t *scal) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k = scal[SC_K];
    const bool take = v < n && alive[v] && d[v] <= k;
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&scal[SC_TOT], (uint32_t)__builtin_popcountll(m));
    base = __shfl(base, leader, 64);
    if (take) {
        core[v] = k;
        if (round) round[v] = r;
        mark[v] = 1;
        queue[base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = v;
    }
}

__global__ void snapshot_kernel(uint32_t *scal, int slot) { scal[SC_ENDS + slot] = scal[SC_TOT]; }

// One level of the affected-set BFS: every vertex queued at the previous
// level pushes to its live unmarked neighbours (one wavefront per queued
// vertex, lanes over its arcs).  Level 1 expands P itself.
__global__ void affected_level_kernel(const uint64_t *row_ptr, const uint32_t *col,
                                      const uint8_t *alive, uint32_t *mark, uint32_t *queue,
                                      uint32_t *scal, int level) {
    const uint32_t begin = level >= 2 ? scal[SC_ENDS + level - 2] : 0u;
    const uint32_t end = scal[SC_ENDS + level - 1];
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t i = begin + wave; i < end; i += nwaves) {
        const uint32_t x = queue[i];
        const uint64_t rb = row_ptr[x], re = row_ptr[x + 1];
        for (uint64_t a = rb + lane; a < re; a += 64) {
            const uint32_t y = col[a];
            if (alive[y] && mark[y] == 0u && atomicCAS(&mark[y], 0u, 1u) == 0u) {
                const uint32_t pos = atomicAdd(&scal[SC_TOT], 1u);
                queue[pos] = y;
            }
        }
    }
}

__global__ void kill_kernel(const uint32_t *queue, const uint32_t *scal, uint8_t *alive) {
    const uint32_t np = scal[SC_ENDS];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x)
        alive[queue[i]] = 0;
}

__global__ void unmark_kernel(const uint32_t *queue, const uint32_t *scal, uint32_t *mark) {
    const uint32_t tot = scal[SC_TOT];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x)
        mark[queue[i]] = 0;
}

}  // namespace
}  // namespace khc

using namespace khc;

extern "C" int khcore_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core,
                                uint32_t *peel_round, khc_stats *stats) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !core) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h == 0) return set_error(ctx, KHC_EINVAL, "h must be >= 1");
    (void)hipSetDevice(ctx->device);
    const auto t0 = std::chrono::steady_clock::now();
    khc_stats st_local;
    std::memset(&st_local, 0, sizeof(st_local));
    const uint32_t n = g->n;
    hipStream_t st = ctx->stream;
    int rc;
    void *alive_v, *d_v, *mark_v, *queue_v, *scal_v;
    const int nscal = SC_ENDS + (int)h + 2;
    if ((rc = ws_get(ctx, WS_ALIVE, (size_t)n + 8, &alive_v)) ||
        (rc = ws_get(ctx, WS_DEG, (size_t)n * 4 + 8, &d_v)) ||
        (rc = ws_get(ctx, WS_MARK, (size_t)n * 4 + 8, &mark_v)) ||
        (rc = ws_get(ctx, WS_QUEUE0, (size_t)n * 4 + 8, &queue_v)) ||
        (rc = ws_get(ctx, WS_SCRATCH, (size_t)nscal * 4, &scal_v)))
        return rc;
    uint8_t *alive = (uint8_t *)alive_v;
    uint32_t *d = (uint32_t *)d_v, *mark = (uint32_t *)mark_v, *queue = (uint32_t *)queue_v;
    uint32_t *scal = (uint32_t *)scal_v;
    const int g_n = (int)std::min<uint64_t>(((uint64_t)n + 255) / 256, (uint64_t)ctx->num_cu * 8);
    const int grid_n = g_n < 1 ? 1 : g_n;

    if (n == 0) {
        if (stats) *stats = st_local;
        return KHC_OK;
    }
    hipLaunchKernelGGL(peel_init_kernel, dim3(grid_n), dim3(256), 0, st, n, alive, mark, core,
                       peel_round, scal, nscal);
    if ((rc = khdeg_compute(ctx, g, alive, h, d))) return rc;
    st_local.h_recomputes += n;

    uint64_t left = n;
    uint32_t r = 0;
    uint32_t k_host = 0;
    uint32_t *hs = ctx->host_scalars;
    while (left > 0) {
        if ((uint64_t)r > (uint64_t)n) return set_error(ctx, KHC_ELIMIT, "more rounds than vertices");
        hipLaunchKernelGGL(reduce_min_kernel, dim3(grid_n), dim3(256), 0, st, n, alive, d, scal);
        hipLaunchKernelGGL(round_begin_kernel, dim3(1), dim3(1), 0, st, scal);
        hipLaunchKernelGGL(select_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, alive, d, mark,
                           core, peel_round, r, queue, scal);
        hipLaunchKernelGGL(snapshot_kernel, dim3(1), dim3(1), 0, st, scal, 0);
        const int agrid = ctx->num_cu * 4;
        for (uint32_t lev = 1; lev <= h; ++lev) {
            hipLaunchKernelGGL(affected_level_kernel, dim3(agrid), dim3(256), 0, st, g->row_ptr,
                               g->col, alive, mark, queue, scal, (int)lev);
            hipLaunchKernelGGL(snapshot_kernel, dim3(1), dim3(1), 0, st, scal, (int)lev);
        }
        hipLaunchKernelGGL(kill_kernel, dim3(grid_n), dim3(256), 0, st, queue, scal, alive);
        hipError_t e = hipMemcpyAsync(hs, scal, (size_t)nscal * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return check_hip(ctx, e, "peel round readback");
        k_host = hs[SC_K];
        const uint32_t np = hs[SC_ENDS];
        const uint32_t tot = hs[SC_TOT];
        if (np == 0) return set_error(ctx, KHC_ELIMIT, "round removed no vertex");
        const uint32_t na = tot - np;
        if (na) {
            if ((rc = msbfs_degrees(ctx, g, alive, h, queue + np, na, nullptr, 1, d))) return rc;
            st_local.h_recomputes += na;
        }
        hipLaunchKernelGGL(unmark_kernel, dim3(grid_n), dim3(256), 0, st, queue, scal, mark);
        st_local.affected_total += na;
        left -= np;
        ++r;
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "peel end");
    if ((e = hipGetLastError()) != hipSuccess) return check_hip(ctx, e, "peel launch");
    st_local.rounds = r;
    st_local.max_level = k_host;
    st_local.width_words = (uint32_t)ctx->max_width;
    st_local.wall_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st_local;
    return KHC_OK;
}
