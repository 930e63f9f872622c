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
// BFS from P).  A small readback per round returns (k, |P|, level ends).
//
// Two schedules give identical results (core numbers and removal rounds):
//  * plain: every affected vertex gets its h-degree recomputed at once;
//  * bounded (h >= 2): exact (h-1)-degrees dm are maintained (they change
//    only within h-1 hops of P) and every affected vertex u only becomes
//    dirty, keeping its old h-degree as an upper bound (h-degrees never
//    grow as vertices are removed) and the lower bound
//        lb(u) = max(dm(u), max over live neighbours w of dm(w))
//    (the closed (h-1)-ball of a neighbour lies inside u's h-ball).  Before
//    each round the level is k = max(k, min over live v of key(v)), key =
//    d for clean and lb for dirty vertices; dirty vertices with lb <= k are
//    recomputed and the step repeats until none is left.  Then every dirty
//    vertex has d^h >= lb > k and P = {clean live v : d(v) <= k} is exactly
//    the set the plain schedule removes.  This carries the lower-bound idea
//    the paper attributes to h-LB (Section III) over to set removal.
#include <chrono>
#include <cstring>

#include "khc_internal.h"

namespace khc {
namespace {

enum : int { SC_MIN = 0, SC_K = 1, SC_TOT = 2, SC_RN = 3, SC_ENDS = 4 };

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

// min over live vertices of key = (dirty ? lb : d), into scal[SC_MIN].
__global__ void key_min_kernel(uint32_t n, const uint8_t *alive, const uint8_t *dirty,
                               const uint32_t *d, const uint32_t *lb, uint32_t *scal) {
    uint32_t m = 0xFFFFFFFFu;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (!alive[v]) continue;
        const uint32_t key = dirty[v] ? lb[v] : d[v];
        if (key < m) m = key;
    }
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t o = __shfl_down(m, off, 64);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m != 0xFFFFFFFFu) atomicMin(&scal[SC_MIN], m);
}

// k <- max(k, min key); reset the per-round counters.
__global__ void round_begin_kernel(uint32_t *scal) {
    const uint32_t m = scal[SC_MIN];
    if (m != 0xFFFFFFFFu && m > scal[SC_K]) scal[SC_K] = m;
    scal[SC_MIN] = 0xFFFFFFFFu;
    scal[SC_TOT] = 0;
    scal[SC_RN] = 0;
}

// Dirty live vertices whose lower bound has reached the level: their
// h-degree must be recomputed before the level can be trusted.
__global__ void collect_dirty_kernel(uint32_t n, const uint8_t *alive, const uint8_t *dirty,
                                     const uint32_t *lb, uint32_t *list, uint32_t *scal) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k = scal[SC_K];
    const bool take = v < n && alive[v] && dirty[v] && lb[v] <= k;
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&scal[SC_RN], (uint32_t)__builtin_popcountll(m));
    base = __shfl(base, leader, 64);
    if (take) list[base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = v;
}

__global__ void set_flag_kernel(const uint32_t *list, const uint32_t *count, uint8_t *flag,
                                uint8_t value) {
    const uint32_t cnt = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
        flag[list[i]] = value;
}

// lb(u) = max(dm(u), max over live neighbours of dm) for the listed live
// vertices u = list[begin .. end) (slots of scal), one wavefront each.
__global__ void lower_bound_kernel(const uint32_t *list, const uint32_t *scal, int begin_slot,
                                   int end_slot, uint32_t n_all, const uint64_t *row_ptr,
                                   const uint32_t *col, const uint8_t *alive, const uint32_t *dm,
                                   uint32_t *lb) {
    const uint32_t begin = list ? scal[begin_slot] : 0u;
    const uint32_t end = list ? scal[end_slot] : n_all;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t i = begin + wave; i < end; i += nwaves) {
        const uint32_t u = list ? list[i] : i;
        if (!alive[u]) continue;
        uint32_t m = 0;
        for (uint64_t a = row_ptr[u] + lane; a < row_ptr[u + 1]; a += 64) {
            const uint32_t w = col[a];
            if (alive[w] && dm[w] > m) m = dm[w];
        }
        for (int off = 32; off > 0; off >>= 1) {
            uint32_t o = __shfl_xor(m, off, 64);
            m = o > m ? o : m;
        }
        if (lane == 0) lb[u] = dm[u] > m ? dm[u] : m;
    }
}

// flag[queue[i]] = value for the affected part of the queue, [|P|, end).
__global__ void set_tail_flag_kernel(const uint32_t *queue, const uint32_t *scal, uint8_t *flag,
                                     uint8_t value) {
    const uint32_t begin = scal[SC_ENDS], end = scal[SC_TOT];
    for (uint32_t i = begin + blockIdx.x * blockDim.x + threadIdx.x; i < end; i += gridDim.x * blockDim.x)
        flag[queue[i]] = value;
}

__global__ void fill_u8_kernel(uint8_t *p, uint8_t value, uint32_t count) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = value;
}

// P = live (clean) vertices with d <= k: core k, removal round r, marked,
// queued.  dirty == null: every vertex is clean.
__global__ void select_kernel(uint32_t n, const uint8_t *alive, const uint8_t *dirty,
                              const uint32_t *d, uint32_t *mark, uint32_t *core, uint32_t *round,
                              uint32_t r, uint32_t *queue, uint32_t *scal) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k = scal[SC_K];
    const bool take = v < n && alive[v] && (!dirty || !dirty[v]) && d[v] <= k;
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

namespace {

struct PeelState {
    uint8_t *alive, *dirty;
    uint32_t *d, *dm, *lb, *mark, *queue, *list, *scal;
    int nscal;
};

// P selection, the depth-h affected-set BFS from P over the graph before
// removal, removal of P, and the readback of (k, |P|, level ends).
int peel_round_common(khc_ctx *ctx, const khc_graph *g, uint32_t h, const PeelState &s, bool bounded,
                      uint32_t r, uint32_t *core, uint32_t *peel_round, int grid_n) {
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    hipLaunchKernelGGL(select_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, s.alive,
                       bounded ? s.dirty : (const uint8_t *)nullptr, s.d, s.mark, core, peel_round, r,
                       s.queue, s.scal);
    hipLaunchKernelGGL(snapshot_kernel, dim3(1), dim3(1), 0, st, s.scal, 0);
    const int agrid = ctx->num_cu * 4;
    for (uint32_t lev = 1; lev <= h; ++lev) {
        hipLaunchKernelGGL(affected_level_kernel, dim3(agrid), dim3(256), 0, st, g->row_ptr, g->col,
                           s.alive, s.mark, s.queue, s.scal, (int)lev);
        hipLaunchKernelGGL(snapshot_kernel, dim3(1), dim3(1), 0, st, s.scal, (int)lev);
    }
    hipLaunchKernelGGL(kill_kernel, dim3(grid_n), dim3(256), 0, st, s.queue, s.scal, s.alive);
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, s.scal, (size_t)s.nscal * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "peel round readback");
    if (ctx->host_scalars[SC_ENDS] == 0) return set_error(ctx, KHC_ELIMIT, "round removed no vertex");
    return KHC_OK;
}

}  // namespace

int khc::host_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core,
                        uint32_t *peel_round, khc_stats *stats) {
    if (g->ngraphs > 1)
        return set_error(ctx, KHC_EINVAL, "graphs packed together need the persistent driver");
    const auto t0 = std::chrono::steady_clock::now();
    khc_stats st_local;
    std::memset(&st_local, 0, sizeof(st_local));
    const uint32_t n = g->n;
    hipStream_t st = ctx->stream;
    const bool bounded = ctx->schedule == 1 && h >= 2;
    int rc;
    void *alive_v, *dirty_v, *d_v, *dm_v, *lb_v, *mark_v, *queue_v, *list_v, *scal_v;
    PeelState s;
    s.nscal = SC_ENDS + (int)h + 2;
    if ((rc = ws_get(ctx, WS_ALIVE, (size_t)n + 8, &alive_v)) ||
        (rc = ws_get(ctx, WS_DIRTY, (size_t)n + 8, &dirty_v)) ||
        (rc = ws_get(ctx, WS_DEG, (size_t)n * 4 + 8, &d_v)) ||
        (rc = ws_get(ctx, WS_DHM1, (size_t)n * 4 + 8, &dm_v)) ||
        (rc = ws_get(ctx, WS_LB, (size_t)n * 4 + 8, &lb_v)) ||
        (rc = ws_get(ctx, WS_MARK, (size_t)n * 4 + 8, &mark_v)) ||
        (rc = ws_get(ctx, WS_QUEUE0, (size_t)n * 4 + 8, &queue_v)) ||
        (rc = ws_get(ctx, WS_QUEUE1, (size_t)n * 4 + 8, &list_v)) ||
        (rc = ws_get(ctx, WS_SCRATCH, (size_t)s.nscal * 4, &scal_v)))
        return rc;
    s.alive = (uint8_t *)alive_v;
    s.dirty = (uint8_t *)dirty_v;
    s.d = (uint32_t *)d_v;
    s.dm = (uint32_t *)dm_v;
    s.lb = (uint32_t *)lb_v;
    s.mark = (uint32_t *)mark_v;
    s.queue = (uint32_t *)queue_v;
    s.list = (uint32_t *)list_v;
    s.scal = (uint32_t *)scal_v;
    const int g_n = (int)std::min<uint64_t>(((uint64_t)n + 255) / 256, (uint64_t)ctx->num_cu * 8);
    const int grid_n = g_n < 1 ? 1 : g_n;
    const int wgrid = ctx->num_cu * 4;  // wavefront-per-vertex kernels

    if (n == 0) {
        if (stats) *stats = st_local;
        return KHC_OK;
    }
    hipLaunchKernelGGL(peel_init_kernel, dim3(grid_n), dim3(256), 0, st, n, s.alive, s.mark, core,
                       peel_round, s.scal, s.nscal);
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_n), dim3(256), 0, st, s.dirty, (uint8_t)0, n);
    if ((rc = khdeg_compute(ctx, g, s.alive, h, s.d))) return rc;
    st_local.h_recomputes += n;
    if (bounded) {
        if ((rc = khdeg_compute(ctx, g, s.alive, h - 1, s.dm))) return rc;
        st_local.hm1_recomputes += n;
        hipLaunchKernelGGL(lower_bound_kernel, dim3(wgrid), dim3(256), 0, st, (const uint32_t *)nullptr,
                           s.scal, 0, 0, n, g->row_ptr, g->col, s.alive, s.dm, s.lb);
    }

    uint64_t left = n;
    uint32_t r = 0;
    uint32_t *hs = ctx->host_scalars;
    while (left > 0) {
        if ((uint64_t)r > (uint64_t)n) return set_error(ctx, KHC_ELIMIT, "more rounds than vertices");
        if (!bounded) {
            hipLaunchKernelGGL(reduce_min_kernel, dim3(grid_n), dim3(256), 0, st, n, s.alive, s.d, s.scal);
            hipLaunchKernelGGL(round_begin_kernel, dim3(1), dim3(1), 0, st, s.scal);
        } else {
            // Raise the level until no dirty vertex's lower bound reaches it.
            for (;;) {
                hipLaunchKernelGGL(key_min_kernel, dim3(grid_n), dim3(256), 0, st, n, s.alive, s.dirty,
                                   s.d, s.lb, s.scal);
                hipLaunchKernelGGL(round_begin_kernel, dim3(1), dim3(1), 0, st, s.scal);
                hipLaunchKernelGGL(collect_dirty_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n,
                                   s.alive, s.dirty, s.lb, s.list, s.scal);
                hipError_t e = hipMemcpyAsync(hs, s.scal, (size_t)SC_ENDS * 4, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) return check_hip(ctx, e, "level readback");
                const uint32_t rn = hs[SC_RN];
                if (rn == 0) break;
                if ((rc = msbfs_degrees(ctx, g, s.alive, h, s.list, rn, nullptr, 1, s.d))) return rc;
                hipLaunchKernelGGL(set_flag_kernel, dim3(grid_n), dim3(256), 0, st, s.list,
                                   s.scal + SC_RN, s.dirty, (uint8_t)0);
                st_local.h_recomputes += rn;
            }
        }
        if ((rc = peel_round_common(ctx, g, h, s, bounded, r, core, peel_round, grid_n))) return rc;
        const uint32_t np = hs[SC_ENDS];
        const uint32_t tot = hs[SC_TOT];
        const uint32_t na = tot - np;
        if (!bounded) {
            if (na) {
                if ((rc = msbfs_degrees(ctx, g, s.alive, h, s.queue + np, na, nullptr, 1, s.d))) return rc;
                st_local.h_recomputes += na;
            }
        } else if (na) {
            // exact (h-1)-degrees change only within h-1 hops of P
            const uint32_t nm = hs[SC_ENDS + h - 1] - np;
            if (nm) {
                if ((rc = msbfs_degrees(ctx, g, s.alive, h - 1, s.queue + np, nm, nullptr, 1, s.dm)))
                    return rc;
                st_local.hm1_recomputes += nm;
            }
            // bounds and dirtiness change only within h hops of P
            hipLaunchKernelGGL(lower_bound_kernel, dim3(wgrid), dim3(256), 0, st, s.queue, s.scal,
                               (int)SC_ENDS, (int)SC_TOT, n, g->row_ptr, g->col, s.alive, s.dm, s.lb);
            hipLaunchKernelGGL(set_tail_flag_kernel, dim3(grid_n), dim3(256), 0, st, s.queue, s.scal,
                               s.dirty, (uint8_t)1);
        }
        hipLaunchKernelGGL(unmark_kernel, dim3(grid_n), dim3(256), 0, st, s.queue, s.scal, s.mark);
        st_local.affected_total += na;
        left -= np;
        ++r;
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "peel end");
    if ((e = hipGetLastError()) != hipSuccess) return check_hip(ctx, e, "peel launch");
    st_local.rounds = r;
    st_local.max_level = hs[SC_K];
    st_local.width_words = (uint32_t)ctx->max_width;
    st_local.wall_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st_local;
    return KHC_OK;
}
