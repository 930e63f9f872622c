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
//  * bounded (h >= 2): lower bounds dm on the (h-1)-degrees are maintained
//    (exact after each recompute; they change only within h-1 hops of P, are
//    recomputed within h-2 hops and lowered by |P| at distance h-1, where
//    only P itself can leave a vertex's (h-1)-ball).  Every affected vertex
//    u only becomes dirty, keeping its old h-degree as an upper bound
//    (h-degrees never grow as vertices are removed) and the lower bound
//        lb(u) = max(dm(u), max over live neighbours w of dm(w), lbx(u))
//    (the closed (h-1)-ball of a neighbour lies inside u's h-ball; lbx is
//    the decrement bound of lower_bound_kernel).  Before
//    each round the level is k = max(k, min over live v of key(v)), key =
//    d for clean and lb for dirty vertices; dirty vertices with
//    lb <= k < d are recomputed and the step repeats until none is left
//    (k only grows while it repeats, since every key is at most the true
//    h-degree).  Then a dirty vertex either has d^h >= lb > k or
//    d^h <= d <= k, and P = {live v : d(v) <= k} is exactly the set the
//    plain schedule removes.  This carries the lower-bound idea the paper
//    attributes to h-LB (Section III) over to set removal.
#include <chrono>
#include <cstring>
#include <vector>

#include "khc_round.h"

namespace khc {
namespace {

using namespace rnd;

__global__ void peel_init_kernel(uint32_t n, uint8_t *alive, uint8_t *dirty, uint32_t *mark, uint32_t *core,
                                 uint32_t *round, uint32_t *s, int nscal) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        alive[v] = 1;
        dirty[v] = 0;
        mark[v] = 0;
        core[v] = 0;
        if (round) round[v] = 0;
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < nscal; i += blockDim.x) s[i] = (i == R_LIVE) ? n : 0u;
}

__global__ void set_flag_kernel(const uint32_t *list, const uint32_t *count, uint8_t *flag, uint8_t value) {
    const uint32_t cnt = *count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
        flag[list[i]] = value;
}

// Lower bounds of the live vertices u = list[begin .. end) (all vertices
// when list is null); the range comes from the round counters (P is
// queue[0, cnt[0]), then the vertices at distance 1, 2, ... h from P).
// Two bounds, the larger is kept in lb:
//  * structural: max(dm(u), max over live neighbours w of dm(w));
//  * decrement (affected vertices only): removing P can cost u only
//    vertices of P and vertices within h - j hops of P, where j is u's
//    distance from P (a lost vertex's every short path from u runs through
//    P), so d(u) falls by at most C(h - j) = |{v : dist(P, v) <= h - j}|.
//    lbx(u) carries the bound from the last exact value: lbx = d - C when u
//    was clean, lbx - C when already dirty.  For the outermost ring, j = h,
//    the drop is at most |P|.
__global__ void lower_bound_kernel(const uint32_t *list, const uint32_t *s, int h, uint32_t n_all,
                                   const uint64_t *row_ptr, const uint32_t *col, const uint8_t *alive,
                                   const uint32_t *dm, uint32_t *lb, const uint8_t *dirty, const uint32_t *d,
                                   uint32_t *lbx) {
    uint32_t begin = 0, end = n_all;
    if (list) {
        begin = s[R_CNT];
        end = 0;
        for (int j = 0; j <= h; ++j) end += s[R_CNT + j];
    }
    // 16 lanes per vertex, at most kLbArcs neighbours each
    const int lane = threadIdx.x & 63, sub = lane & 15;
    const uint32_t grp = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const uint32_t ngrp = (gridDim.x * blockDim.x) >> 4;
    const uint32_t span = end - begin;
    const uint32_t trips = (span + ngrp - 1) / ngrp;
    for (uint32_t t = 0; t < trips; ++t) {
        const uint32_t i = begin + t * ngrp + grp;
        uint32_t m = 0, u = 0;
        bool live = false;
        if (i < end) {
            u = list ? list[i] : i;
            live = alive[u] != 0;
        }
        if (live) {
            const uint64_t rb = row_ptr[u], re0 = row_ptr[u + 1];
            const uint64_t re = re0 - rb > kLbArcs ? rb + kLbArcs : re0;
            // four arcs per lane and step, their loads independent; slots
            // past the end repeat the step's first arc (max is idempotent).
            // Measured 2-3% off the R-MAT-18 and Chung-Lu 200K h = 3
            // decompositions against one arc per step.
            for (uint64_t a = rb + sub; a < re; a += 64) {
                uint32_t w[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint64_t ak = a + 16u * k;
                    w[k] = col[ak < re ? ak : a];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t x = dm[w[k]];
                    if (alive[w[k]] && x > m) m = x;
                }
            }
        }
        for (int off = 8; off > 0; off >>= 1) {
            const uint32_t o = __shfl_xor(m, off, 64);
            m = o > m ? o : m;
        }
        if (live && sub == 0) {
            uint32_t b = dm[u] > m ? dm[u] : m;
            if (list) {
                // distance j of queue entry i from P, and C(h - j)
                uint32_t j = 0, at = s[R_CNT];
                while (i >= at) at += s[R_CNT + ++j];
                uint32_t loss = 0;
                for (int r = 0; r <= h - (int)j; ++r) loss += s[R_CNT + r];
                const uint32_t base = dirty[u] ? lbx[u] : d[u];
                const uint32_t x = base > loss ? base - loss : 0u;
                lbx[u] = x;
                b = b > x ? b : x;
            }
            lb[u] = b;
        }
    }
}

// Local update (schedule 2): mark (set != 0) or clear the region of the
// round, the queued vertices (P and every live vertex within h hops of it):
// pre[v] = 1 on the whole region, post[v] = 1 on it without P; clearing
// also zeroes the two row counters.
__global__ void region_kernel(const uint32_t *queue, const uint32_t *s, int h, const uint32_t *mark, uint8_t *pre,
                              uint8_t *post, uint32_t *cpre, uint32_t *cpost, int set) {
    uint32_t tot = 0;
    for (int j = 0; j <= h; ++j) tot += s[R_CNT + j];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
        const uint32_t v = queue[i];
        if (set) {
            pre[v] = 1;
            post[v] = mark[v] > 1u ? 1 : 0;
        } else {
            pre[v] = 0;
            post[v] = 0;
            cpre[v] = 0;
            cpost[v] = 0;
        }
    }
}

// d(u) loses the vertices it reached within h hops before the removal but
// not after (counted inside the region), for every affected u.
__global__ void local_apply_kernel(const uint32_t *queue, const uint32_t *s, int h, const uint32_t *cpre,
                                   const uint32_t *cpost, uint32_t *d) {
    const uint32_t np = s[R_CNT];
    uint32_t tot = 0;
    for (int j = 0; j <= h; ++j) tot += s[R_CNT + j];
    for (uint32_t i = np + blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
        const uint32_t u = queue[i];
        d[u] -= cpre[u] - cpost[u];
    }
}

// Schedule 3: the (h-1)-degree bounds of the vertices within h - 2 hops of
// P (queue levels 1 .. h-2) drop by the decrement bound instead of being
// recomputed: a vertex at distance j from P loses at most the vertices
// within h - 1 - j hops of P from its (h-1)-ball.  (Level h - 1 loses at
// most |P|, applied by kill_kernel.)
__global__ void dm_decrement_kernel(const uint32_t *queue, const uint32_t *s, int h, uint32_t *dm) {
    const uint32_t np = s[R_CNT];
    uint32_t e = np;
    for (int j = 1; j + 1 < h; ++j) e += s[R_CNT + j];
    for (uint32_t i = np + blockIdx.x * blockDim.x + threadIdx.x; i < e; i += gridDim.x * blockDim.x) {
        uint32_t j = 0, at = s[R_CNT];
        while (i >= at) at += s[R_CNT + ++j];
        uint32_t loss = 0;
        for (int r = 0; r <= h - 1 - (int)j; ++r) loss += s[R_CNT + r];
        const uint32_t u = queue[i];
        dm[u] = dm[u] > loss ? dm[u] - loss : 0u;
    }
}

// Keep the round's removed and affected counts where the next cleaning
// readback finds them (the level counters are cleared before it).
__global__ void round_tally_kernel(uint32_t *s, int h) {
    if (blockIdx.x || threadIdx.x) return;
    uint32_t na = 0;
    for (int j = 1; j <= h; ++j) na += s[R_CNT + j];
    s[R_PNP] = s[R_CNT];
    s[R_PNA] = na;
}

struct PeelState {
    uint8_t *alive, *dirty;
    uint32_t *d, *dm, *lb, *lbx, *mark, *queue, *list, *s, *part;
    unsigned long long *s64;
    uint2 *items;
    int nscal;
};

// Select P, find the vertices within h hops of P before removal, remove P,
// and (readback) read back the round counters.
int peel_round_common(khc_ctx *ctx, const khc_graph *g, uint32_t h, const PeelState &p, bool bounded, uint32_t r,
                      uint32_t *core, uint32_t *peel_round, int grid_n, bool readback) {
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    hipLaunchKernelGGL(select_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, g->row_ptr, p.alive,
                       bounded ? p.dirty : (const uint8_t *)nullptr, p.d, p.part, p.mark, core, peel_round, r,
                       p.queue, p.s, p.s64, p.items, (int)h);
    const int agrid = ctx->num_cu * 4;
    const RoundGraph rg = round_graph(g);
    for (uint32_t lev = 1; lev <= h; ++lev)
        hipLaunchKernelGGL(affected_kernel, dim3(agrid), dim3(256), 0, st, rg, p.alive, p.mark, p.queue, p.s, p.s64,
                           p.items, (int)lev, (int)h);
    hipLaunchKernelGGL(kill_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, p.alive,
                       bounded ? p.dm : (uint32_t *)nullptr, (int)h);
    if (!readback) return KHC_OK;
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, p.s, (size_t)p.nscal * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "peel round readback");
    if (ctx->host_scalars[R_CNT] == 0) return set_error(ctx, KHC_ELIMIT, "round removed no vertex");
    return KHC_OK;
}

}  // namespace
}  // namespace khc

using namespace khc;

int khc::host_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core,
                        uint32_t *peel_round, khc_stats *stats, const GateArgs *gate) {
    if (g->ngraphs > 1)
        return set_error(ctx, KHC_EINVAL, "graphs packed together need the persistent driver");
    if (h > kMaxRoundH) return set_error(ctx, KHC_EINVAL, "h above 1024");
    static_assert((size_t)(R_CNT + 2 * kMaxRoundH + 3) * 4 <= kHostScalarBytes, "round scalars fit the readback");
    const auto t0 = std::chrono::steady_clock::now();
    khc_stats st_local;
    std::memset(&st_local, 0, sizeof(st_local));
    const uint32_t n = g->n;
    hipStream_t st = ctx->stream;
    const bool gated = gate && gate->mlp && h >= 2;
    // schedule 3: (h-1)-degree bounds by decrement, refreshed with every recompute
    const bool lazy = ctx->schedule == 3 && h >= 2;
    const bool bounded = (ctx->schedule == 1 || gated || lazy) && h >= 2;
    // schedule 2: each round updates the affected h-degrees inside the
    // region N^h[P] (Section IV-A's update, for a removed set) when that is
    // cheaper than recomputing them
    const bool local = ctx->schedule == 2 && !gated;
    int rc;
    void *alive_v, *dirty_v, *d_v, *dm_v, *lb_v, *lbx_v, *mark_v, *queue_v, *list_v, *s_v, *part_v, *items_v;
    PeelState p;
    p.nscal = round_nscal(h);
    if ((rc = ws_get(ctx, WS_ALIVE, (size_t)n + 8, &alive_v)) ||
        (rc = ws_get(ctx, WS_DIRTY, (size_t)n + 8, &dirty_v)) ||
        (rc = ws_get(ctx, WS_DEG, (size_t)n * 4 + 8, &d_v)) ||
        (rc = ws_get(ctx, WS_DHM1, (size_t)n * 4 + 8, &dm_v)) ||
        (rc = ws_get(ctx, WS_LB, (size_t)n * 4 + 8, &lb_v)) ||
        (rc = ws_get(ctx, WS_LBX, (size_t)n * 4 + 8, &lbx_v)) ||
        (rc = ws_get(ctx, WS_MARK, (size_t)n * 4 + 8, &mark_v)) ||
        (rc = ws_get(ctx, WS_QUEUE0, (size_t)n * 4 + 8, &queue_v)) ||
        (rc = ws_get(ctx, WS_QUEUE1, (size_t)n * 4 + 8, &list_v)) ||
        (rc = ws_get(ctx, WS_SCRATCH, round_scalar_bytes(h), &s_v)) ||
        (rc = ws_get(ctx, WS_MINPART, (size_t)kMinBlocks * 4, &part_v)) ||
        (rc = ws_get(ctx, WS_ITEMS, round_item_capacity(n, g->nnz) * sizeof(uint2), &items_v)))
        return rc;
    float *gate_x = nullptr, *gate_y = nullptr;
    uint32_t *gate_list = nullptr;
    if (gated) {
        void *x_v, *y_v, *l_v;
        if ((rc = ws_get(ctx, WS_APPROX_X, (size_t)n * 8 * 4 + 32, &x_v)) ||
            (rc = ws_get(ctx, WS_APPROX_Y, (size_t)n * 4 + 8, &y_v)) ||
            (rc = ws_get(ctx, WS_GATE_LIST, (size_t)n * 4 + 8, &l_v)))
            return rc;
        gate_x = (float *)x_v;
        gate_y = (float *)y_v;
        gate_list = (uint32_t *)l_v;
    }
    uint8_t *region_pre = nullptr, *region_post = nullptr;
    uint32_t *cnt_pre = nullptr, *cnt_post = nullptr;
    if (local) {
        void *reg_v, *cnt_v;
        if ((rc = ws_get(ctx, WS_REGION, (size_t)2 * n + 16, &reg_v)) ||
            (rc = ws_get(ctx, WS_ROWCNT, (size_t)8 * n + 16, &cnt_v)))
            return rc;
        region_pre = (uint8_t *)reg_v;
        region_post = region_pre + n;
        cnt_pre = (uint32_t *)cnt_v;
        cnt_post = cnt_pre + n;
    }
    p.alive = (uint8_t *)alive_v;
    p.dirty = (uint8_t *)dirty_v;
    p.d = (uint32_t *)d_v;
    p.dm = (uint32_t *)dm_v;
    p.lb = (uint32_t *)lb_v;
    p.lbx = (uint32_t *)lbx_v;
    p.mark = (uint32_t *)mark_v;
    p.queue = (uint32_t *)queue_v;
    p.list = (uint32_t *)list_v;
    p.s = (uint32_t *)s_v;
    p.s64 = round_s64(s_v, h);
    p.items = (uint2 *)items_v;
    p.part = (uint32_t *)part_v;
    const int g_n = (int)std::min<uint64_t>(((uint64_t)n + 255) / 256, (uint64_t)ctx->num_cu * 8);
    const int grid_n = g_n < 1 ? 1 : g_n;
    const int wgrid = ctx->num_cu * 4;  // wavefront-per-vertex kernels

    if (n == 0) {
        if (stats) *stats = st_local;
        return KHC_OK;
    }
    hipLaunchKernelGGL(peel_init_kernel, dim3(grid_n), dim3(256), 0, st, n, p.alive, p.dirty, p.mark, core,
                       peel_round, p.s, p.nscal);
    if ((rc = khdeg_compute(ctx, g, p.alive, h, p.d))) return rc;
    st_local.h_recomputes += n;
    if (bounded) {
        if ((rc = khdeg_compute(ctx, g, p.alive, h - 1, p.dm))) return rc;
        st_local.hm1_recomputes += n;
        hipLaunchKernelGGL(lower_bound_kernel, dim3(wgrid), dim3(256), 0, st, (const uint32_t *)nullptr, p.s,
                           (int)h, n, g->row_ptr, g->col, p.alive, p.dm, p.lb, (const uint8_t *)p.dirty,
                           (const uint32_t *)p.d, p.lbx);
    }

    uint64_t left = n;
    uint32_t r = 0;
    uint32_t *hs = ctx->host_scalars;
    auto last_report = std::chrono::steady_clock::now();
    // Schedule 3 needs no host value between the removal and the bounds, so
    // a round does not wait for its counters: the next cleaning readback
    // brings them (R_PNP, R_PNA, R_LIVE).
    bool pending = false;
    auto take_tally = [&]() -> int {
        pending = false;
        if (hs[R_PNP] == 0) return set_error(ctx, KHC_ELIMIT, "round removed no vertex");
        st_local.affected_total += hs[R_PNA];
        left = hs[R_LIVE];
        report_progress(ctx, &last_report, r, (uint64_t)n - left, hs[R_K]);
        return KHC_OK;
    };
    while (left > 0 && !(ctx->round_limit && r >= ctx->round_limit)) {
        if ((uint64_t)r > (uint64_t)n) return set_error(ctx, KHC_ELIMIT, "more rounds than vertices");
        bool done = false;
        for (;;) {
            hipLaunchKernelGGL(keymin_kernel, dim3(kMinBlocks), dim3(256), 0, st, n, p.alive,
                               bounded ? p.dirty : (const uint8_t *)nullptr, p.d, p.lb, p.part, p.s, p.s64, (int)h);
            if (!bounded) break;
            // dirty vertices whose lower bound reached the level are recomputed first
            hipLaunchKernelGGL(collect_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, p.alive, p.dirty, p.lb,
                               p.d, p.part, p.list, p.s);
            hipError_t e = hipMemcpyAsync(hs, p.s, (size_t)R_CNT * 4, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return check_hip(ctx, e, "level readback");
            if (pending && (rc = take_tally())) return rc;
            if (lazy && hs[R_LIVE] == 0) {
                done = true;
                break;
            }
            const uint32_t rn = hs[R_RN];
            if (rn == 0) break;
            const uint32_t *rlist = p.list, *rcount = p.s + R_RN;
            uint32_t rcnt = rn;
            if (gated) {
                // the network defers the recomputes it expects to find far above the level
                if ((rc = gate_pass(ctx, g, gate->mlp, gate->margin, p.alive, p.dm, p.list, rn, p.lb, p.d, p.dirty,
                                    p.part, p.s, gate_x, gate_y, gate_list)))
                    return rc;
                e = hipMemcpyAsync(hs + R_GKEEP, p.s + R_GKEEP, 4, hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) return check_hip(ctx, e, "gate readback");
                rcnt = hs[R_GKEEP];
                st_local.gate_deferrals += rn - rcnt;
                if (rcnt == 0) continue;
                rlist = gate_list;
                rcount = p.s + R_GKEEP;
            }
            if (lazy) {
                // the same BFS gives the exact (h-1)-degrees at its level h - 1
                std::vector<uint32_t *> lv(h, nullptr);
                lv[h - 2] = p.dm;
                lv[h - 1] = p.d;
                if ((rc = msbfs_all_levels(ctx, g, p.alive, h, rlist, rcnt, lv.data()))) return rc;
                st_local.hm1_recomputes += rcnt;
            } else if ((rc = msbfs_degrees(ctx, g, p.alive, h, rlist, rcnt, nullptr, 1, p.d))) {
                return rc;
            }
            hipLaunchKernelGGL(set_flag_kernel, dim3(grid_n), dim3(256), 0, st, rlist, rcount, p.dirty, (uint8_t)0);
            st_local.h_recomputes += rcnt;
        }
        if (done) break;
        if ((rc = peel_round_common(ctx, g, h, p, bounded, r, core, peel_round, grid_n, !lazy))) return rc;
        if (lazy) {
            // every range below comes from the device counters
            hipLaunchKernelGGL(dm_decrement_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h, p.dm);
            hipLaunchKernelGGL(lower_bound_kernel, dim3(wgrid), dim3(256), 0, st, p.queue, p.s, (int)h, n,
                               g->row_ptr, g->col, p.alive, p.dm, p.lb, (const uint8_t *)p.dirty,
                               (const uint32_t *)p.d, p.lbx);
            hipLaunchKernelGGL(finish_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h, p.mark, p.dirty,
                               (uint8_t)1);
            hipLaunchKernelGGL(round_tally_kernel, dim3(1), dim3(64), 0, st, p.s, (int)h);
            pending = true;
            ++r;
            continue;
        }
        const uint32_t np = hs[R_CNT];
        uint32_t e_hm2 = 0, e_h = 0;
        for (uint32_t j = 0; j <= h; ++j) {
            if (j + 1 < h) e_hm2 += hs[R_CNT + j];
            e_h += hs[R_CNT + j];
        }
        const uint32_t na = e_h - np;
        if (!bounded) {
            uint32_t e_hm1 = 0;  // P and the vertices within h - 1 hops of it
            for (uint32_t j = 0; j < h; ++j) e_hm1 += hs[R_CNT + j];
            if (na && local && 2ull * e_hm1 < na) {
                // two bounded BFS from the vertices within h-1 hops of P (ordered
                // by distance), inside the region before and after removal; each
                // affected u loses what it reached before but not after
                hipLaunchKernelGGL(region_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h, p.mark,
                                   region_pre, region_post, cnt_pre, cnt_post, 1);
                RowCount rcnt{p.queue + np, na, p.mark, p.s + R_CNT, h, cnt_pre};
                if ((rc = msbfs_row_counts(ctx, g, region_pre, h, p.queue, e_hm1, rcnt))) return rc;
                rcnt.acc = cnt_post;
                if ((rc = msbfs_row_counts(ctx, g, region_post, h, p.queue, e_hm1, rcnt))) return rc;
                hipLaunchKernelGGL(local_apply_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h,
                                   cnt_pre, cnt_post, p.d);
                hipLaunchKernelGGL(region_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h, p.mark,
                                   region_pre, region_post, cnt_pre, cnt_post, 0);
                st_local.local_rounds += 1;
                st_local.local_sources += 2ull * e_hm1;
            } else if (na) {
                if ((rc = msbfs_degrees(ctx, g, p.alive, h, p.queue + np, na, nullptr, 1, p.d))) return rc;
                st_local.h_recomputes += na;
            }
            hipLaunchKernelGGL(finish_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h, p.mark,
                               (uint8_t *)nullptr, (uint8_t)0);
        } else {
            // (h-1)-degree bounds change only within h-1 hops of P: recomputed
            // exactly within h-2 hops; the ring at h-1 lost at most |P| (kill)
            if (e_hm2 > np && lazy) {
                hipLaunchKernelGGL(dm_decrement_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h, p.dm);
            } else if (e_hm2 > np) {
                if ((rc = msbfs_degrees(ctx, g, p.alive, h - 1, p.queue + np, e_hm2 - np, nullptr, 1, p.dm)))
                    return rc;
                st_local.hm1_recomputes += e_hm2 - np;
            }
            // bounds and dirtiness change only within h hops of P
            if (na)
                hipLaunchKernelGGL(lower_bound_kernel, dim3(wgrid), dim3(256), 0, st, p.queue, p.s, (int)h, n,
                                   g->row_ptr, g->col, p.alive, p.dm, p.lb, (const uint8_t *)p.dirty,
                                   (const uint32_t *)p.d, p.lbx);
            hipLaunchKernelGGL(finish_kernel, dim3(grid_n), dim3(256), 0, st, p.queue, p.s, (int)h, p.mark, p.dirty,
                               (uint8_t)1);
        }
        st_local.affected_total += na;
        left -= np;
        ++r;
        report_progress(ctx, &last_report, r, (uint64_t)n - left, hs[R_K]);
    }
    if (pending) {
        // stopped by the round limit: read the last round's counters
        hipError_t e = hipMemcpyAsync(hs, p.s, (size_t)R_CNT * 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return check_hip(ctx, e, "last round readback");
        if ((rc = take_tally())) return rc;
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "peel end");
    if ((e = hipGetLastError()) != hipSuccess) return check_hip(ctx, e, "peel launch");
    st_local.rounds = r;
    st_local.max_level = hs[R_K];
    st_local.width_words = (uint32_t)ctx->max_width;
    st_local.wall_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st_local;
    return KHC_OK;
}
