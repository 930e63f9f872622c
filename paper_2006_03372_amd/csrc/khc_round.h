// Kernels of one level-synchronous peeling round, shared by the exact
// host-driven driver and the approximate driver.
//
// A round: the level k = max(k, min over live v of key(v)), P = live
// vertices with key <= k (they get core k), the vertices within h hops of P
// in the graph before removal (Observations 1-2 of Section IV-A, applied to
// the removed set), then removal of P.
//
// Round scalars (u32 array s): s[R_K] level, s[R_KNEW] level of this round,
// s[R_RN] recompute count, s[R_LIVE] live vertices, s[R_SMIN] (sampling
// mode) nearest queue level holding a sampled vertex, s[R_GKEEP] (learned
// gate) recomputes kept by the gate, s[R_PNP] / s[R_PNA] the removed and
// affected counts of the last round (kept for a later readback),
// s[R_CNT + j] vertices put
// on the queue at BFS level j (level 0 = P), s[R_CNT + h + 1 + j] push items
// of level j; u64 array s64[j]: total degree of the level-j vertices.
// queue = [P | level 1 | ... | level h]; a queued row with more than
// kPushArcs arcs is also listed as ceil(deg / kPushArcs) push items
// (row, piece) so that the next level's push splits it over wavefronts.
// mark[v] = level + 1 of the level v was queued at (0: not queued).  The
// minimum key comes from per-block partial minima (kMinBlocks entries) that
// each consumer reduces itself, so no reset launch is needed between rounds.
#pragma once

#include "khc_internal.h"

namespace khc {
namespace rnd {
namespace {  // each including source gets its own copy of the kernels

constexpr int kMinBlocks = 1024;
enum : int { R_K = 0, R_KNEW = 1, R_RN = 2, R_LIVE = 3, R_SMIN = 4, R_GKEEP = 5, R_PNP = 6, R_PNA = 7, R_CNT = 8 };
constexpr uint32_t kPushArcs = 256;  // arcs per push item

inline int round_nscal(uint32_t h) { return R_CNT + 2 * (int)h + 3; }
// byte size of the scalar block (u32 scalars, then the u64 degree sums)
inline size_t round_scalar_bytes(uint32_t h) { return (((size_t)round_nscal(h) * 4 + 63) / 64) * 64 + (size_t)(h + 2) * 8; }
inline unsigned long long *round_s64(void *s, uint32_t h) {
    return (unsigned long long *)((char *)s + (((size_t)round_nscal(h) * 4 + 63) / 64) * 64);
}
// push items a round can hold: every row's pieces at most once
inline size_t round_item_capacity(uint32_t n, uint64_t nnz) { return (size_t)(nnz / kPushArcs) + n + 8; }

// The graph as the round kernels read it: CSR plus the row schedule (light
// rows by descending degree, the first n_mid of them with more than kMidDeg
// arcs, the first n_nz with at least one; heavy rows cut into chunks).
struct RoundGraph {
    uint32_t n;
    uint64_t nnz;
    const uint64_t *row_ptr;
    const uint32_t *col;
    const uint32_t *light_rows, *heavy_rows, *chunk_heavy, *chunk_first;
    uint32_t n_mid, n_nz, n_chunks;
};

inline RoundGraph round_graph(const khc_graph *g) {
    return RoundGraph{g->n,          g->nnz,         g->row_ptr,   g->col,        g->light_rows, g->heavy_rows,
                      g->chunk_heavy, g->chunk_first, g->n_light_mid, g->n_light_nz, g->n_chunks};
}

// Per-block minimum of key(v) = (dirty && dirty[v]) ? lb[v] : d[v] over
// live v into part[blockIdx.x] (grid must be kMinBlocks).  Block 0 also
// clears the counters of the coming select / collect.
[[maybe_unused]] __global__ void keymin_kernel(uint32_t n, const uint8_t *alive, const uint8_t *dirty, const uint32_t *d,
                              const uint32_t *lb, uint32_t *part, uint32_t *s, unsigned long long *s64,
                              int h) {
    __shared__ uint32_t red[4];
    uint32_t m = 0xFFFFFFFFu;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (!alive[v]) continue;
        const uint32_t key = (dirty && dirty[v]) ? lb[v] : d[v];
        m = key < m ? key : m;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(m, off, 64);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = red[w] < m ? red[w] : m;
        part[blockIdx.x] = m;
    }
    if (blockIdx.x == 0)
        for (int j = threadIdx.x; j <= h; j += blockDim.x) {
            s[R_CNT + j] = 0;
            s[R_CNT + h + 1 + j] = 0;
            s64[j] = 0;
            if (j == 0) {
                s[R_RN] = 0;
                s[R_GKEEP] = 0;
            }
        }
}

// k = max(K, min of the partial minima), computed by each block.
__device__ __forceinline__ uint32_t block_level(const uint32_t *part, const uint32_t *s) {
    __shared__ uint32_t red[4];
    uint32_t m = 0xFFFFFFFFu;
    for (int i = threadIdx.x; i < kMinBlocks; i += blockDim.x) m = part[i] < m ? part[i] : m;
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(m, off, 64);
        m = o < m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = red[w] < m ? red[w] : m;
    const uint32_t k = s[R_K];
    return (m != 0xFFFFFFFFu && m > k) ? m : k;
}

__device__ __forceinline__ uint32_t wave_reserve(bool take, uint32_t *counter) {
    const uint64_t m = __ballot(take);
    if (!m) return 0;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__builtin_popcountll(m));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
}

// List row x (degree deg, queued at level L) as push items when it is heavy.
__device__ __forceinline__ void add_items(uint32_t x, uint64_t deg, int L, int h, uint32_t *s, uint2 *items) {
    if (deg <= kPushArcs) return;
    const uint32_t cnt = (uint32_t)((deg + kPushArcs - 1) / kPushArcs);
    uint32_t base = 0;
    for (int j = 0; j < L; ++j) base += s[R_CNT + h + 1 + j];
    base += atomicAdd(&s[R_CNT + h + 1 + L], cnt);
    for (uint32_t c = 0; c < cnt; ++c) items[base + c] = make_uint2(x, c);
}

// Dirty live vertices whose lower bound reached the level while their stale
// h-degree (an upper bound) is still above it: only for these is it open
// whether they leave at this level.
[[maybe_unused]] __global__ void collect_kernel(uint32_t n, const uint8_t *alive, const uint8_t *dirty,
                                                const uint32_t *lb, const uint32_t *d, const uint32_t *part,
                                                uint32_t *list, uint32_t *s) {
    const uint32_t k = block_level(part, s);
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const bool take = v < n && alive[v] && dirty[v] && lb[v] <= k && d[v] > k;
    const uint32_t at = wave_reserve(take, &s[R_RN]);
    if (take) list[at] = v;
}

// P = live vertices with d <= k: core k, removal round r, queued at level 0
// with mark 1.  d is exact for clean vertices and an upper bound for dirty
// ones, so a dirty vertex with d <= k leaves at this level without a
// recompute; the dirty vertices left open were resolved by the cleaning
// loop (their lower bound exceeds k).
[[maybe_unused]] __global__ void select_kernel(uint32_t n, const uint64_t *row_ptr, const uint8_t *alive, const uint8_t *dirty,
                              const uint32_t *d, const uint32_t *part, uint32_t *mark, uint32_t *core,
                              uint32_t *round, uint32_t r, uint32_t *queue, uint32_t *s,
                              unsigned long long *s64, uint2 *items, int h) {
    const uint32_t k = block_level(part, s);
    if (blockIdx.x == 0 && threadIdx.x == 0) s[R_KNEW] = k;
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    (void)dirty;
    const bool take = v < n && alive[v] && d[v] <= k;
    const uint32_t at = wave_reserve(take, &s[R_CNT]);
    if (take) {
        core[v] = k;
        if (round) round[v] = r;
        mark[v] = 1;
        queue[at] = v;
        const uint64_t dv = row_ptr[v + 1] - row_ptr[v];
        atomicAdd(&s64[0], (unsigned long long)dv);
        add_items(v, dv, 0, h, s, items);
    }
}

// Queue y at level L (its mark already set): append, add its degree and its
// push items.  Called by the lanes that take a vertex; wave-aggregated.
__device__ __forceinline__ void queue_take(bool take, uint32_t y, const RoundGraph &g, int L, int h, uint32_t end,
                                           uint32_t *queue, uint32_t *s, unsigned long long *s64, uint2 *items) {
    const uint32_t at = wave_reserve(take, &s[R_CNT + L]);
    if (take) {
        queue[end + at] = y;
        const uint64_t dy = g.row_ptr[y + 1] - g.row_ptr[y];
        atomicAdd(&s64[L], (unsigned long long)dy);
        add_items(y, dy, L, h, s, items);
    }
}

// Level L of the affected-set BFS from P over the live graph (P still
// live).  Push while the rows of level L-1 have few arcs: light rows of
// level L-1 by groups of 16 lanes, heavy ones as kPushArcs-arc items by
// whole wavefronts, marks claimed with compare-and-swap.  Otherwise pull:
// every unqueued live row looks for a neighbour of level L-1, heavy rows by
// chunks (one wavefront each), rows above kMidDeg arcs by groups of 8
// lanes, the rest one lane each, all stopping at the first hit.
[[maybe_unused]] __global__ void affected_kernel(RoundGraph g, const uint8_t *alive, uint32_t *mark, uint32_t *queue, uint32_t *s,
                                unsigned long long *s64, uint2 *items, int L, int h) {
    uint32_t begin = 0, ibegin = 0;
    for (int j = 0; j + 1 < L; ++j) {
        begin += s[R_CNT + j];
        ibegin += s[R_CNT + h + 1 + j];
    }
    const uint32_t end = begin + s[R_CNT + L - 1];
    const uint32_t iend = ibegin + s[R_CNT + h + 1 + L - 1];
    const bool pull = s64[L - 1] * 8ull > g.nnz;
    const uint32_t tag = (uint32_t)L + 1u;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    if (pull) {
        const uint32_t mid_units = (g.n_mid + 7) / 8;
        const uint32_t small_units = (g.n_nz - g.n_mid + 63) / 64;
        const uint32_t units = g.n_chunks + mid_units + small_units;
        for (uint32_t u = wave; u < units; u += nwaves) {
            bool take = false;
            uint32_t y = 0;
            if (u < g.n_chunks) {
                const uint32_t hr = g.chunk_heavy[u];
                y = g.heavy_rows[hr];
                if (alive[y] && mark[y] == 0u) {
                    const uint64_t re = g.row_ptr[y + 1];
                    const uint64_t a0 = g.row_ptr[y] + (uint64_t)(u - g.chunk_first[hr]) * kChunkArcs;
                    const uint64_t a1 = a0 + kChunkArcs < re ? a0 + kChunkArcs : re;
                    bool found = false;
                    for (uint64_t b = a0; b < a1; b += 64) {
                        const uint64_t a = b + lane;
                        const bool hit = a < a1 && mark[g.col[a]] == tag - 1u;
                        if (__ballot(hit)) {
                            found = true;
                            break;
                        }
                    }
                    take = found && lane == 0 && atomicCAS(&mark[y], 0u, tag) == 0u;
                }
            } else if (u < g.n_chunks + mid_units) {
                const uint32_t grp = lane >> 3, sub = lane & 7;
                const uint32_t i = (u - g.n_chunks) * 8 + grp;
                if (i < g.n_mid) {
                    y = g.light_rows[i];
                    if (alive[y] && mark[y] == 0u) {
                        const uint64_t rb = g.row_ptr[y], re = g.row_ptr[y + 1];
                        bool found = false;
                        for (uint64_t a0 = rb; a0 < re; a0 += 8) {
                            const uint64_t a = a0 + sub;
                            const bool hit = a < re && mark[g.col[a]] == tag - 1u;
                            if ((__ballot(hit) >> (grp * 8)) & 0xFFull) {
                                found = true;
                                break;
                            }
                        }
                        if (found && sub == 0) {
                            mark[y] = tag;  // the group is the only reader of row y
                            take = true;
                        }
                    }
                }
            } else {
                const uint32_t i = g.n_mid + (u - g.n_chunks - mid_units) * 64 + lane;
                if (i < g.n_nz) {
                    y = g.light_rows[i];
                    if (alive[y] && mark[y] == 0u) {
                        const uint64_t rb = g.row_ptr[y], re = g.row_ptr[y + 1];
                        for (uint64_t a = rb; a < re; ++a)
                            if (mark[g.col[a]] == tag - 1u) {
                                take = true;
                                break;
                            }
                        if (take) mark[y] = tag;
                    }
                }
            }
            queue_take(take, y, g, L, h, end, queue, s, s64, items);
        }
        return;
    }
    // push: 4 light rows per wavefront (16 lanes each), then the items
    const uint32_t light_units = (end - begin + 3) / 4;
    const uint32_t units = light_units + (iend - ibegin);
    for (uint32_t u = wave; u < units; u += nwaves) {
        uint64_t a0 = 0, a1 = 0;
        uint32_t step = 64, off = (uint32_t)lane;
        if (u < light_units) {
            const uint32_t i = begin + u * 4 + (lane >> 4);
            step = 16;
            off = lane & 15;
            if (i < end) {
                const uint32_t x = queue[i];
                a0 = g.row_ptr[x];
                a1 = g.row_ptr[x + 1];
                if (a1 - a0 > kPushArcs) a1 = a0;  // pushed by its items
            }
        } else {
            const uint2 it = items[ibegin + (u - light_units)];
            const uint64_t rb = g.row_ptr[it.x], re = g.row_ptr[it.x + 1];
            a0 = rb + (uint64_t)it.y * kPushArcs;
            a1 = a0 + kPushArcs < re ? a0 + kPushArcs : re;
        }
        // same trip count on every lane of the wavefront
        uint64_t len = a1 - a0, maxlen = len;
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t t = __shfl_xor(maxlen, o, 64);
            maxlen = t > maxlen ? t : maxlen;
        }
        for (uint64_t b = 0; b < maxlen; b += step) {
            const uint64_t a = a0 + b + off;
            bool take = false;
            uint32_t y = 0;
            if (b + off < len) {
                y = g.col[a];
                take = alive[y] && mark[y] == 0u && atomicCAS(&mark[y], 0u, tag) == 0u;
            }
            queue_take(take, y, g, L, h, end, queue, s, s64, items);
        }
    }
}

// Remove P; the level of this round becomes the level.  With dm (lower
// bounds on the (h-1)-degrees), the vertices at distance h-1 from P lower
// their bound by |P|: their (h-1)-ball reaches P only at its rim, so they
// can lose the vertices of P and nothing else.
[[maybe_unused]] __global__ void kill_kernel(const uint32_t *queue, uint32_t *s, uint8_t *alive, uint32_t *dm, int h) {
    const uint32_t np = s[R_CNT];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x)
        alive[queue[i]] = 0;
    if (dm && h >= 2) {
        uint32_t b = 0;
        for (int j = 0; j + 1 < h; ++j) b += s[R_CNT + j];
        const uint32_t e = b + s[R_CNT + h - 1];
        for (uint32_t i = b + blockIdx.x * blockDim.x + threadIdx.x; i < e; i += gridDim.x * blockDim.x) {
            const uint32_t u = queue[i];
            dm[u] = dm[u] > np ? dm[u] - np : 0u;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s[R_K] = s[R_KNEW];
        s[R_LIVE] -= np;
    }
}

// Clear the marks of every queued vertex; optionally set flag[] on the
// affected part (queue entries after P).
[[maybe_unused]] __global__ void finish_kernel(const uint32_t *queue, const uint32_t *s, int h, uint32_t *mark, uint8_t *flag,
                              uint8_t value) {
    uint32_t np = s[R_CNT], tot = 0;
    for (int j = 0; j <= h; ++j) tot += s[R_CNT + j];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += gridDim.x * blockDim.x) {
        const uint32_t v = queue[i];
        mark[v] = 0;
        if (flag && i >= np) flag[v] = value;
    }
}

}  // namespace
}  // namespace rnd
}  // namespace khc
