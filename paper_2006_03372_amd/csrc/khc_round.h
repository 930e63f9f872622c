// Kernels of one level-synchronous peeling round, shared by the exact
// host-driven driver and the approximate driver.
//
// A round: the level k = max(k, min over live v of key(v)), P = live
// vertices with key <= k (they get core k), the vertices within h hops of P
// in the graph before removal (Observations 1-2 of Section IV-A, applied to
// the removed set), then removal of P.
//
// Round scalars (u32 array s): s[R_K] level, s[R_KNEW] level of this round,
// s[R_RN] recompute count, s[R_LIVE] live vertices, s[R_CNT + j] vertices put
// on the queue at BFS level j (level 0 = P); u64 array s64[j]: their total
// degree.  queue = [P | level 1 | ... | level h].  mark[v] = level + 1 of
// the level v was queued at (0: not queued).  The minimum key comes from
// per-block partial minima (kMinBlocks entries) that each consumer reduces
// itself, so no reset launch is needed between rounds.
#pragma once

#include "khc_internal.h"

namespace khc {
namespace rnd {
namespace {  // each including source gets its own copy of the kernels

constexpr int kMinBlocks = 1024;
enum : int { R_K = 0, R_KNEW = 1, R_RN = 2, R_LIVE = 3, R_CNT = 8 };

// Per-block minimum of key(v) = (dirty && dirty[v]) ? lb[v] : d[v] over
// live v into part[blockIdx.x] (grid must be kMinBlocks).  Block 0 also
// clears the counters of the coming select / collect.
__global__ void keymin_kernel(uint32_t n, const uint8_t *alive, const uint8_t *dirty, const uint32_t *d,
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
            s64[j] = 0;
            if (j == 0) s[R_RN] = 0;
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

// Dirty live vertices whose lower bound reached the level.
[[maybe_unused]] __global__ void collect_kernel(uint32_t n, const uint8_t *alive, const uint8_t *dirty, const uint32_t *lb,
                               const uint32_t *part, uint32_t *list, uint32_t *s) {
    const uint32_t k = block_level(part, s);
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const bool take = v < n && alive[v] && dirty[v] && lb[v] <= k;
    const uint32_t at = wave_reserve(take, &s[R_RN]);
    if (take) list[at] = v;
}

// P = live (clean) vertices whose key <= k: core k, removal round r, queued
// at level 0 with mark 1.
__global__ void select_kernel(uint32_t n, const uint64_t *row_ptr, const uint8_t *alive, const uint8_t *dirty,
                              const uint32_t *d, const uint32_t *part, uint32_t *mark, uint32_t *core,
                              uint32_t *round, uint32_t r, uint32_t *queue, uint32_t *s,
                              unsigned long long *s64) {
    const uint32_t k = block_level(part, s);
    if (blockIdx.x == 0 && threadIdx.x == 0) s[R_KNEW] = k;
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const bool take = v < n && alive[v] && !(dirty && dirty[v]) && d[v] <= k;
    const uint32_t at = wave_reserve(take, &s[R_CNT]);
    if (take) {
        core[v] = k;
        if (round) round[v] = r;
        mark[v] = 1;
        queue[at] = v;
        atomicAdd(&s64[0], (unsigned long long)(row_ptr[v + 1] - row_ptr[v]));
    }
}

// Level L of the affected-set BFS from P over the live graph (P still
// live).  Push (one wavefront per queued row of level L-1, atomics on the
// marks) while that level's rows have few arcs; otherwise pull (one thread
// per unqueued live vertex, looking for a neighbour of level L-1).
__global__ void affected_kernel(uint32_t n, uint64_t nnz, const uint64_t *row_ptr, const uint32_t *col,
                                const uint8_t *alive, uint32_t *mark, uint32_t *queue, uint32_t *s,
                                unsigned long long *s64, int L) {
    uint32_t begin = 0;
    for (int j = 0; j + 1 < L; ++j) begin += s[R_CNT + j];
    const uint32_t end = begin + s[R_CNT + L - 1];
    const bool pull = s64[L - 1] * 8ull > nnz;
    const uint32_t tag = (uint32_t)L + 1u;
    if (pull) {
        for (uint32_t y0 = blockIdx.x * blockDim.x; y0 < n; y0 += gridDim.x * blockDim.x) {
            const uint32_t y = y0 + threadIdx.x;
            bool take = false;
            uint64_t dy = 0;
            if (y < n && alive[y] && mark[y] == 0u) {
                const uint64_t rb = row_ptr[y], re = row_ptr[y + 1];
                for (uint64_t a = rb; a < re; ++a) {
                    if (mark[col[a]] == tag - 1u) {
                        take = true;
                        break;
                    }
                }
                dy = re - rb;
            }
            const uint32_t at = wave_reserve(take, &s[R_CNT + L]);
            if (take) {
                mark[y] = tag;
                queue[end + at] = y;
                atomicAdd(&s64[L], (unsigned long long)dy);
            }
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t i = begin + wave; i < end; i += nwaves) {
        const uint32_t x = queue[i];
        const uint64_t rb = row_ptr[x], re = row_ptr[x + 1];
        for (uint64_t a0 = rb; a0 < re; a0 += 64) {
            const uint64_t a = a0 + lane;
            bool take = false;
            uint32_t y = 0;
            uint64_t dy = 0;
            if (a < re) {
                y = col[a];
                take = alive[y] && mark[y] == 0u && atomicCAS(&mark[y], 0u, tag) == 0u;
                if (take) dy = row_ptr[y + 1] - row_ptr[y];
            }
            const uint32_t at = wave_reserve(take, &s[R_CNT + L]);
            if (take) {
                queue[end + at] = y;
                atomicAdd(&s64[L], (unsigned long long)dy);
            }
        }
    }
}

// Remove P; the level of this round becomes the level.
__global__ void kill_kernel(const uint32_t *queue, uint32_t *s, uint8_t *alive) {
    const uint32_t np = s[R_CNT];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x)
        alive[queue[i]] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s[R_K] = s[R_KNEW];
        s[R_LIVE] -= np;
    }
}

// Clear the marks of every queued vertex; optionally set flag[] on the
// affected part (queue entries after P).
__global__ void finish_kernel(const uint32_t *queue, const uint32_t *s, int h, uint32_t *mark, uint8_t *flag,
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
