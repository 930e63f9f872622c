// Multi-source h-bounded BFS for h-degrees (gfx950).
//
// The h-degree d_v^h(G(S)) (Section II) of many sources is computed at once:
// one batch carries 64*W sources as bit lanes of W uint64 words per vertex.
// For every vertex y, vis[y] holds the lanes whose source has reached y and
// frt[y] the lanes that reached y at the previous hop.  One level of the
// bounded BFS is, for every live y,
//     new[y] = (OR over live neighbours x of frt[x]) AND NOT vis[y]
//     vis[y] |= new[y];  frt'[y] = new[y]
// and d^h(source of lane l) = sum over the h levels of the number of rows
// whose new[] has bit l set.  This transposes the paper's bitmap idea
// (Section IV-B: bit j of a vertex's bitmap marks reachability of the j-th
// vertex) -- here a bit marks a source lane, so one wide OR advances 64*W
// bounded BFS runs by one hop.
//
// Each level runs in one of two directions, chosen on the device from the
// size of the frontier (the total degree of the rows put on it by the
// previous level):
//  * pull: every live row gathers the frontier words of its neighbours.
//    Rows up to kHeavyRowArcs arcs are handled by one group of W/2 lanes
//    (16-byte loads; rows sorted by degree so a wavefront's rows are
//    alike); heavier rows are cut into chunks of kChunkArcs arcs that whole
//    workgroups OR together, the last chunk to finish completing the row.
//  * push: every frontier row ORs its non-zero words into its live
//    neighbours with atomics; the atomic's old value tells which bits are
//    new, so each (row, lane) is counted once.
// Workgroups are persistent and take work items from an atomic counter.
// Frontier rows of each level are also kept as a list, which drives the
// push direction and lets the batch clean up exactly the rows it touched:
// between batches vis and the three frontier buffers are all zero.
#include "khc_internal.h"

namespace khc {

namespace {

struct alignas(16) U2 {
    uint64_t a, b;
};

template <int WPL>
__device__ __forceinline__ void load_words(const uint64_t *p, uint64_t (&w)[WPL]) {
    if constexpr (WPL == 2) {
        U2 v = *reinterpret_cast<const U2 *>(p);
        w[0] = v.a;
        w[1] = v.b;
    } else {
        w[0] = *p;
    }
}

template <int WPL>
__device__ __forceinline__ void store_words(uint64_t *p, const uint64_t (&w)[WPL]) {
    if constexpr (WPL == 2) {
        U2 v;
        v.a = w[0];
        v.b = w[1];
        *reinterpret_cast<U2 *>(p) = v;
    } else {
        *p = w[0];
    }
}

constexpr int kPlanes = 8;            // bit-sliced per-lane counters hold up to 255
constexpr int kUnroll = 8;            // independent gathers in flight per lane
constexpr int kPushFactor = 16;       // push when frontier arcs * factor < all arcs
constexpr int kGrab = 4;              // push work grab: one frontier item per wavefront
constexpr uint32_t kPushChunk = 256;  // arcs per push item of a heavy frontier row
constexpr int kStage = 1024;          // LDS staging of frontier rows (pull levels)

// Frontier list of one level: every row once (q, count, total degree) and,
// for rows with more than kPushChunk arcs, one push item per kPushChunk arcs
// (row | chunk << 32) so heavy rows spread over many wavefronts.
struct Frontier {
    uint32_t *q;
    uint32_t *qcnt;
    unsigned long long *qdeg;
    uint64_t *hq;
    uint32_t *hcnt;
};

struct LevelParams {
    const uint64_t *row_ptr;
    const uint32_t *col;
    const uint8_t *alive;
    const uint32_t *light_rows;
    const uint32_t *heavy_rows;
    const uint32_t *chunk_heavy;
    const uint32_t *chunk_first;
    const uint64_t *frt_in;  // frontier of the previous level
    uint64_t *frt_out;       // frontier of this level (all zero on entry)
    uint64_t *frt_clr;       // buffer whose rows of q_clr are cleared here
    uint64_t *vis;
    const uint32_t *q_in;   // rows of the previous frontier
    const uint64_t *hq_in;  // push items of its heavy rows
    const uint32_t *qcnt_in;
    const uint32_t *hcnt_in;
    const unsigned long long *qdeg_in;
    Frontier out;           // this level's frontier
    const uint32_t *q_clr;  // rows of the frontier two levels back
    const uint32_t *qcnt_clr;
    uint32_t *fnz_out;  // 1 bit per vertex: row is on this level's frontier
    uint32_t *fnz_clr;
    uint64_t *hacc;
    uint32_t *hdone;
    uint32_t *work;    // work-item counter of this level
    uint32_t *counts;  // per-lane reached-vertex totals, summed over levels
    uint64_t nnz;
    uint32_t n;
    uint32_t n_light;
    uint32_t n_chunks;
};

// Add the WPL words of x to the bit-sliced counters (one ripple-carry add
// per word: plane k holds bit k of every bit position's count).
template <int WPL>
__device__ __forceinline__ void planes_add(uint64_t (&pl)[WPL][kPlanes], const uint64_t (&x)[WPL]) {
#pragma unroll
    for (int j = 0; j < WPL; ++j) {
        uint64_t c = x[j];
#pragma unroll
        for (int k = 0; k < kPlanes; ++k) {
            uint64_t t = pl[j][k] & c;
            pl[j][k] ^= c;
            c = t;
        }
    }
}

template <int WPL>
__device__ __forceinline__ void planes_flush(uint64_t (&pl)[WPL][kPlanes], uint32_t *s_counts,
                                             int word0) {
#pragma unroll
    for (int j = 0; j < WPL; ++j) {
        uint64_t any = 0;
#pragma unroll
        for (int k = 0; k < kPlanes; ++k) any |= pl[j][k];
        while (any) {
            int b = __builtin_ctzll(any);
            any &= any - 1;
            uint32_t c = 0;
#pragma unroll
            for (int k = 0; k < kPlanes; ++k) c |= (uint32_t)((pl[j][k] >> b) & 1u) << k;
            atomicAdd(&s_counts[(word0 + j) * 64 + b], c);
        }
#pragma unroll
        for (int k = 0; k < kPlanes; ++k) pl[j][k] = 0;
    }
}

__device__ __forceinline__ void count_word_bits(uint32_t *s_counts, int word, uint64_t bits) {
    while (bits) {
        int b = __builtin_ctzll(bits);
        bits &= bits - 1;
        atomicAdd(&s_counts[word * 64 + b], 1u);
    }
}

// Push items of a heavy frontier row (called by the lane that lists it).
__device__ __forceinline__ void add_push_items(const Frontier &f, uint32_t y, uint64_t dy) {
    if (dy <= kPushChunk) return;
    const uint32_t nch = (uint32_t)((dy + kPushChunk - 1) / kPushChunk);
    const uint32_t at = atomicAdd(f.hcnt, nch);
    for (uint32_t c = 0; c < nch; ++c) f.hq[at + c] = (uint64_t)y | ((uint64_t)c << 32);
}

// Wave-aggregated append straight to the global frontier list.  Must be
// reached by every lane of the wavefront.
__device__ __forceinline__ void append_direct(bool take, uint32_t y, uint64_t dy, const Frontier &f) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    uint64_t dsum = take ? dy : 0;
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off, 64);
    uint32_t base = 0;
    if (lane == leader) {
        base = atomicAdd(f.qcnt, (uint32_t)__builtin_popcountll(m));
        atomicAdd(f.qdeg, (unsigned long long)dsum);
    }
    base = __shfl(base, leader, 64);
    if (take) {
        f.q[base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = y;
        add_push_items(f, y, dy);
    }
}

// Wave-aggregated append to the workgroup's LDS staging list.
__device__ __forceinline__ void append_staged(bool take, uint32_t y, uint32_t *s_stage,
                                              uint32_t *s_sn) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(s_sn, (uint32_t)__builtin_popcountll(m));
    base = __shfl(base, leader, 64);
    if (take) s_stage[base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = y;
}

// Move the staged rows to the global frontier list (whole workgroup; one
// pair of global atomics per flush).
__device__ void flush_staged(const Frontier &f, const uint64_t *row_ptr, uint32_t *s_stage,
                             uint32_t *s_sn, uint32_t *s_base, unsigned long long *s_deg) {
    __syncthreads();
    const uint32_t cnt = *s_sn;
    if (cnt == 0) return;
    if (threadIdx.x == 0) {
        *s_base = atomicAdd(f.qcnt, cnt);
        *s_deg = 0;
    }
    __syncthreads();
    const uint32_t base = *s_base;
    uint64_t dsum = 0;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        const uint32_t y = s_stage[i];
        const uint64_t dy = row_ptr[y + 1] - row_ptr[y];
        f.q[base + i] = y;
        add_push_items(f, y, dy);
        dsum += dy;
    }
    for (int off = 32; off > 0; off >>= 1) dsum += __shfl_xor(dsum, off, 64);
    if ((threadIdx.x & 63) == 0 && dsum) atomicAdd(s_deg, (unsigned long long)dsum);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(f.qdeg, *s_deg);
        *s_sn = 0;
    }
    __syncthreads();
}

// Push one frontier row x over its arcs [ab, ae): OR its non-zero words
// into live neighbours; bits the atomic shows as new are counted and put
// on this level's frontier.  One wavefront, lanes over (arc, word) pairs.
template <int W, bool LAST>
__device__ void push_range(const LevelParams &p, uint32_t x, uint64_t ab, uint64_t ae,
                           uint32_t *s_counts) {
    const int lane = threadIdx.x & 63;
    const uint64_t myw = lane < W ? p.frt_in[(size_t)x * W + lane] : 0ull;
    const uint64_t nzmask = __ballot(myw != 0);
    const uint32_t nz = (uint32_t)__builtin_popcountll(nzmask);
    const uint64_t pairs = (ae - ab) * nz;
    for (uint64_t base = 0; base < pairs; base += 64) {
        const uint64_t pr = base + lane;
        bool take = false;
        uint32_t y = 0;
        uint64_t dy = 0;
        if (pr < pairs) {
            const uint64_t arc = pr / nz;
            uint32_t k = (uint32_t)(pr - arc * nz);
            uint64_t mm = nzmask;
            for (; k > 0; --k) mm &= mm - 1;  // k-th set bit
            const int w = __builtin_ctzll(mm);
            y = p.col[ab + arc];
            if (!p.alive || p.alive[y]) {
                const uint64_t bits = p.frt_in[(size_t)x * W + w];
                uint64_t *vp = p.vis + (size_t)y * W + w;
                const uint64_t nb = bits & ~*vp;
                if (nb) {
                    const uint64_t tn =
                        nb & ~(uint64_t)atomicOr((unsigned long long *)vp, (unsigned long long)nb);
                    if (tn) {
                        count_word_bits(s_counts, w, tn);
                        if constexpr (!LAST)
                            atomicOr((unsigned long long *)(p.frt_out + (size_t)y * W + w),
                                     (unsigned long long)tn);
                        const uint32_t ybit = 1u << (y & 31);
                        if (!(atomicOr(&p.fnz_out[y >> 5], ybit) & ybit)) {
                            take = true;
                            dy = p.row_ptr[y + 1] - p.row_ptr[y];
                        }
                    }
                }
            }
        }
        append_direct(take, y, dy, p.out);
    }
}

template <int W, bool LAST>
__global__ __launch_bounds__(kBlockThreads) void level_kernel(LevelParams p) {
    using L = RowLayout<W>;
    constexpr int WPL = L::WPL, LPR = L::LPR, RPW = L::RPW, GROUPS = L::GROUPS;
    // light rows handled per work item: several passes of all lane groups
    constexpr int PASSES = GROUPS >= 64 ? 1 : 64 / GROUPS;
    __shared__ uint64_t s_red[GROUPS * W];
    __shared__ uint64_t s_fin[W];
    __shared__ uint32_t s_counts[64 * W];
    __shared__ uint32_t s_stage[LAST ? 1 : kStage];
    __shared__ uint32_t s_sn, s_base, s_item, s_flag;
    __shared__ unsigned long long s_deg;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lig = lane % LPR;  // lane within its row group
    const int group = wave * RPW + lane / LPR;
    const size_t gstride = (size_t)gridDim.x * kBlockThreads;
    const size_t gtid = (size_t)blockIdx.x * kBlockThreads + tid;

    // Clear the rows of the frontier two levels back: its buffer and map
    // are written by the next level.
    if (p.q_clr) {
        const uint32_t nclr = *p.qcnt_clr;
        for (size_t i = gtid; i < (size_t)nclr * W; i += gstride) {
            const uint32_t y = p.q_clr[i / W];
            p.frt_clr[(size_t)y * W + (i % W)] = 0;
        }
        for (size_t i = gtid; i < nclr; i += gstride) p.fnz_clr[p.q_clr[i] >> 5] = 0;
    }

    for (int i = tid; i < 64 * W; i += kBlockThreads) s_counts[i] = 0;
    if (tid == 0) s_sn = 0;
    uint64_t pl[WPL][kPlanes];
#pragma unroll
    for (int j = 0; j < WPL; ++j)
#pragma unroll
        for (int k = 0; k < kPlanes; ++k) pl[j][k] = 0;
    uint32_t pcount = 0;

    const bool push = (unsigned long long)(*p.qdeg_in) * kPushFactor < (unsigned long long)p.nnz;
    const uint32_t qn_in = *p.qcnt_in;
    const uint32_t hn_in = *p.hcnt_in;
    const uint32_t light_grabs = (qn_in + kGrab - 1) / kGrab;
    const uint32_t n_items = push ? light_grabs + (hn_in + kGrab - 1) / kGrab
                                  : p.n_chunks + (p.n_light + GROUPS * PASSES - 1) / (GROUPS * PASSES);
    __syncthreads();

    for (;;) {
        if (tid == 0) s_item = atomicAdd(p.work, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= n_items) break;

        if (push) {
            // ---- push: one frontier item per wavefront ----
            if (item < light_grabs) {
                const uint32_t qi = item * kGrab + wave;
                if (qi < qn_in) {
                    const uint32_t x = p.q_in[qi];
                    const uint64_t rb = p.row_ptr[x], re = p.row_ptr[x + 1];
                    if (re - rb <= kPushChunk) push_range<W, LAST>(p, x, rb, re, s_counts);
                }
            } else {
                const uint32_t hi = (item - light_grabs) * kGrab + wave;
                if (hi < hn_in) {
                    const uint64_t it = p.hq_in[hi];
                    const uint32_t x = (uint32_t)it;
                    const uint64_t rb = p.row_ptr[x], re = p.row_ptr[x + 1];
                    const uint64_t ab = rb + (it >> 32) * kPushChunk;
                    const uint64_t ae = ab + kPushChunk < re ? ab + kPushChunk : re;
                    push_range<W, LAST>(p, x, ab, ae, s_counts);
                }
            }
        } else if (item < p.n_chunks) {
            // ---- pull, one chunk of a heavy row, whole workgroup ----
            const uint32_t hi = p.chunk_heavy[item];
            const uint32_t y = p.heavy_rows[hi];
            const bool live = !p.alive || p.alive[y];
            if (live) {
                const uint32_t c0 = p.chunk_first[hi];
                const uint32_t nch = p.chunk_first[hi + 1] - c0;
                const uint64_t rb = p.row_ptr[y], re = p.row_ptr[y + 1];
                const uint64_t b = rb + (uint64_t)(item - c0) * kChunkArcs;
                const uint64_t e = (b + kChunkArcs < re) ? b + kChunkArcs : re;
                uint64_t acc[WPL];
#pragma unroll
                for (int j = 0; j < WPL; ++j) acc[j] = 0;
                uint64_t a = b + group;
                for (; a + (uint64_t)(kUnroll - 1) * GROUPS < e; a += (uint64_t)kUnroll * GROUPS) {
                    uint32_t xs[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) xs[u] = p.col[a + (uint64_t)u * GROUPS];
                    uint64_t t[kUnroll][WPL];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        load_words<WPL>(p.frt_in + (size_t)xs[u] * W + lig * WPL, t[u]);
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                        for (int j = 0; j < WPL; ++j) acc[j] |= t[u][j];
                }
                for (; a < e; a += GROUPS) {
                    uint64_t t[WPL];
                    load_words<WPL>(p.frt_in + (size_t)p.col[a] * W + lig * WPL, t);
#pragma unroll
                    for (int j = 0; j < WPL; ++j) acc[j] |= t[j];
                }
#pragma unroll
                for (int j = 0; j < WPL; ++j) s_red[group * W + lig * WPL + j] = acc[j];
                __syncthreads();
                if (tid < W) {
                    uint64_t r = 0;
                    for (int g = 0; g < GROUPS; ++g) r |= s_red[g * W + tid];
                    s_fin[tid] = r;
                }
                __syncthreads();
                bool finalize = true;
                if (nch > 1) {
                    if (tid < W && s_fin[tid])
                        atomicOr((unsigned long long *)&p.hacc[(size_t)hi * W + tid],
                                 (unsigned long long)s_fin[tid]);
                    __threadfence();
                    __syncthreads();
                    if (tid == 0) s_flag = (atomicAdd(&p.hdone[hi], 1u) == nch - 1) ? 1u : 0u;
                    __syncthreads();
                    finalize = s_flag != 0;
                    if (finalize) {
                        __threadfence();
                        if (tid < W)
                            s_fin[tid] = atomicExch((unsigned long long *)&p.hacc[(size_t)hi * W + tid], 0ull);
                        if (tid == 0) atomicExch(&p.hdone[hi], 0u);
                        __syncthreads();
                    }
                }
                if (finalize && tid < 64) {
                    // wave 0 completes the row: lane t < W owns word t
                    uint64_t nw = 0;
                    if (tid < W) {
                        const uint64_t v = p.vis[(size_t)y * W + tid];
                        nw = s_fin[tid] & ~v;
                        if (nw) {
                            count_word_bits(s_counts, tid, nw);
                            if constexpr (!LAST) {
                                p.frt_out[(size_t)y * W + tid] = nw;
                                p.vis[(size_t)y * W + tid] = v | nw;
                            }
                        }
                    }
                    if constexpr (!LAST) {
                        const bool any = __ballot(nw != 0) != 0;
                        if (tid == 0 && any) atomicOr(&p.fnz_out[y >> 5], 1u << (y & 31));
                        append_staged(tid == 0 && any, y, s_stage, &s_sn);
                    }
                }
            }
        } else {
            // ---- pull, light rows: one lane group per row ----
            const uint32_t tile = item - p.n_chunks;
            for (int pass = 0; pass < PASSES; ++pass) {
                const uint32_t idx = (tile * PASSES + pass) * GROUPS + group;
                bool valid = idx < p.n_light;
                const uint32_t y = valid ? p.light_rows[idx] : 0u;
                if (valid && p.alive && !p.alive[y]) valid = false;
                uint64_t acc[WPL];
#pragma unroll
                for (int j = 0; j < WPL; ++j) acc[j] = 0;
                if (valid) {
                    const uint64_t rb = p.row_ptr[y], re = p.row_ptr[y + 1];
                    uint64_t a = rb;
                    for (; a + kUnroll <= re; a += kUnroll) {
                        uint32_t xs[kUnroll];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u) xs[u] = p.col[a + u];
                        uint64_t t[kUnroll][WPL];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            load_words<WPL>(p.frt_in + (size_t)xs[u] * W + lig * WPL, t[u]);
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                            for (int j = 0; j < WPL; ++j) acc[j] |= t[u][j];
                    }
                    for (; a < re; ++a) {
                        uint64_t t[WPL];
                        load_words<WPL>(p.frt_in + (size_t)p.col[a] * W + lig * WPL, t);
#pragma unroll
                        for (int j = 0; j < WPL; ++j) acc[j] |= t[j];
                    }
                }
                uint64_t v[WPL], nw[WPL];
                if (valid) {
                    load_words<WPL>(p.vis + (size_t)y * W + lig * WPL, v);
                } else {
#pragma unroll
                    for (int j = 0; j < WPL; ++j) v[j] = ~0ull;
                }
                uint64_t any = 0;
#pragma unroll
                for (int j = 0; j < WPL; ++j) {
                    nw[j] = acc[j] & ~v[j];
                    any |= nw[j];
                }
                planes_add<WPL>(pl, nw);
                if (++pcount == (1u << kPlanes) - 1u) {
                    planes_flush<WPL>(pl, s_counts, lig * WPL);
                    pcount = 0;
                }
                if constexpr (!LAST) {
                    if (any) {
                        uint64_t vv[WPL];
#pragma unroll
                        for (int j = 0; j < WPL; ++j) vv[j] = v[j] | nw[j];
                        store_words<WPL>(p.frt_out + (size_t)y * W + lig * WPL, nw);
                        store_words<WPL>(p.vis + (size_t)y * W + lig * WPL, vv);
                    }
                    const uint64_t m = __ballot(any != 0);
                    const uint64_t gmask = (LPR == 64) ? ~0ull : ((1ull << LPR) - 1ull);
                    const int gshift = (lane / LPR) * LPR;
                    const bool lead = valid && lig == 0 && ((m >> gshift) & gmask);
                    if (lead) atomicOr(&p.fnz_out[y >> 5], 1u << (y & 31));
                    append_staged(lead, y, s_stage, &s_sn);
                }
            }
        }
        __syncthreads();
        if constexpr (!LAST) {
            // at most 256 rows are staged per work item
            if (s_sn > kStage - 256) flush_staged(p.out, p.row_ptr, s_stage, &s_sn, &s_base, &s_deg);
        }
    }

    if constexpr (!LAST) flush_staged(p.out, p.row_ptr, s_stage, &s_sn, &s_base, &s_deg);
    planes_flush<WPL>(pl, s_counts, lig * WPL);
    __syncthreads();
    for (int i = tid; i < 64 * W; i += kBlockThreads)
        if (s_counts[i]) atomicAdd(&p.counts[i], s_counts[i]);
}

// Reset the per-batch counters: level work counters, frontier list sizes
// and degree totals, per-lane counts.
__global__ void batch_reset_kernel(uint32_t *work, uint32_t *qcnt, uint32_t *hcnt,
                                   unsigned long long *qdeg, int nlev, uint32_t *counts, int ncounts) {
    for (int i = threadIdx.x; i < nlev; i += blockDim.x) {
        work[i] = 0;
        qcnt[i] = 0;
        hcnt[i] = 0;
        qdeg[i] = 0;
    }
    for (int i = threadIdx.x; i < ncounts; i += blockDim.x) counts[i] = 0;
}

// Put source lane l on its vertex: vis and the level-0 frontier get bit l,
// and the vertex becomes entry l of the level-0 frontier list.  A dead
// source is listed but not seeded; its lane stays empty and reports 0.
// srcs == null means the implicit list first, first+1, ...
__global__ void batch_seed_kernel(const uint32_t *srcs, uint32_t first, uint32_t cnt, int W,
                                  const uint8_t *alive, const uint64_t *row_ptr, uint64_t *vis,
                                  uint64_t *f0, uint32_t *fnz0, Frontier f) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l == 0) *f.qcnt = cnt;
    if (l >= cnt) return;
    const uint32_t s = srcs ? srcs[first + l] : first + l;
    f.q[l] = s;
    if (alive && !alive[s]) return;
    const uint64_t bit = 1ull << (l & 63);
    // sources are distinct vertices, so each (vertex, word) has one writer
    vis[(size_t)s * W + (l >> 6)] |= bit;
    f0[(size_t)s * W + (l >> 6)] |= bit;
    atomicOr(&fnz0[s >> 5], 1u << (s & 31));
    const uint64_t ds = row_ptr[s + 1] - row_ptr[s];
    atomicAdd(f.qdeg, (unsigned long long)ds);
    add_push_items(f, s, ds);
}

// Zero the W words of every row on a frontier list in `buf` (and, if given,
// the row's word of a frontier map).
__global__ void clear_rows_kernel(const uint32_t *q, const uint32_t *qcnt, uint64_t *buf, int W,
                                  uint32_t *fnz) {
    const uint32_t cnt = *qcnt;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)cnt * W; i += stride)
        buf[(size_t)q[i / W] * W + (i % W)] = 0;
    if (fnz)
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride)
            fnz[q[i] >> 5] = 0;
}

// d = number of vertices other than the source that its lane reached.
__global__ void batch_scatter_kernel(const uint32_t *srcs, uint32_t first, uint32_t cnt,
                                     const uint32_t *counts, uint32_t *deg_list, uint32_t *deg_full) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= cnt) return;
    const uint32_t d = counts[l];
    if (deg_full) {
        const uint32_t s = srcs ? srcs[first + l] : first + l;
        deg_full[s] = d;
    } else {
        deg_list[first + l] = d;
    }
}

// Scanned-arc totals: for every source lane, the sum over the vertices it
// has reached (within h-1 hops, itself included) of their live degree, i.e.
// the arcs a scalar bounded BFS from that source examines.  One thread per
// (listed row, word); a row may be listed at several levels, so each vis
// word is claimed (and cleared) with an atomic exchange and counted once.
// LDS totals per lane, flushed with 64-bit atomics.
template <int W>
__global__ __launch_bounds__(256) void scanned_arcs_kernel(const uint32_t *const *queues,
                                                           const uint32_t *qcnt, int nq,
                                                           const uint64_t *row_ptr,
                                                           const uint32_t *col, const uint8_t *alive,
                                                           uint64_t *vis,
                                                           unsigned long long *te) {
    __shared__ unsigned long long s_te[64 * W];
    for (int i = threadIdx.x; i < 64 * W; i += blockDim.x) s_te[i] = 0;
    __syncthreads();
    for (int qi = 0; qi < nq; ++qi) {
        const uint32_t *q = queues[qi];
        const size_t total = (size_t)qcnt[qi] * W;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
             i += (size_t)gridDim.x * blockDim.x) {
            const uint32_t y = q[i / W];
            const int j = (int)(i % W);
            uint64_t word = (uint64_t)atomicExch((unsigned long long *)&vis[(size_t)y * W + j], 0ull);
            if (!word) continue;
            uint64_t dy = 0;
            if (!alive) {
                dy = row_ptr[y + 1] - row_ptr[y];
            } else {
                for (uint64_t a = row_ptr[y]; a < row_ptr[y + 1]; ++a) dy += alive[col[a]] ? 1u : 0u;
            }
            while (word) {
                const int b = __builtin_ctzll(word);
                word &= word - 1;
                atomicAdd(&s_te[j * 64 + b], (unsigned long long)dy);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * W; i += blockDim.x)
        if (s_te[i]) atomicAdd(&te[i], s_te[i]);
}

__global__ void te_scatter_kernel(const uint32_t *srcs, uint32_t first, uint32_t cnt,
                                  const unsigned long long *te, uint64_t *te_full) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= cnt) return;
    const uint32_t s = srcs ? srcs[first + l] : first + l;
    te_full[s] = te[l];
}

__global__ void zero_u64_kernel(unsigned long long *p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

template <int W>
void launch_level(const LevelParams &p, int grid, bool last, hipStream_t st) {
    if (last)
        hipLaunchKernelGGL((level_kernel<W, true>), dim3(grid), dim3(kBlockThreads), 0, st, p);
    else
        hipLaunchKernelGGL((level_kernel<W, false>), dim3(grid), dim3(kBlockThreads), 0, st, p);
}

void dispatch_level(int W, const LevelParams &p, int grid, bool last, hipStream_t st) {
    switch (W) {
        case 1: launch_level<1>(p, grid, last, st); break;
        case 2: launch_level<2>(p, grid, last, st); break;
        case 4: launch_level<4>(p, grid, last, st); break;
        case 8: launch_level<8>(p, grid, last, st); break;
        case 16: launch_level<16>(p, grid, last, st); break;
        default: launch_level<32>(p, grid, last, st); break;
    }
}

template <int W>
void launch_scanned(int grid, hipStream_t st, const uint32_t *const *queues, const uint32_t *qcnt,
                    int nq, const uint64_t *row_ptr, const uint32_t *col, const uint8_t *alive,
                    uint64_t *vis, unsigned long long *te) {
    hipLaunchKernelGGL((scanned_arcs_kernel<W>), dim3(grid), dim3(256), 0, st, queues, qcnt, nq,
                       row_ptr, col, alive, vis, te);
}

int width_for(uint32_t cnt, int max_width) {
    int w = 1;
    while (w < max_width && (uint64_t)w * 64 < cnt) w <<= 1;
    return w;
}

// Batches of up to 64*max_width sources.  Per batch: reset counters, seed,
// h levels (the scanned-arc mode stops after h-1 and weights the reached
// rows instead), scatter the per-lane results, clear the touched rows.
int msbfs_run(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
              const uint32_t *srcs, uint32_t nsrc, uint32_t *deg_list, int scatter,
              uint32_t *deg_full, uint64_t *te_full) {
    if (nsrc == 0) return KHC_OK;
    const uint32_t levels = te_full ? h - 1 : h;
    const uint32_t n = g->n;
    const int maxW = ctx->max_width;
    const size_t words = (size_t)n * maxW;
    const uint32_t fnz_words = (n + 31) / 32;
    const uint32_t nq = levels + 1;  // frontier lists 0..levels
    void *vis, *f0, *f1, *f2, *fnz, *hacc, *hdone, *counts, *misc, *queues, *hqueues, *qptrs;
    // push items per level: at most one per row plus one per kPushChunk arcs
    const size_t hq_len = (size_t)n + g->nnz / kPushChunk + 1;
    int rc;
    if ((rc = ws_get(ctx, WS_VIS, words * 8, &vis)) ||
        (rc = ws_get(ctx, WS_FRT0, words * 8, &f0)) ||
        (rc = ws_get(ctx, WS_FRT1, words * 8, &f1)) ||
        (rc = ws_get(ctx, WS_FRT2, words * 8, &f2)) ||
        (rc = ws_get(ctx, WS_FNZ, (size_t)fnz_words * 3 * 4, &fnz)) ||
        (rc = ws_get(ctx, WS_HACC, ((size_t)g->n_heavy + 1) * maxW * 8, &hacc)) ||
        (rc = ws_get(ctx, WS_HDONE, ((size_t)g->n_heavy + 1) * 4, &hdone)) ||
        (rc = ws_get(ctx, WS_COUNTS, (size_t)64 * kMaxWidth * 4, &counts)) ||
        (rc = ws_get(ctx, WS_MISC, (size_t)nq * 24 + 64, &misc)) ||
        (rc = ws_get(ctx, WS_BQUEUE, (size_t)nq * n * 4 + 4, &queues)) ||
        (rc = ws_get(ctx, WS_HQUEUE, (size_t)nq * hq_len * 8, &hqueues)) ||
        (rc = ws_get(ctx, WS_QPTRS, (size_t)nq * 8, &qptrs)))
        return rc;
    void *te = nullptr;
    if (te_full && (rc = ws_get(ctx, WS_TE, (size_t)64 * kMaxWidth * 8, &te))) return rc;
    uint64_t *frt[3] = {(uint64_t *)f0, (uint64_t *)f1, (uint64_t *)f2};
    uint32_t *fnzp = (uint32_t *)fnz;
    // misc: qdeg[nq] (u64), then work[nq], qcnt[nq], hcnt[nq] (u32)
    unsigned long long *qdeg = (unsigned long long *)misc;
    uint32_t *work = (uint32_t *)(qdeg + nq);
    uint32_t *qcnt = work + nq;
    uint32_t *hcnt = qcnt + nq;
    uint32_t *qbase = (uint32_t *)queues;
    uint64_t *hqbase = (uint64_t *)hqueues;
    auto Q = [&](uint32_t j) { return qbase + (size_t)j * n; };
    auto F = [&](uint32_t j) {
        Frontier f;
        f.q = Q(j);
        f.qcnt = qcnt + j;
        f.qdeg = qdeg + j;
        f.hq = hqbase + (size_t)j * hq_len;
        f.hcnt = hcnt + j;
        return f;
    };
    const int grid = ctx->num_cu * ((ctx->waves_per_cu + 3) / 4);
    hipStream_t st = ctx->stream;

    if (te_full) {
        std::vector<const uint32_t *> hq(nq);
        for (uint32_t j = 0; j < nq; ++j) hq[j] = Q(j);
        hipError_t e = hipMemcpyAsync(qptrs, hq.data(), nq * sizeof(void *), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return check_hip(ctx, e, "queue table upload");
    }

    for (uint32_t first = 0; first < nsrc;) {
        const uint32_t remaining = nsrc - first;
        const int W = width_for(remaining, maxW);
        const uint32_t cnt = remaining < (uint32_t)(64 * W) ? remaining : (uint32_t)(64 * W);
        hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, st, work, qcnt, hcnt, qdeg, (int)nq,
                           (uint32_t *)counts, 64 * W);
        hipLaunchKernelGGL(batch_seed_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, srcs, first,
                           cnt, W, alive, g->row_ptr, (uint64_t *)vis, frt[0], fnzp, F(0));
        for (uint32_t lev = 1; lev <= levels; ++lev) {
            LevelParams p;
            p.row_ptr = g->row_ptr;
            p.col = g->col;
            p.alive = alive;
            p.light_rows = g->light_rows;
            p.heavy_rows = g->heavy_rows;
            p.chunk_heavy = g->chunk_heavy;
            p.chunk_first = g->chunk_first;
            p.frt_in = frt[(lev - 1) % 3];
            p.frt_out = frt[lev % 3];
            p.frt_clr = frt[(lev + 1) % 3];
            p.vis = (uint64_t *)vis;
            const Frontier fin = F(lev - 1);
            p.q_in = fin.q;
            p.hq_in = fin.hq;
            p.qcnt_in = fin.qcnt;
            p.hcnt_in = fin.hcnt;
            p.qdeg_in = fin.qdeg;
            p.out = F(lev);
            p.q_clr = lev >= 2 ? Q(lev - 2) : nullptr;
            p.qcnt_clr = lev >= 2 ? qcnt + lev - 2 : nullptr;
            p.fnz_out = fnzp + (size_t)(lev % 3) * fnz_words;
            p.fnz_clr = fnzp + (size_t)((lev + 1) % 3) * fnz_words;
            p.hacc = (uint64_t *)hacc;
            p.hdone = (uint32_t *)hdone;
            p.work = work + lev;
            p.counts = (uint32_t *)counts;
            p.nnz = g->nnz;
            p.n = n;
            p.n_light = g->n_light;
            p.n_chunks = g->n_chunks;
            // algorithmic bytes of a pull level over the whole graph
            const double bytes = alive ? 0.0
                                       : (double)n * (8.0 + 8.0 * W) + (double)g->nnz * (4.0 + 8.0 * W);
            const bool last = !te_full && lev == h;
            const int prec = prof_begin(ctx, last ? 3 : (lev == 1 ? 1 : 2), bytes);
            dispatch_level(W, p, grid, last, st);
            prof_end(ctx, prec);
        }
        if (te_full) {
            unsigned long long *tep = (unsigned long long *)te;
            hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, st, tep, 64 * W);
            const int sgrid = ctx->num_cu * 4;
            uint64_t *visp = (uint64_t *)vis;
            const uint32_t *const *qp = (const uint32_t *const *)qptrs;
            // the rows reached within h-1 hops are exactly those on lists 0..h-1
            const int nql = (int)levels + 1;
            switch (W) {
                case 1: launch_scanned<1>(sgrid, st, qp, qcnt, nql, g->row_ptr, g->col, alive, visp, tep); break;
                case 2: launch_scanned<2>(sgrid, st, qp, qcnt, nql, g->row_ptr, g->col, alive, visp, tep); break;
                case 4: launch_scanned<4>(sgrid, st, qp, qcnt, nql, g->row_ptr, g->col, alive, visp, tep); break;
                case 8: launch_scanned<8>(sgrid, st, qp, qcnt, nql, g->row_ptr, g->col, alive, visp, tep); break;
                case 16: launch_scanned<16>(sgrid, st, qp, qcnt, nql, g->row_ptr, g->col, alive, visp, tep); break;
                default: launch_scanned<32>(sgrid, st, qp, qcnt, nql, g->row_ptr, g->col, alive, visp, tep); break;
            }
            hipLaunchKernelGGL(te_scatter_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, srcs, first,
                               cnt, (const unsigned long long *)tep, te_full);
        } else {
            hipLaunchKernelGGL(batch_scatter_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, srcs,
                               first, cnt, (const uint32_t *)counts, deg_list, scatter ? deg_full : nullptr);
        }
        // Clean up: vis rows of every list, the last two frontier buffers
        // and maps (older ones were cleared by the levels themselves).
        const int prec = prof_begin(ctx, 0, 0.0);
        const int cgrid = ctx->num_cu * 4;
        for (uint32_t j = 0; j <= levels; ++j)
            hipLaunchKernelGGL(clear_rows_kernel, dim3(cgrid), dim3(256), 0, st, Q(j), qcnt + j,
                               (uint64_t *)vis, W, (uint32_t *)nullptr);
        for (uint32_t j = (levels >= 1 ? levels - 1 : 0); j <= levels; ++j)
            hipLaunchKernelGGL(clear_rows_kernel, dim3(cgrid), dim3(256), 0, st, Q(j), qcnt + j,
                               frt[j % 3], W, fnzp + (size_t)(j % 3) * fnz_words);
        prof_end(ctx, prec);
        first += cnt;
    }
    return check_hip(ctx, hipGetLastError(), "msbfs launch");
}

}  // namespace

int msbfs_degrees(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                  const uint32_t *srcs, uint32_t nsrc, uint32_t *deg_list, int scatter,
                  uint32_t *deg_full) {
    return msbfs_run(ctx, g, alive, h, srcs, nsrc, deg_list, scatter, deg_full, nullptr);
}

int msbfs_scanned_arcs(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                       const uint32_t *srcs, uint32_t nsrc, uint64_t *te_full) {
    return msbfs_run(ctx, g, alive, h, srcs, nsrc, nullptr, 1, nullptr, te_full);
}

}  // namespace khc
