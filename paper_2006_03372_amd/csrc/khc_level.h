// Device code of one bounded-BFS level, shared by the level kernel of the
// host-driven path and by the persistent peeling kernel.
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
#pragma once

#include "khc_internal.h"

namespace khc {
namespace lvl {

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

// Per kind of level: bit-sliced counter planes of each lane (a plane set
// holds counts up to 2^planes - 1 before it is flushed to LDS) and
// independent gathers in flight per lane.  Together they set the level's
// register use, its occupancy and its ripple-carry work per row.  Measured
// on the R-MAT-20 h = 3 pass (W = 32, per launch): 8 planes / 8 gathers
// took 1170 us (inner) and 766 us (counting); 6 / 6 took 1023 us inner,
// 4 / 6 took 740 us counting (147 and 127 VGPRs).
template <bool LAST>
constexpr int planes_of() { return LAST ? 4 : 6; }
template <bool LAST>
constexpr int unroll_of() { return 6; }
// Push when frontier arcs * factor < all arcs.  A pull level costs a fixed
// pass over every row plus 8W bytes per arc; a push costs about 8 bytes and
// one atomic per (frontier arc, non-zero word).  Narrow batches therefore
// push up to larger frontiers.
template <int W>
constexpr int push_factor() { return W >= 32 ? 16 : (W / 2 > 2 ? W / 2 : 2); }
constexpr int kGrab = 4;              // push work grab: one frontier item per wavefront
constexpr uint32_t kPushChunk = 256;  // arcs per push item of a heavy frontier row
constexpr int kStage = 4096;          // LDS staging of frontier rows
constexpr int kStageItem = 1024;      // most rows one work item can stage

// Frontier list of one level: every row once (q, count, total degree) and,
// for rows with more than kPushChunk arcs, one push item per kPushChunk arcs
// (row | chunk << 32) so heavy rows spread over many wavefronts.  qdeg
// points to two sums over the frontier rows: qdeg[0] = their degrees,
// qdeg[1] = degree times non-zero words (the (arc, word) pairs a push of
// the next level would process).
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
    const unsigned long long *qdeg_in;  // {degree sum, push pairs} of the previous frontier
    Frontier out;           // this level's frontier
    const uint32_t *q_clr;  // rows of the frontier two levels back
    const uint32_t *qcnt_clr;
    uint32_t *fnz_out;  // 1 bit per vertex: row is on this level's frontier
    uint32_t *fnz_clr;
    uint64_t *hacc;
    uint32_t *hdone;
    uint32_t *work;    // work-item counter of this level
    uint32_t *counts;  // per-lane reached-vertex totals, summed over levels
    // One persistent kernel: the workgroup's LDS totals carry over between
    // the levels of a batch (cleared at its first level) and are added to
    // counts once, at the last level, instead of after every level.
    int count_keep;
    int count_first;
    uint64_t nnz;  // arcs the pull direction would read (push/pull choice)
    uint32_t n;
    // push/pull choice: 0 pushes while (frontier degree) * push_factor<W>
    // < nnz; c > 0 pushes while (push pairs) * c < nnz * W + 4 * rows, the
    // pull's word gathers plus a per-row share (a push pair is a few
    // random 8-byte atomics, a pull gather one word of a 16-byte load)
    uint32_t push_cost;
    // rows y with count_mask[y] == 0 are reached but not counted (null: all
    // counted); the sampling mode counts the sampled vertices of a ball
    const uint8_t *count_mask;
    // pull visits light rows light_rows[light_lo, light_hi) and heavy-row
    // chunks [chunk_lo, chunk_hi) (all of them for one graph; the batch's
    // graphs for graphs packed together)
    uint32_t light_lo, light_hi;
    uint32_t chunk_lo, chunk_hi;
    // Graph windows (batched graphs; null for one graph): the batch's
    // sources are grouped by graph, graph g owning source slots
    // [seg_pfx[g], seg_pfx[g+1]) of the job and this batch the slots
    // [batch_base, batch_base + 64 W).  A row of graph g can only hold the
    // lanes of g's sources, so pull reads and writes only those words and
    // skips rows of graphs without a source in the batch.
    const uint32_t *gid;
    const uint32_t *seg_pfx;
    uint32_t batch_base;
};

// Words [*w0, *w1] of row y that can hold bits of this batch; false if none.
template <int W>
__device__ __forceinline__ bool row_window(const LevelParams &p, uint32_t y, int *w0, int *w1) {
    if (!p.gid) {
        *w0 = 0;
        *w1 = W - 1;
        return true;
    }
    const uint32_t g = p.gid[y];
    const uint32_t lo = p.seg_pfx[g], hi = p.seg_pfx[g + 1];
    const uint32_t b0 = p.batch_base, b1 = p.batch_base + 64u * W;
    if (hi <= b0 || lo >= b1) return false;
    *w0 = (int)(((lo > b0 ? lo : b0) - b0) >> 6);
    *w1 = (int)(((hi < b1 ? hi : b1) - 1u - b0) >> 6);
    return true;
}

// True when every bit of the lane's words is set in a | b: no gather can
// add a new bit, so the lane stops gathering.
template <int WPL>
__device__ __forceinline__ bool saturated(const uint64_t (&a)[WPL], const uint64_t (&b)[WPL]) {
    uint64_t all = ~0ull;
#pragma unroll
    for (int j = 0; j < WPL; ++j) all &= a[j] | b[j];
    return all == ~0ull;
}

// Add the WPL words of x to the bit-sliced counters (one ripple-carry add
// per word: plane k holds bit k of every bit position's count).
template <int WPL, int kPlanes>
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

template <int WPL, int kPlanes>
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

static __device__ __forceinline__ void count_word_bits(uint32_t *s_counts, int word, uint64_t bits) {
    while (bits) {
        int b = __builtin_ctzll(bits);
        bits &= bits - 1;
        atomicAdd(&s_counts[word * 64 + b], 1u);
    }
}

// Push items of a heavy frontier row (called by the lane that lists it).
static __device__ __forceinline__ void add_push_items(const Frontier &f, uint32_t y, uint64_t dy) {
    if (dy <= kPushChunk) return;
    const uint32_t nch = (uint32_t)((dy + kPushChunk - 1) / kPushChunk);
    const uint32_t at = atomicAdd(f.hcnt, nch);
    for (uint32_t c = 0; c < nch; ++c) f.hq[at + c] = (uint64_t)y | ((uint64_t)c << 32);
}

// Wave-aggregated append to the workgroup's LDS staging list.
static __device__ __forceinline__ void append_staged(bool take, uint32_t y, uint32_t *s_stage,
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
static __device__ void flush_staged(const Frontier &f, const uint64_t *row_ptr, uint32_t *s_stage,
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
                           uint32_t *s_counts, uint32_t *s_stage, uint32_t *s_sn, unsigned long long *s_work) {
    const int lane = threadIdx.x & 63;
    const uint64_t myw = lane < W ? p.frt_in[(size_t)x * W + lane] : 0ull;
    const uint64_t nzmask = __ballot(myw != 0);
    const uint32_t nz = (uint32_t)__builtin_popcountll(nzmask);
    const uint64_t pairs = (ae - ab) * nz;
    for (uint64_t base = 0; base < pairs; base += 64) {
        const uint64_t pr = base + lane;
        bool take = false;
        uint32_t y = 0;
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
                        if (!p.count_mask || p.count_mask[y]) count_word_bits(s_counts, w, tn);
                        if constexpr (!LAST) {
                            const uint64_t was = atomicOr((unsigned long long *)(p.frt_out + (size_t)y * W + w),
                                                          (unsigned long long)tn);
                            // a word that turns non-zero adds the row's arcs to the next push
                            if (!was) atomicAdd(s_work, (unsigned long long)(p.row_ptr[y + 1] - p.row_ptr[y]));
                        }
                        // listed even at the counting level: its vis words
                        // changed, and the batch clears exactly the listed rows
                        const uint32_t ybit = 1u << (y & 31);
                        take = !(atomicOr(&p.fnz_out[y >> 5], ybit) & ybit);
                    }
                }
            }
        }
        append_staged(take, y, s_stage, s_sn);
    }
}


// LDS of one bounded-BFS level (one per workgroup).
template <int W>
struct LevelLds {
    uint64_t red[RowLayout<W>::GROUPS * W];
    uint64_t fin[W];
    uint32_t counts[64 * W];
    uint32_t stage[kStage];
    uint32_t sn, base, item, flag;
    unsigned long long deg, work;
};

// One level of the multi-source bounded BFS over the whole grid (see the
// direction and work-split description at the top of this file).  Every
// workgroup of the launch must call it; work comes from p.work, which must
// be zero on entry.  LAST: the counting level (no frontier written).
template <int W, bool LAST>
__device__ void level_body(const LevelParams &p, LevelLds<W> &sh) {
    using L = RowLayout<W>;
    constexpr int WPL = L::WPL, LPR = L::LPR, RPW = L::RPW, GROUPS = L::GROUPS;
    constexpr int kPlanes = planes_of<LAST>(), kUnroll = unroll_of<LAST>();
    // light rows handled per work item: several passes of all lane groups
    constexpr int PASSES = GROUPS >= 64 ? 1 : 64 / GROUPS;
    uint64_t *const s_red = sh.red;
    uint64_t *const s_fin = sh.fin;
    uint32_t *const s_counts = sh.counts;
    uint32_t *const s_stage = sh.stage;
    uint32_t &s_sn = sh.sn, &s_base = sh.base, &s_item = sh.item, &s_flag = sh.flag;
    unsigned long long &s_deg = sh.deg, &s_work = sh.work;

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

    if (!p.count_keep || p.count_first)
        for (int i = tid; i < 64 * W; i += kBlockThreads) s_counts[i] = 0;
    if (tid == 0) {
        s_sn = 0;
        s_work = 0;
    }
    uint64_t pl[WPL][kPlanes];
#pragma unroll
    for (int j = 0; j < WPL; ++j)
#pragma unroll
        for (int k = 0; k < kPlanes; ++k) pl[j][k] = 0;
    uint32_t pcount = 0;

    const bool push =
        p.push_cost ? p.qdeg_in[1] * p.push_cost < (unsigned long long)p.nnz * W + 4ull * (p.light_hi - p.light_lo)
                    : p.qdeg_in[0] * push_factor<W>() < (unsigned long long)p.nnz;
    const uint32_t qn_in = *p.qcnt_in;
    const uint32_t hn_in = *p.hcnt_in;
    const uint32_t light_grabs = (qn_in + kGrab - 1) / kGrab;
    const uint32_t n_chunk_items = p.chunk_hi - p.chunk_lo;
    const uint32_t n_light_rows = p.light_hi - p.light_lo;
    const uint32_t n_items = push ? light_grabs + (hn_in + kGrab - 1) / kGrab
                                  : n_chunk_items + (n_light_rows + GROUPS * PASSES - 1) / (GROUPS * PASSES);
    __syncthreads();

    // The first item of each workgroup is its block index; later items come
    // from the counter (offset by the grid size), so workgroups without work
    // leave without touching it.  Measured against the alternatives (several
    // items per atomic; three quarters of the items dealt round-robin first)
    // taking one item per atomic balanced the big levels best: they lost
    // 7-32% (up to 20% of the R-MAT-20 level rate).
    for (bool first = true;; first = false) {
        if (tid == 0) s_item = first ? blockIdx.x : gridDim.x + atomicAdd(p.work, 1u);
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
                    if (re - rb <= kPushChunk) push_range<W, LAST>(p, x, rb, re, s_counts, s_stage, &s_sn, &s_work);
                }
            } else {
                const uint32_t hi = (item - light_grabs) * kGrab + wave;
                if (hi < hn_in) {
                    const uint64_t it = p.hq_in[hi];
                    const uint32_t x = (uint32_t)it;
                    const uint64_t rb = p.row_ptr[x], re = p.row_ptr[x + 1];
                    const uint64_t ab = rb + (it >> 32) * kPushChunk;
                    const uint64_t ae = ab + kPushChunk < re ? ab + kPushChunk : re;
                    push_range<W, LAST>(p, x, ab, ae, s_counts, s_stage, &s_sn, &s_work);
                }
            }
        } else if (item < n_chunk_items) {
            // ---- pull, one chunk of a heavy row, whole workgroup ----
            const uint32_t chunk = p.chunk_lo + item;
            const uint32_t hi = p.chunk_heavy[chunk];
            const uint32_t y = p.heavy_rows[hi];
            int w0 = 0, w1 = W - 1;
            const bool live = (!p.alive || p.alive[y]) && row_window<W>(p, y, &w0, &w1);
            // this lane's words [lig * WPL, lig * WPL + WPL) meet the window
            const bool lane_on = lig * WPL + WPL - 1 >= w0 && lig * WPL <= w1;
            if (live) {
                const uint32_t c0 = p.chunk_first[hi];
                const uint32_t nch = p.chunk_first[hi + 1] - c0;
                const uint64_t rb = p.row_ptr[y], re = p.row_ptr[y + 1];
                const uint64_t b = rb + (uint64_t)(chunk - c0) * kChunkArcs;
                const uint64_t e = (b + kChunkArcs < re) ? b + kChunkArcs : re;
                uint64_t acc[WPL];
#pragma unroll
                for (int j = 0; j < WPL; ++j) acc[j] = 0;
                uint64_t a = b + group;
                // words this lane's sources have all reached need no gather
                uint64_t v0[WPL];
                if (lane_on) load_words<WPL>(p.vis + (size_t)y * W + lig * WPL, v0);
                if (lane_on && !saturated<WPL>(acc, v0)) {
                    // slots past the chunk's end repeat the step's first arc
                    for (; a < e; a += (uint64_t)kUnroll * GROUPS) {
                        uint32_t xs[kUnroll];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u) {
                            const uint64_t au = a + (uint64_t)u * GROUPS;
                            xs[u] = p.col[au < e ? au : a];
                        }
                        uint64_t t[kUnroll][WPL];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            load_words<WPL>(p.frt_in + (size_t)xs[u] * W + lig * WPL, t[u]);
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                            for (int j = 0; j < WPL; ++j) acc[j] |= t[u][j];
                        if (saturated<WPL>(acc, v0)) {
                            a = e;
                            break;
                        }
                    }
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
                    if (tid >= w0 && tid <= w1) {
                        const uint64_t v = p.vis[(size_t)y * W + tid];
                        nw = s_fin[tid] & ~v;
                        if (nw) {
                            if (!p.count_mask || p.count_mask[y]) count_word_bits(s_counts, tid, nw);
                            if constexpr (!LAST) {
                                p.frt_out[(size_t)y * W + tid] = nw;
                                p.vis[(size_t)y * W + tid] = v | nw;
                            }
                        }
                    }
                    if constexpr (!LAST) {
                        const uint64_t nzw = __ballot(nw != 0);
                        const bool any = nzw != 0;
                        if (tid == 0 && any) {
                            atomicOr(&p.fnz_out[y >> 5], 1u << (y & 31));
                            atomicAdd(&s_work, (unsigned long long)(re - rb) * __builtin_popcountll(nzw));
                        }
                        append_staged(tid == 0 && any, y, s_stage, &s_sn);
                    }
                }
            }
        } else {
            // ---- pull, light rows: one lane group per row ----
            const uint32_t tile = item - n_chunk_items;
            for (int pass = 0; pass < PASSES; ++pass) {
                const uint32_t idx = (tile * PASSES + pass) * GROUPS + group;
                bool valid = idx < n_light_rows;
                const uint32_t y = valid ? p.light_rows[p.light_lo + idx] : 0u;
                if (valid && p.alive && !p.alive[y]) valid = false;
                int w0 = 0, w1 = W - 1;
                if (valid && !row_window<W>(p, y, &w0, &w1)) valid = false;
                // Narrow window (batched graphs: the row's lanes fit in one
                // lane's words): the group's lanes split the arcs instead of
                // the words, and OR their gathers into the owning lane.
                const bool narrow = LPR > 1 && valid && p.gid != nullptr && w0 / WPL == w1 / WPL;
                const int own = w0 / WPL;
                // this lane's words meet the row's window
                const bool lane_on =
                    valid && (narrow ? lig == own : (lig * WPL + WPL - 1 >= w0 && lig * WPL <= w1));
                uint64_t acc[WPL];
#pragma unroll
                for (int j = 0; j < WPL; ++j) acc[j] = 0;
                // the row's visited words, read first: a lane whose words
                // are all set already (every source reached y) gathers nothing
                uint64_t v[WPL], nw[WPL];
                if (lane_on) {
                    load_words<WPL>(p.vis + (size_t)y * W + lig * WPL, v);
                } else {
#pragma unroll
                    for (int j = 0; j < WPL; ++j) v[j] = ~0ull;
                }
                if (narrow) {
                    const uint64_t rb = p.row_ptr[y], re = p.row_ptr[y + 1];
                    uint64_t a = rb + lig;
                    // slots past the row's end repeat the step's first arc
                    for (; a < re; a += (uint64_t)kUnroll * LPR) {
                        uint32_t xs[kUnroll];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u) {
                            const uint64_t au = a + (uint64_t)u * LPR;
                            xs[u] = p.col[au < re ? au : a];
                        }
                        uint64_t t[kUnroll][WPL];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            load_words<WPL>(p.frt_in + (size_t)xs[u] * W + own * WPL, t[u]);
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                            for (int j = 0; j < WPL; ++j) acc[j] |= t[u][j];
                    }
                } else if (lane_on && !saturated<WPL>(acc, v)) {
                    const uint64_t rb = p.row_ptr[y], re = p.row_ptr[y + 1];
                    uint64_t a = rb;
                    // Every step issues kUnroll independent gathers; slots past
                    // the row's end repeat the step's first arc (OR-ing a word
                    // twice changes nothing), so a short row costs one round
                    // trip instead of one per arc.  Measured on the R-MAT-20
                    // h = 3 pass: inner level 1022 -> 1001 us per launch.
                    for (; a < re; a += kUnroll) {
                        uint32_t xs[kUnroll];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u) xs[u] = p.col[a + u < re ? a + u : a];
                        uint64_t t[kUnroll][WPL];
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            load_words<WPL>(p.frt_in + (size_t)xs[u] * W + lig * WPL, t[u]);
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                            for (int j = 0; j < WPL; ++j) acc[j] |= t[u][j];
                        // every source of the lane's words has reached y
                        if (saturated<WPL>(acc, v)) {
                            a = re;
                            break;
                        }
                    }
                }
                if constexpr (LPR > 1) {
                    // OR the narrow rows' partial gathers over the lane group
#pragma unroll
                    for (int j = 0; j < WPL; ++j) {
                        uint32_t lo = narrow ? (uint32_t)acc[j] : 0u, hi = narrow ? (uint32_t)(acc[j] >> 32) : 0u;
#pragma unroll
                        for (int off = LPR / 2; off > 0; off >>= 1) {
                            lo |= __shfl_xor(lo, off, 64);
                            hi |= __shfl_xor(hi, off, 64);
                        }
                        if (narrow) acc[j] = lig == own ? ((uint64_t)hi << 32 | lo) : 0ull;
                    }
                }
                uint64_t any = 0;
#pragma unroll
                for (int j = 0; j < WPL; ++j) {
                    nw[j] = acc[j] & ~v[j];
                    any |= nw[j];
                }
                // a row outside the count mask passes its bits on uncounted
                if (!p.count_mask || !valid || p.count_mask[y]) planes_add<WPL, kPlanes>(pl, nw);
                if (++pcount == (1u << kPlanes) - 1u) {
                    planes_flush<WPL, kPlanes>(pl, s_counts, lig * WPL);
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
                    // non-zero words of the row, summed over its lane group
                    uint32_t nzw = 0;
#pragma unroll
                    for (int j = 0; j < WPL; ++j) nzw += nw[j] != 0;
#pragma unroll
                    for (int off = LPR / 2; off > 0; off >>= 1) nzw += __shfl_xor(nzw, off, 64);
                    if (lead) {
                        atomicOr(&p.fnz_out[y >> 5], 1u << (y & 31));
                        atomicAdd(&s_work, (unsigned long long)(p.row_ptr[y + 1] - p.row_ptr[y]) * nzw);
                    }
                    append_staged(lead, y, s_stage, &s_sn);
                }
            }
        }
        __syncthreads();
        // (the counting level stages rows only when it pushes: their vis changed)
        if (s_sn > kStage - kStageItem) flush_staged(p.out, p.row_ptr, s_stage, &s_sn, &s_base, &s_deg);
    }

    flush_staged(p.out, p.row_ptr, s_stage, &s_sn, &s_base, &s_deg);
    if (!LAST && tid == 0 && s_work) atomicAdd(p.out.qdeg + 1, s_work);
    planes_flush<WPL, kPlanes>(pl, s_counts, lig * WPL);
    __syncthreads();
    if (!p.count_keep || LAST)
        for (int i = tid; i < 64 * W; i += kBlockThreads)
            if (s_counts[i]) atomicAdd(&p.counts[i], s_counts[i]);
    __syncthreads();
}

}  // namespace lvl
}  // namespace khc
