// Multi-source h-bounded BFS for h-degrees (gfx950).
//
// The h-degree d_v^h(G(S)) (Section II) of many sources is computed at once:
// one batch carries 64*W sources as bit lanes of W uint64 words per vertex.
// For every vertex y, vis[y] holds the lanes whose source has reached y and
// frt[y] the lanes that reached y at the previous hop.  One level of the
// bounded BFS is, for every live y,
//     new[y] = (OR over live neighbours x of frt[x]) AND NOT vis[y]
//     vis[y] |= new[y];  frt'[y] = new[y]
// and after h levels d^h(source of lane l) = |{y : bit l of vis[y]}| - 1.
// This transposes the paper's bitmap idea (Section IV-B, bit j of a
// vertex's bitmap marks reachability of the j-th vertex): here a bit marks
// a source lane, so one wide OR advances 64*W BFS runs by one hop.
//
// Rows are pulled: lane groups gather the frontier words of a row's
// neighbours with 16-byte loads.  Rows up to kHeavyRowArcs arcs are handled
// by one group of W/2 lanes (rows sorted by degree so a wavefront's rows are
// alike); heavier rows are cut into chunks of kChunkArcs arcs that whole
// workgroups OR together, the last chunk to finish completing the row.
// Workgroups are persistent and take work items from an atomic counter.
// A 1-bit-per-vertex map of non-empty frontier rows lets sparse levels skip
// gathers of empty rows.  Counts are kept per lane in bit-sliced
// registers and reduced through LDS at the end.
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

constexpr int kPlanes = 8;  // bit-sliced per-lane counters hold up to 255

struct LevelParams {
    const uint64_t *row_ptr;
    const uint32_t *col;
    const uint8_t *alive;
    const uint32_t *light_rows;
    const uint32_t *heavy_rows;
    const uint32_t *chunk_heavy;
    const uint32_t *chunk_first;
    const uint64_t *frt_in;
    uint64_t *frt_out;
    uint64_t *vis;
    const uint32_t *fnz_in;
    uint32_t *fnz_out;
    uint32_t *fnz_clear;
    uint64_t *hacc;
    uint32_t *hdone;
    uint32_t *work;          // work-item counter of this level
    const uint32_t *fc_in;   // frontier rows produced by the previous level
    uint32_t *fc_out;        // frontier rows produced by this level
    uint32_t *counts;        // per-lane reached-vertex totals (last level)
    uint32_t n;
    uint32_t n_light;
    uint32_t n_chunks;
    uint32_t fnz_words;
};

__device__ __forceinline__ bool fnz_test(const uint32_t *fnz, uint32_t x) {
    return (fnz[x >> 5] >> (x & 31)) & 1u;
}

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

template <int W, bool LAST>
__global__ __launch_bounds__(kBlockThreads) void level_kernel(LevelParams p) {
    using L = RowLayout<W>;
    constexpr int WPL = L::WPL, LPR = L::LPR, RPW = L::RPW, GROUPS = L::GROUPS;
    __shared__ uint64_t s_red[GROUPS * W];
    __shared__ uint64_t s_fin[W];
    __shared__ uint32_t s_counts[LAST ? 64 * W : 1];
    __shared__ uint32_t s_item;
    __shared__ uint32_t s_flag;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lig = lane % LPR;           // lane within its row group
    const int group = wave * RPW + lane / LPR;

    // Clear the frontier map that the level after next will write.
    for (uint32_t i = blockIdx.x * kBlockThreads + tid; i < p.fnz_words;
         i += gridDim.x * kBlockThreads)
        p.fnz_clear[i] = 0;

    const bool use_fnz = p.fc_in[0] < (p.n >> 3);

    uint64_t pl[WPL][kPlanes];
    uint32_t pcount = 0;
    if constexpr (LAST) {
        for (int i = tid; i < 64 * W; i += kBlockThreads) s_counts[i] = 0;
#pragma unroll
        for (int j = 0; j < WPL; ++j)
#pragma unroll
            for (int k = 0; k < kPlanes; ++k) pl[j][k] = 0;
    }
    uint32_t my_front = 0;  // rows this lane (as group leader) put on the next frontier

    const uint32_t n_tiles = (p.n_light + GROUPS - 1) / GROUPS;
    const uint32_t total = p.n_chunks + n_tiles;
    __syncthreads();

    for (;;) {
        if (tid == 0) s_item = atomicAdd(p.work, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= total) break;

        if (item < p.n_chunks) {
            // ---- one chunk of a heavy row, whole workgroup ----
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
                for (uint64_t a = b + group; a < e; a += GROUPS) {
                    const uint32_t x = p.col[a];
                    if (use_fnz && !fnz_test(p.fnz_in, x)) continue;
                    uint64_t t[WPL];
                    load_words<WPL>(p.frt_in + (size_t)x * W + lig * WPL, t);
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
                    if (tid < W && s_fin[tid]) atomicOr((unsigned long long *)&p.hacc[(size_t)hi * W + tid],
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
                    uint64_t nw = 0, v = 0;
                    if (tid < W) {
                        v = p.vis[(size_t)y * W + tid];
                        nw = s_fin[tid] & ~v;
                    }
                    if constexpr (LAST) {
                        uint64_t f = v | nw;
                        while (f) {
                            int bb = __builtin_ctzll(f);
                            f &= f - 1;
                            atomicAdd(&s_counts[tid * 64 + bb], 1u);
                        }
                    } else {
                        if (tid < W) {
                            p.frt_out[(size_t)y * W + tid] = nw;
                            if (nw) p.vis[(size_t)y * W + tid] = v | nw;
                        }
                        if (__ballot(nw != 0) != 0 && tid == 0) {
                            atomicOr(&p.fnz_out[y >> 5], 1u << (y & 31));
                            my_front++;
                        }
                    }
                }
            }
        } else {
            // ---- a tile of light rows: one lane group per row ----
            const uint32_t idx = (item - p.n_chunks) * GROUPS + group;
            bool valid = idx < p.n_light;
            uint32_t y = valid ? p.light_rows[idx] : 0u;
            if (valid && p.alive && !p.alive[y]) valid = false;
            uint64_t acc[WPL];
#pragma unroll
            for (int j = 0; j < WPL; ++j) acc[j] = 0;
            if (valid) {
                const uint64_t b = p.row_ptr[y], e = p.row_ptr[y + 1];
                for (uint64_t a = b; a < e; ++a) {
                    const uint32_t x = p.col[a];
                    if (use_fnz && !fnz_test(p.fnz_in, x)) continue;
                    uint64_t t[WPL];
                    load_words<WPL>(p.frt_in + (size_t)x * W + lig * WPL, t);
#pragma unroll
                    for (int j = 0; j < WPL; ++j) acc[j] |= t[j];
                }
            }
            uint64_t v[WPL], nw[WPL];
            if (valid) {
                load_words<WPL>(p.vis + (size_t)y * W + lig * WPL, v);
            } else {
#pragma unroll
                for (int j = 0; j < WPL; ++j) v[j] = 0;
            }
            uint64_t any = 0;
#pragma unroll
            for (int j = 0; j < WPL; ++j) {
                nw[j] = acc[j] & ~v[j];
                any |= nw[j];
            }
            if constexpr (LAST) {
                uint64_t f[WPL];
#pragma unroll
                for (int j = 0; j < WPL; ++j) f[j] = v[j] | nw[j];
                planes_add<WPL>(pl, f);
                if (++pcount == (1u << kPlanes) - 1u) {
                    planes_flush<WPL>(pl, s_counts, lig * WPL);
                    pcount = 0;
                }
            } else {
                if (valid) {
                    store_words<WPL>(p.frt_out + (size_t)y * W + lig * WPL, nw);
                    if (any) {
                        uint64_t vv[WPL];
#pragma unroll
                        for (int j = 0; j < WPL; ++j) vv[j] = v[j] | nw[j];
                        store_words<WPL>(p.vis + (size_t)y * W + lig * WPL, vv);
                    }
                }
                const uint64_t m = __ballot(any != 0);
                const uint64_t gmask = (LPR == 64) ? ~0ull : ((1ull << LPR) - 1ull);
                const int gshift = (lane / LPR) * LPR;
                if (valid && lig == 0 && ((m >> gshift) & gmask)) {
                    atomicOr(&p.fnz_out[y >> 5], 1u << (y & 31));
                    my_front++;
                }
            }
        }
        __syncthreads();
    }

    if constexpr (LAST) {
        planes_flush<WPL>(pl, s_counts, lig * WPL);
        __syncthreads();
        for (int i = tid; i < 64 * W; i += kBlockThreads)
            if (s_counts[i]) atomicAdd(&p.counts[i], s_counts[i]);
    } else {
        // wave-aggregated count of new frontier rows
        uint32_t c = my_front;
        for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
        if (lane == 0 && c) atomicAdd(p.fc_out, c);
    }
}

// Zero the batch state: vis and both frontier arrays (n*W words each), the
// three frontier maps, per-lane counts, level work counters and frontier
// counts.
__global__ void batch_clear_kernel(uint64_t *vis, uint64_t *f0, uint64_t *f1, size_t words,
                                   uint32_t *fnz, size_t fnz_total, uint32_t *counts, int ncounts,
                                   uint32_t *misc, int nmisc) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) {
        vis[i] = 0;
        f0[i] = 0;
        f1[i] = 0;
    }
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < fnz_total; i += stride) fnz[i] = 0;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < ncounts; i += blockDim.x) counts[i] = 0;
        for (int i = threadIdx.x; i < nmisc; i += blockDim.x) misc[i] = 0;
    }
}

// Put source lane l on its vertex: vis and level-0 frontier get bit l.
// srcs == null means the implicit list first, first+1, ...
// A dead source is not seeded; its lane stays empty and reports 0.
__global__ void batch_seed_kernel(const uint32_t *srcs, uint32_t first, uint32_t cnt, int W,
                                  const uint8_t *alive, uint64_t *vis, uint64_t *f0, uint32_t *fnz0,
                                  uint32_t *fc0) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l == 0) fc0[0] = cnt;
    if (l >= cnt) return;
    const uint32_t s = srcs ? srcs[first + l] : first + l;
    if (alive && !alive[s]) return;
    const uint64_t bit = 1ull << (l & 63);
    // sources are distinct vertices, so each (vertex, word) has one writer
    vis[(size_t)s * W + (l >> 6)] |= bit;
    f0[(size_t)s * W + (l >> 6)] |= bit;
    atomicOr(&fnz0[s >> 5], 1u << (s & 31));
}

// d = reached-vertex count of the lane minus the source itself.
__global__ void batch_scatter_kernel(const uint32_t *srcs, uint32_t first, uint32_t cnt,
                                     const uint32_t *counts, uint32_t *deg_list, uint32_t *deg_full) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= cnt) return;
    const uint32_t d = counts[l] ? counts[l] - 1u : 0u;
    if (deg_full) {
        const uint32_t s = srcs ? srcs[first + l] : first + l;
        deg_full[s] = d;
    } else {
        deg_list[first + l] = d;
    }
}

// Scanned-arc totals: for every source lane, the sum over vertices it has
// reached (within h-1 hops, including itself) of their live degree, i.e. the
// arcs a scalar bounded BFS from that source examines.  One thread per
// (row, word); LDS totals per lane, flushed with 64-bit atomics.
template <int W>
__global__ __launch_bounds__(256) void scanned_arcs_kernel(uint32_t n, const uint64_t *row_ptr,
                                                           const uint32_t *col, const uint8_t *alive,
                                                           const uint64_t *vis,
                                                           unsigned long long *te) {
    __shared__ unsigned long long s_te[64 * W];
    for (int i = threadIdx.x; i < 64 * W; i += blockDim.x) s_te[i] = 0;
    __syncthreads();
    const size_t total = (size_t)n * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        uint64_t word = vis[i];
        if (!word) continue;
        const uint32_t y = (uint32_t)(i / W);
        const int j = (int)(i % W);
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
void launch_scanned(int grid, hipStream_t st, uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                    const uint8_t *alive, const uint64_t *vis, unsigned long long *te) {
    hipLaunchKernelGGL((scanned_arcs_kernel<W>), dim3(grid), dim3(256), 0, st, n, row_ptr, col, alive,
                       vis, te);
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

int width_for(uint32_t cnt, int max_width) {
    int w = 1;
    while (w < max_width && (uint64_t)w * 64 < cnt) w <<= 1;
    return w;
}

}  // namespace

int msbfs_run(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
              const uint32_t *srcs, uint32_t nsrc, uint32_t *deg_list, int scatter,
              uint32_t *deg_full, uint64_t *te_full) {
    if (nsrc == 0) return KHC_OK;
    // scanned-arc mode: expand h-1 levels, then weight the reached vertices
    const uint32_t levels = te_full ? h - 1 : h;
    const uint32_t n = g->n;
    const int maxW = ctx->max_width;
    const size_t words = (size_t)n * maxW;
    const uint32_t fnz_words = (n + 31) / 32;
    void *vis, *f0, *f1, *fnz, *hacc, *hdone, *counts, *misc;
    int rc;
    if ((rc = ws_get(ctx, WS_VIS, words * 8, &vis)) ||
        (rc = ws_get(ctx, WS_FRT0, words * 8, &f0)) ||
        (rc = ws_get(ctx, WS_FRT1, words * 8, &f1)) ||
        (rc = ws_get(ctx, WS_FNZ, (size_t)fnz_words * 3 * 4, &fnz)) ||
        (rc = ws_get(ctx, WS_HACC, ((size_t)g->n_heavy + 1) * maxW * 8, &hacc)) ||
        (rc = ws_get(ctx, WS_HDONE, ((size_t)g->n_heavy + 1) * 4, &hdone)) ||
        (rc = ws_get(ctx, WS_COUNTS, (size_t)64 * kMaxWidth * 4, &counts)) ||
        (rc = ws_get(ctx, WS_MISC, ((size_t)2 * h + 4) * 4, &misc)))
        return rc;
    void *te = nullptr;
    if (te_full && (rc = ws_get(ctx, WS_LB, (size_t)64 * kMaxWidth * 8, &te))) return rc;
    uint32_t *fnzp = (uint32_t *)fnz;
    // misc: [0, h] level work counters, [h+1, 2h+2] frontier row counts
    uint32_t *miscp = (uint32_t *)misc;
    uint32_t *fcp = miscp + h + 1;
    const int grid = ctx->num_cu * ((ctx->waves_per_cu + 3) / 4);
    hipStream_t st = ctx->stream;

    for (uint32_t first = 0; first < nsrc;) {
        const uint32_t remaining = nsrc - first;
        const int W = width_for(remaining, maxW);
        const uint32_t cnt = remaining < (uint32_t)(64 * W) ? remaining : (uint32_t)(64 * W);
        const size_t bw = (size_t)n * W;
        int cgrid = (int)((bw + 255) / 256);
        if (cgrid > ctx->num_cu * 8) cgrid = ctx->num_cu * 8;
        if (cgrid < 1) cgrid = 1;
        int prec = prof_begin(ctx, 0, 0.0);
        hipLaunchKernelGGL(batch_clear_kernel, dim3(cgrid), dim3(256), 0, st, (uint64_t *)vis,
                           (uint64_t *)f0, (uint64_t *)f1, bw, fnzp, (size_t)fnz_words * 3,
                           (uint32_t *)counts, 64 * W, miscp, (int)(2 * h + 3));
        prof_end(ctx, prec);
        hipLaunchKernelGGL(batch_seed_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, srcs,
                           first, cnt, W, alive, (uint64_t *)vis, (uint64_t *)f0, fnzp, fcp);
        for (uint32_t lev = 1; lev <= levels; ++lev) {
            LevelParams p;
            p.row_ptr = g->row_ptr;
            p.col = g->col;
            p.alive = alive;
            p.light_rows = g->light_rows;
            p.heavy_rows = g->heavy_rows;
            p.chunk_heavy = g->chunk_heavy;
            p.chunk_first = g->chunk_first;
            p.frt_in = (lev & 1) ? (const uint64_t *)f0 : (const uint64_t *)f1;
            p.frt_out = (lev & 1) ? (uint64_t *)f1 : (uint64_t *)f0;
            p.vis = (uint64_t *)vis;
            p.fnz_in = fnzp + (size_t)((lev - 1) % 3) * fnz_words;
            p.fnz_out = fnzp + (size_t)(lev % 3) * fnz_words;
            p.fnz_clear = fnzp + (size_t)((lev + 1) % 3) * fnz_words;
            p.hacc = (uint64_t *)hacc;
            p.hdone = (uint32_t *)hdone;
            p.work = miscp + lev;
            p.fc_in = fcp + (lev - 1);
            p.fc_out = fcp + lev;
            p.counts = (uint32_t *)counts;
            p.n = n;
            p.n_light = g->n_light;
            p.n_chunks = g->n_chunks;
            p.fnz_words = (lev + 1 <= levels) ? fnz_words : 0u;
            // algorithmic bytes of a pull level over the whole graph
            const double bytes = alive ? 0.0
                                       : (double)n * (8.0 + 8.0 * W) + (double)g->nnz * (4.0 + 8.0 * W);
            const bool last = !te_full && lev == h;
            prec = prof_begin(ctx, last ? 3 : (lev == 1 ? 1 : 2), bytes);
            dispatch_level(W, p, grid, last, st);
            prof_end(ctx, prec);
        }
        if (te_full) {
            unsigned long long *tep = (unsigned long long *)te;
            hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, st, tep, 64 * W);
            const int sgrid = ctx->num_cu * 4;
            const uint64_t *visp = (const uint64_t *)vis;
            switch (W) {
                case 1: launch_scanned<1>(sgrid, st, n, g->row_ptr, g->col, alive, visp, tep); break;
                case 2: launch_scanned<2>(sgrid, st, n, g->row_ptr, g->col, alive, visp, tep); break;
                case 4: launch_scanned<4>(sgrid, st, n, g->row_ptr, g->col, alive, visp, tep); break;
                case 8: launch_scanned<8>(sgrid, st, n, g->row_ptr, g->col, alive, visp, tep); break;
                case 16: launch_scanned<16>(sgrid, st, n, g->row_ptr, g->col, alive, visp, tep); break;
                default: launch_scanned<32>(sgrid, st, n, g->row_ptr, g->col, alive, visp, tep); break;
            }
            hipLaunchKernelGGL(te_scatter_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, srcs, first,
                               cnt, (const unsigned long long *)tep, te_full);
        } else {
            hipLaunchKernelGGL(batch_scatter_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, srcs,
                               first, cnt, (const uint32_t *)counts, deg_list, scatter ? deg_full : nullptr);
        }
        first += cnt;
    }
    return check_hip(ctx, hipGetLastError(), "msbfs launch");
}

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
