// Host-driven multi-source bounded BFS (gfx950): h-degrees of a list of
// sources in batches of 64*W, one kernel launch per BFS level.  The level
// itself is lvl::level_body (khc_level.h).
#include "khc_level.h"

namespace khc {

namespace {

using namespace lvl;

template <int W, bool LAST>
__global__ __launch_bounds__(kBlockThreads) void level_kernel(LevelParams p) {
    __shared__ LevelLds<W> sh;
    level_body<W, LAST>(p, sh);
}

// Reset the per-batch counters: level work counters, frontier list sizes
// and degree totals, per-lane counts.
__global__ void batch_reset_kernel(uint32_t *work, uint32_t *qcnt, uint32_t *hcnt,
                                   unsigned long long *qdeg, int nlev, uint32_t *counts, int ncounts) {
    for (int i = threadIdx.x; i < nlev; i += blockDim.x) {
        work[i] = 0;
        qcnt[i] = 0;
        hcnt[i] = 0;
        qdeg[2 * i] = 0;
        qdeg[2 * i + 1] = 0;
    }
    for (int i = threadIdx.x; i < ncounts; i += blockDim.x) counts[i] = 0;
}

// Put source lane l on its vertex: vis and the level-0 frontier get bit l,
// and the vertex becomes entry l of the level-0 frontier list.  A dead
// source is listed but not seeded; its lane stays empty and reports 0.
// srcs == null means the implicit list first, first+1, ...  A vertex listed
// twice is seeded on both lanes and listed twice on the level-0 frontier;
// pushing a row twice finds no new bits the second time, so both lanes
// report its h-degree.
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
    // a caller's list may name one vertex twice: two lanes of one word can
    // then seed the same row, so the bits go in with atomics
    atomicOr((unsigned long long *)&vis[(size_t)s * W + (l >> 6)], (unsigned long long)bit);
    atomicOr((unsigned long long *)&f0[(size_t)s * W + (l >> 6)], (unsigned long long)bit);
    atomicOr(&fnz0[s >> 5], 1u << (s & 31));
    const uint64_t ds = row_ptr[s + 1] - row_ptr[s];
    atomicAdd(f.qdeg, (unsigned long long)ds);
    atomicAdd(f.qdeg + 1, (unsigned long long)ds);  // one non-zero word per seeded lane
    add_push_items(f, s, ds);
}

// End of a batch, in one launch: per-lane results to their sources, the
// touched rows cleared (vis rows of every frontier list, frontier buffer
// rows and map words of the last two lists; older ones were cleared by the
// levels), and the other counter set zeroed for the next batch.
struct BatchEnd {
    const uint32_t *srcs;
    uint32_t first, cnt;
    const uint32_t *counts;
    uint32_t *deg_list, *deg_full;
    const uint32_t *qbase;
    uint32_t n;
    const uint32_t *qcnt;
    uint32_t levels;
    uint64_t *vis;
    uint64_t *frt[3];
    uint32_t *fnz;
    uint32_t fnz_words;
    int W;
    // counter set of the next batch
    uint32_t *nwork, *nqcnt, *nhcnt, *ncounts;
    unsigned long long *nqdeg;
    uint32_t nq, ncounts_len;
};

__global__ void batch_end_kernel(BatchEnd b) {
    const size_t gt = (size_t)blockIdx.x * blockDim.x + threadIdx.x, gs = (size_t)gridDim.x * blockDim.x;
    for (size_t l = gt; l < b.cnt; l += gs) {
        const uint32_t d = b.counts[l];
        if (b.deg_full) {
            const uint32_t s = b.srcs ? b.srcs[b.first + l] : b.first + (uint32_t)l;
            b.deg_full[s] = d;
        } else if (b.deg_list) {
            b.deg_list[b.first + l] = d;
        }
    }
    const int W = b.W;
    for (uint32_t j = 0; j <= b.levels; ++j) {
        const uint32_t c = b.qcnt[j];
        const uint32_t *q = b.qbase + (size_t)j * b.n;
        const bool recent = j + 1 >= b.levels;
        uint64_t *buf = b.frt[j % 3];
        uint32_t *fz = b.fnz + (size_t)(j % 3) * b.fnz_words;
        for (size_t i = gt; i < (size_t)c * W; i += gs) {
            const size_t at = (size_t)q[i / W] * W + (i % W);
            b.vis[at] = 0;
            if (recent) buf[at] = 0;
        }
        if (recent)
            for (size_t i = gt; i < c; i += gs) fz[q[i] >> 5] = 0;
    }
    for (size_t i = gt; i < b.nq; i += gs) {
        b.nwork[i] = 0;
        b.nqcnt[i] = 0;
        b.nhcnt[i] = 0;
        b.nqdeg[2 * i] = 0;
        b.nqdeg[2 * i + 1] = 0;
    }
    for (size_t i = gt; i < b.ncounts_len; i += gs) b.ncounts[i] = 0;
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

// Row-count mode (the local h-degree update): after the last level of a
// batch, every listed row u adds the number of this batch's lanes that
// reached it and whose source index is below limit(u), the end of the
// sources at distance <= h - s(u) from the removed set, s(u) = mark[u] - 1
// (sources are listed by that distance; lvl[j] counts those at distance j).
__global__ void row_count_kernel(RowCount rc, const uint64_t *vis, int W, uint32_t first) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < rc.nrows; i += gridDim.x * blockDim.x) {
        const uint32_t u = rc.rows[i];
        const uint32_t s = rc.mark[u] - 1u;
        uint32_t limit = 0;
        for (uint32_t j = 0; j + s <= rc.h; ++j) limit += rc.lvl[j];
        if (limit <= first) continue;
        const uint32_t span = limit - first;  // lanes [0, span) of this batch count
        uint32_t c = 0;
        for (int w = 0; w < W && (uint32_t)w * 64u < span; ++w) {
            uint64_t bits = vis[(size_t)u * W + w];
            const uint32_t left = span - (uint32_t)w * 64u;
            if (left < 64u) bits &= (1ull << left) - 1ull;
            c += (uint32_t)__builtin_popcountll(bits);
        }
        if (c) rc.acc[u] += c;
    }
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
// Buffers of the multi-source BFS, in this order: vis, three frontier
// buffers, frontier maps, heavy-row accumulators and completion counters,
// per-lane counts, counters, frontier lists, push items, list table, and
// scanned-arc totals (te mode only).
enum { B_VIS, B_F0, B_F1, B_F2, B_FNZ, B_HACC, B_HDONE, B_COUNTS, B_MISC, B_QUEUES, B_HQUEUES, B_QPTRS, B_TE, B_NUM };
const int kBufSlot[B_NUM] = {WS_VIS,  WS_FRT0,   WS_FRT1,   WS_FRT2,    WS_FNZ,    WS_HACC, WS_HDONE,
                             WS_COUNTS, WS_MISC, WS_BQUEUE, WS_HQUEUE, WS_QPTRS, WS_TE};

void msbfs_sizes(const khc_graph *g, uint32_t nq, int maxW, bool te, size_t *sz) {
    const uint32_t n = g->n;
    const size_t words = (size_t)n * maxW;
    const uint32_t fnz_words = (n + 31) / 32;
    // push items per level: at most one per row plus one per kPushChunk arcs
    const size_t hq_len = (size_t)n + g->nnz / kPushChunk + 1;
    sz[B_VIS] = sz[B_F0] = sz[B_F1] = sz[B_F2] = words * 8;
    sz[B_FNZ] = (size_t)fnz_words * 3 * 4;
    sz[B_HACC] = ((size_t)g->n_heavy + 1) * maxW * 8;
    sz[B_HDONE] = ((size_t)g->n_heavy + 1) * 4;
    sz[B_COUNTS] = (size_t)2 * 64 * kMaxWidth * 4;
    sz[B_MISC] = (size_t)2 * (nq * 32 + 64);
    sz[B_QUEUES] = (size_t)nq * n * 4 + 4;
    sz[B_HQUEUES] = (size_t)nq * hq_len * 8;
    sz[B_QPTRS] = (size_t)nq * 8;
    sz[B_TE] = te ? (size_t)64 * kMaxWidth * 8 : 0;
}

int msbfs_run(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
              const uint32_t *srcs, uint32_t nsrc, uint32_t *deg_list, int scatter,
              uint32_t *deg_full, uint64_t *te_full, uint32_t *const *level_out = nullptr,
              Arena *arena = nullptr, int arena_width = 0, const uint8_t *count_mask = nullptr,
              const RowCount *row_count = nullptr) {
    if (nsrc == 0) return KHC_OK;
    const uint32_t levels = te_full ? h - 1 : h;
    const uint32_t n = g->n;
    const int maxW = arena ? arena_width : ctx->max_width;
    const uint32_t fnz_words = (n + 31) / 32;
    const uint32_t nq = levels + 1;  // frontier lists 0..levels
    const size_t hq_len = (size_t)n + g->nnz / kPushChunk + 1;
    size_t sz[B_NUM];
    msbfs_sizes(g, nq, maxW, te_full != nullptr, sz);
    void *buf[B_NUM] = {};
    for (int b = 0; b < B_NUM; ++b) {
        if (!sz[b]) continue;
        if (!arena) {
            int rc = ws_get(ctx, kBufSlot[b], sz[b], &buf[b]);
            if (rc) return rc;
        } else if (!(buf[b] = arena->take(sz[b]))) {
            return set_error(ctx, KHC_ENOMEM, "BFS buffers exceed the caller's scratch region");
        }
    }
    if (arena) {
        // a carved region holds whatever its last user left: the buffers the
        // levels expect to start zero are cleared here
        for (int b : {B_VIS, B_F0, B_F1, B_F2, B_FNZ, B_HACC, B_HDONE})
            fill_u32(ctx, (uint32_t *)buf[b], 0u, sz[b] / 4);
    }
    void *vis = buf[B_VIS], *f0 = buf[B_F0], *f1 = buf[B_F1], *f2 = buf[B_F2], *fnz = buf[B_FNZ];
    void *hacc = buf[B_HACC], *hdone = buf[B_HDONE], *counts = buf[B_COUNTS], *misc = buf[B_MISC];
    void *queues = buf[B_QUEUES], *hqueues = buf[B_HQUEUES], *qptrs = buf[B_QPTRS], *te = buf[B_TE];
    uint64_t *frt[3] = {(uint64_t *)f0, (uint64_t *)f1, (uint64_t *)f2};
    uint32_t *fnzp = (uint32_t *)fnz;
    // Two counter sets, used by alternate batches (the end of a batch zeros
    // the other): misc = [set 0: qdeg[2 nq] (u64 pairs), work, qcnt, hcnt
    // (u32)] then set 1; counts = per-lane totals of set 0 then set 1.
    unsigned long long *qdeg_s[2];
    uint32_t *work_s[2], *qcnt_s[2], *hcnt_s[2], *counts_s[2];
    for (int ps = 0; ps < 2; ++ps) {
        qdeg_s[ps] = (unsigned long long *)((char *)misc + (size_t)ps * (nq * 32 + 64));
        work_s[ps] = (uint32_t *)(qdeg_s[ps] + 2 * nq);
        qcnt_s[ps] = work_s[ps] + nq;
        hcnt_s[ps] = qcnt_s[ps] + nq;
        counts_s[ps] = (uint32_t *)counts + (size_t)ps * 64 * kMaxWidth;
    }
    unsigned long long *qdeg = qdeg_s[0];
    uint32_t *work = work_s[0], *qcnt = qcnt_s[0], *hcnt = hcnt_s[0];
    uint32_t *qbase = (uint32_t *)queues;
    uint64_t *hqbase = (uint64_t *)hqueues;
    auto Q = [&](uint32_t j) { return qbase + (size_t)j * n; };
    auto F = [&](uint32_t j) {
        Frontier f;
        f.q = Q(j);
        f.qcnt = qcnt + j;
        f.qdeg = qdeg + 2 * j;
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

    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, st, work_s[0], qcnt_s[0], hcnt_s[0], qdeg_s[0],
                       (int)nq, counts_s[0], 64 * kMaxWidth);
    for (uint32_t first = 0, parity = 0; first < nsrc; parity ^= 1u) {
        const uint32_t remaining = nsrc - first;
        // one batch as narrow as holds the rest: a pull level costs a large
        // fixed part (a latency-bound pass over every row) plus a little per
        // word, so splitting a batch into narrower ones never pays
        const int W = width_for(remaining, maxW);
        const uint32_t cnt = remaining < (uint32_t)(64 * W) ? remaining : (uint32_t)(64 * W);
        qdeg = qdeg_s[parity];
        work = work_s[parity];
        qcnt = qcnt_s[parity];
        hcnt = hcnt_s[parity];
        counts = counts_s[parity];
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
            p.push_cost = (uint32_t)ctx->push_cost;
            p.count_mask = count_mask;
            // rows without arcs are a suffix of the schedule: they can never
            // gain a bit, so the pull does not visit them
            p.light_lo = 0;
            p.light_hi = g->n_light_nz;
            p.chunk_lo = 0;
            p.chunk_hi = g->n_chunks;
            p.count_keep = 0;
            p.gid = nullptr;  // one graph, or batched graphs with every lane of every row read
            p.seg_pfx = nullptr;
            p.batch_base = 0;
            // algorithmic bytes of a pull level over the whole graph
            const double bytes = alive ? 0.0
                                       : (double)n * (8.0 + 8.0 * W) + (double)g->nnz * (4.0 + 8.0 * W);
            // row-count mode reads vis after the last level, so every level writes it
            const bool last = !te_full && !row_count && lev == h;
            const int prec = arena ? -1 : prof_begin(ctx, last ? 3 : (lev == 1 ? 1 : 2), bytes);
            dispatch_level(W, p, grid, last, st);
            prof_end(ctx, prec);
            // cumulative counts after level lev are the lev-hop degrees
            if (level_out && level_out[lev - 1] && !last)
                hipLaunchKernelGGL(batch_scatter_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, srcs, first,
                                   cnt, (const uint32_t *)counts, (uint32_t *)nullptr, level_out[lev - 1]);
        }
        if (row_count && row_count->nrows)
            hipLaunchKernelGGL(row_count_kernel, dim3((row_count->nrows + 255) / 256 < 4096 ? (row_count->nrows + 255) / 256 : 4096),
                               dim3(256), 0, st, *row_count, (const uint64_t *)vis, W, first);
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
        }
        BatchEnd be;
        be.srcs = srcs;
        be.first = first;
        be.cnt = te_full ? 0u : cnt;
        be.counts = (const uint32_t *)counts;
        be.deg_list = scatter ? nullptr : deg_list;
        be.deg_full = scatter ? deg_full : nullptr;
        be.qbase = qbase;
        be.n = n;
        be.qcnt = qcnt;
        be.levels = levels;
        be.vis = (uint64_t *)vis;
        for (int i = 0; i < 3; ++i) be.frt[i] = frt[i];
        be.fnz = fnzp;
        be.fnz_words = fnz_words;
        be.W = W;
        be.nwork = work_s[parity ^ 1u];
        be.nqcnt = qcnt_s[parity ^ 1u];
        be.nhcnt = hcnt_s[parity ^ 1u];
        be.nqdeg = qdeg_s[parity ^ 1u];
        be.ncounts = counts_s[parity ^ 1u];
        be.nq = nq;
        be.ncounts_len = 64u * kMaxWidth;
        const int prec = arena ? -1 : prof_begin(ctx, 0, 0.0);
        hipLaunchKernelGGL(batch_end_kernel, dim3(ctx->num_cu * 4), dim3(256), 0, st, be);
        prof_end(ctx, prec);
        first += cnt;
    }
    return check_hip(ctx, hipGetLastError(), "msbfs launch");
}

}  // namespace

int msbfs_degrees(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                  const uint32_t *srcs, uint32_t nsrc, uint32_t *deg_list, int scatter,
                  uint32_t *deg_full, Arena *arena, int arena_width) {
    return msbfs_run(ctx, g, alive, h, srcs, nsrc, deg_list, scatter, deg_full, nullptr, nullptr, arena,
                     arena_width);
}

size_t msbfs_arena_bytes(const khc_graph *g, uint32_t h, int W) {
    size_t sz[B_NUM];
    msbfs_sizes(g, h + 1, W, false, sz);
    size_t total = 0;
    for (int b = 0; b < B_NUM; ++b)
        if (sz[b]) total = ((total + 255) & ~(size_t)255) + sz[b];
    return total;
}

int msbfs_masked_counts(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                        const uint32_t *srcs, uint32_t nsrc, const uint8_t *count_mask, uint32_t *deg_full) {
    return msbfs_run(ctx, g, alive, h, srcs, nsrc, nullptr, 1, deg_full, nullptr, nullptr, nullptr, 0, count_mask);
}

int msbfs_row_counts(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, const uint32_t *srcs,
                     uint32_t nsrc, const RowCount &rc) {
    return msbfs_run(ctx, g, alive, h, srcs, nsrc, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, nullptr, &rc);
}

int msbfs_scanned_arcs(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                       const uint32_t *srcs, uint32_t nsrc, uint64_t *te_full) {
    return msbfs_run(ctx, g, alive, h, srcs, nsrc, nullptr, 1, nullptr, te_full);
}

int msbfs_all_levels(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t levels,
                     const uint32_t *srcs, uint32_t nsrc, uint32_t *const *level_out) {
    return msbfs_run(ctx, g, alive, levels, srcs, nsrc, nullptr, 1, level_out[levels - 1], nullptr, level_out);
}

}  // namespace khc
