// Device-resident (k,h)-core peeling: one persistent kernel runs the whole
// decomposition (gfx950).
//
// The host-driven driver (khc_peel.hip) pays a kernel launch per step and a
// host round trip per round; peeling needs hundreds to tens of thousands of
// rounds, most of them small.  Here every step is a phase of one persistent
// kernel whose workgroups are all resident (grid sized from the occupancy
// of this kernel), and phases are separated by grid barriers.  Each barrier
// wait has a wall-clock deadline: a wait that exceeds it raises an abort
// flag that every workgroup checks, so the kernel always exits.  The launch
// is captured once in a hipGraph and replayed.
//
// The algorithm is a bounded schedule of khc_peel.hip (or the plain one):
// levels k <- max(k, min key), dirty vertices whose lower bound reaches the
// level are recomputed first, P = {clean live v : d(v) <= k} is removed, the
// vertices within h hops of P in the graph before removal are found by a
// push BFS, the (h-1)-degrees near P are brought up to date, and the
// vertices within h hops of P become dirty with fresh lower bounds.  The
// (h-1)-degrees of the ring at distance h-1 from P lose |P|; those within
// h-2 hops of P are recomputed exactly (schedule 1) or lowered by the
// decrement bound and refreshed whenever the vertex's h-degree is
// recomputed, from the same BFS (schedule 3).
//
// Several graphs can be decomposed together: their disjoint union is one
// CSR and gid[v] names the graph of v.  Each graph keeps its own level
// K[g]; every step removes, in every graph that still has vertices, the
// vertices at or below that graph's level, so a graph's removal rounds are
// the steps and each graph's core numbers are exactly its own (core numbers
// of a disjoint union are per component).  Sources of different graphs
// share BFS batches: the graphs are disjoint, so their lanes never meet.
#include <chrono>
#include <cstring>
#include <thread>

#include "khc_level.h"

namespace khc {
namespace {

using namespace lvl;

constexpr int kMaxPersistH = 32;
constexpr uint32_t kAffChunk = 1024;  // arcs per work item of a heavy affected-BFS row

struct PCtl {
    unsigned long long left;  // live vertices
    uint32_t rn;              // dirty vertices to recompute
    uint32_t round;
    uint32_t nsrc;            // initial sources (live vertices with a live neighbour)
    uint32_t abort_reason;
    uint32_t acnt[kMaxPersistH + 2];   // affected BFS: rows appended per level (0: P)
    uint32_t ahcnt[kMaxPersistH + 2];  // heavy-row work items per level
    unsigned long long stat_hrec, stat_hm1, stat_aff, stat_batches;
    // per phase: wall-clock ticks from the previous barrier to the end of
    // the phase's own barrier, and how often it ran (workgroup 0's view)
    unsigned long long phase_ticks[KHC_PERSIST_PHASES], phase_count[KHC_PERSIST_PHASES];
};

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b % 8), and each XCD has its own L2, which is not coherent with the
// others for ordinary device memory.  The barrier therefore groups
// workgroups by XCD: members release at workgroup scope (their stores reach
// the XCD's L2) and, after the barrier, invalidate only their CU's L1; the
// last arrival of each XCD writes back and invalidates that XCD's L2 once
// (agent-scope fences) around the global step.  Every workgroup reads its
// hardware XCC id when the kernel starts; if the placement is not b % 8 the
// run aborts before its first barrier completes and the host reruns it with
// the flat barrier, in which every workgroup releases and acquires at agent
// scope (correct on any placement, slower).
constexpr uint32_t kXcds = 8;

// Barrier words: count[0] global arrivals, gen[0] global generation,
// abort[0]; then per group g: gcount[g], ggen[g] (each on its own 128-byte
// line to keep pollers of different groups apart).
struct Sync {
    uint32_t *count;
    uint32_t *gen;
    uint32_t *abort;
    uint32_t *groups;  // group g: groups[g * 32] arrivals, groups[g * 32 + 16] generation
    uint32_t nblocks;
    uint32_t ngroups;
    uint32_t grouped;  // 1: XCD-grouped barrier, 0: flat barrier
    uint64_t timeout_ticks;
};

// Abort codes in the abort word (the first to set it wins).
enum : uint32_t { ABORT_TIMEOUT = 1, ABORT_PLACEMENT = 2 };

// hwreg(HW_REG_XCC_ID, 0, 4): the XCD this wave runs on.
constexpr int kHwregXccId = 20 | (0 << 6) | ((4 - 1) << 11);

// The graphs a BFS batch covers: their arcs (push/pull choice) and their
// ranges of the light-row and heavy-chunk schedules.
struct BatchRange {
    unsigned long long arcs;
    uint32_t light_lo, light_hi, chunk_lo, chunk_hi;
};

struct PParams {
    const uint64_t *row_ptr;
    const uint32_t *col;
    uint64_t nnz;
    uint32_t n;
    uint32_t n_light, n_chunks;
    const uint32_t *light_rows, *heavy_rows, *chunk_heavy, *chunk_first;
    const uint32_t *gid;  // graph of each vertex (null: one graph)
    uint32_t ngraphs;
    uint32_t h;
    int bounded;  // 0 plain, 1 schedule 1, 2 schedule 3
    uint32_t push_cost;  // push/pull rule of the BFS levels (KHC_OPT_PUSH_COST)
    int profile;  // time the phases (KHC_OPT_PROFILE)
    uint32_t round_limit;  // stop after this many rounds (0: none)
    unsigned long long *progress;  // host-visible [rounds, removed], or null
    // peeling state
    uint8_t *alive, *dirty;
    uint32_t *d, *dm, *lb, *lbx, *mark, *queue, *list, *core, *round;
    uint32_t *K, *MIN;
    uint64_t *ahq;  // affected BFS heavy items, per level
    size_t ahq_len;
    PCtl *ctl;
    // BFS workspace
    uint64_t *vis;
    uint64_t *frt0, *frt1, *frt2;
    uint32_t *fnz;
    uint32_t fnz_words;
    uint64_t *hacc;
    uint32_t *hdone;
    uint32_t *counts;
    uint32_t *counts2;  // split jobs: the last level's per-lane totals
    uint32_t *bq;   // frontier lists, n entries per level
    uint64_t *bhq;  // push items, hq_len per level
    size_t hq_len;
    uint32_t *bqcnt, *bhcnt, *bwork;
    unsigned long long *bqdeg;
    // BFS sources grouped by graph: graph g's sources sit at
    // list[vbase[g] ...) (seg_cnt[g] of them); seg_pfx is their exclusive
    // prefix over graphs, computed when a job starts.
    uint32_t *seg_cnt, *seg_pfx;
    const uint64_t *vbase;      // graph offsets [ngraphs + 1] (null: one graph)
    const uint32_t *light_first, *gchunk_first;  // schedule ranges per graph (null: one graph)
    BatchRange *brange;         // what the current batch covers
    uint32_t *gring;            // graphs packed together: ring sizes [graph][0..h] of the round
    Sync sync;
};

// Wait until *word != g; false on abort or deadline (which raises abort).
__device__ bool wait_change(const Sync &s, const uint32_t *word, uint32_t g) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(word, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(s.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > s.timeout_ticks) {
            atomicCAS(s.abort, 0u, (uint32_t)ABORT_TIMEOUT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Two-level grid barrier.  Thread 0 of each workgroup arrives at its
// group's counter; the last of a group arrives at the global counter; the
// last group resets the global counter and bumps the global generation.
// Each group's last arrival waits for the global generation and then bumps
// its group's generation, which the rest of the group polls.  Every wait
// has a deadline and watches the abort flag.  Returns false if the kernel
// must exit.
__device__ bool grid_sync(const Sync &s, uint32_t *s_gen, uint32_t *s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t g = *s_gen;
        uint32_t ok = 1;
        if (s.grouped) {
            const uint32_t grp = blockIdx.x % kXcds;
            const uint32_t gsize = s.nblocks / kXcds + (grp < s.nblocks % kXcds ? 1u : 0u);
            uint32_t *gcount = s.groups + grp * 32;
            uint32_t *ggen = s.groups + grp * 32 + 16;
            // the workgroup's stores have reached this XCD's L2
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (atomicAdd(gcount, 1u) == gsize - 1) {
                atomicExch(gcount, 0u);
                __threadfence();  // write back this XCD's L2
                if (atomicAdd(s.count, 1u) == s.ngroups - 1) {
                    atomicExch(s.count, 0u);
                    __threadfence();
                    atomicAdd(s.gen, 1u);
                } else {
                    ok = wait_change(s, s.gen, g) ? 1u : 0u;
                }
                __threadfence();  // invalidate this XCD's L2 (and this CU's L1)
                atomicAdd(ggen, 1u);
            } else {
                ok = wait_change(s, ggen, g) ? 1u : 0u;
                asm volatile("buffer_inv sc0" ::: "memory");  // invalidate this CU's L1
            }
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (atomicAdd(s.count, 1u) == s.nblocks - 1) {
                atomicExch(s.count, 0u);
                atomicAdd(s.gen, 1u);
            } else {
                ok = wait_change(s, s.gen, g) ? 1u : 0u;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (__hip_atomic_load(s.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        *s_gen = g + 1;
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

__device__ __forceinline__ uint32_t graph_of(const PParams &p, uint32_t v) { return p.gid ? p.gid[v] : 0u; }

__device__ __forceinline__ size_t gtid() { return (size_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ size_t gstride() { return (size_t)gridDim.x * blockDim.x; }

__device__ __forceinline__ uint32_t seg_base(const PParams &p, uint32_t g) {
    return p.vbase ? (uint32_t)p.vbase[g] : 0u;
}

// Append the `take` lanes' vertices to their graphs' segments of p.list and
// count them in *total (may be null).  Wave-aggregated when the takers
// share a graph.  Every lane of the wavefront must call it.
__device__ void seg_append(const PParams &p, bool take, uint32_t v, uint32_t *total) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    const uint32_t g = take ? graph_of(p, v) : 0u;
    const uint32_t gl = __shfl(g, leader, 64);
    const uint32_t cnt = (uint32_t)__builtin_popcountll(m);
    if (__ballot(take && g != gl) == 0ull) {
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&p.seg_cnt[gl], cnt);
        base = __shfl(base, leader, 64);
        if (take) p.list[seg_base(p, gl) + base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = v;
    } else if (take) {
        p.list[seg_base(p, g) + atomicAdd(&p.seg_cnt[g], 1u)] = v;
    }
    if (total && lane == leader) atomicAdd(total, cnt);
}

// Graphs packed together: count the `take` lanes' vertices (of graph g)
// in their graph's ring L.  Every lane of the wavefront must call it.
__device__ void ring_count(const PParams &p, bool take, uint32_t g, uint32_t L) {
    if (p.ngraphs == 1) return;
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    const uint32_t gl = __shfl(g, leader, 64);
    if (__ballot(take && g != gl) == 0ull) {
        if (lane == leader) atomicAdd(&p.gring[gl * (p.h + 1) + L], (uint32_t)__builtin_popcountll(m));
    } else if (take) {
        atomicAdd(&p.gring[g * (p.h + 1) + L], 1u);
    }
}

// Size of the rings 0..r around the round's removed set, as seen from
// vertex u (its own graph's rings when graphs are packed together).
__device__ __forceinline__ uint32_t ring_total(const PParams &p, uint32_t u, int r) {
    uint32_t t = 0;
    if (p.ngraphs == 1) {
        for (int q = 0; q <= r; ++q) t += p.ctl->acnt[q];
    } else {
        const uint32_t *row = p.gring + (size_t)graph_of(p, u) * (p.h + 1);
        for (int q = 0; q <= r; ++q) t += row[q];
    }
    return t;
}

// Source slot i of the current job: graph g with seg_pfx[g] <= i < seg_pfx[g+1].
__device__ __forceinline__ uint32_t job_source(const PParams &p, uint32_t i) {
    uint32_t lo = 0, hi = p.ngraphs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (p.seg_pfx[mid] <= i) lo = mid;
        else hi = mid;
    }
    return p.list[seg_base(p, lo) + (i - p.seg_pfx[lo])];
}

// seg_pfx = exclusive prefix of seg_cnt over the graphs (one workgroup).
__device__ void scan_segments(const PParams &p, uint32_t *s_ws) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t G = p.ngraphs;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < G; c0 += kBlockThreads) {
        const uint32_t g = c0 + threadIdx.x;
        const uint32_t x = g < G ? p.seg_cnt[g] : 0u;
        uint32_t v = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = __shfl_up(v, off, 64);
            if (lane >= off) v += t;
        }
        if (lane == 63) s_ws[wave] = v;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int w = 0; w < kBlockThreads / 64; ++w) {
            if (w < wave) before += s_ws[w];
            total += s_ws[w];
        }
        if (g < G) p.seg_pfx[g] = carry + before + v - x;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) p.seg_pfx[G] = carry;
}

__device__ __forceinline__ uint64_t *frt_buf(const PParams &p, uint32_t i) {
    return i == 0 ? p.frt0 : (i == 1 ? p.frt1 : p.frt2);
}

// lb(u) = max(dm(u), max over live neighbours of dm), the neighbours read
// limited to the first kLbArcs; 16 lanes per u.  For the affected vertices
// (list = the round's queue) also the decrement bound: the last exact
// h-degree (or carried bound lbx) minus the number of vertices within h - j
// hops of P, j being u's distance from P.
__device__ void lower_bounds(const PParams &p, const uint32_t *list, uint32_t begin, uint32_t end,
                             bool mark_dirty) {
    const int lane = threadIdx.x & 63, sub = lane & 15;
    const size_t grp = gtid() >> 4, ngrp = gstride() >> 4;
    const size_t trips = ((size_t)(end - begin) + ngrp - 1) / ngrp;
    for (size_t t = 0; t < trips; ++t) {
        const size_t i = begin + t * ngrp + grp;
        uint32_t m = 0, u = 0;
        bool live = false;
        if (i < end) {
            u = list ? list[i] : (uint32_t)i;
            live = p.alive[u] != 0;
        }
        if (live) {
            const uint64_t rb = p.row_ptr[u], re0 = p.row_ptr[u + 1];
            const uint64_t re = re0 - rb > kLbArcs ? rb + kLbArcs : re0;
            for (uint64_t a = rb + sub; a < re; a += 16) {
                const uint32_t w = p.col[a];
                if (p.alive[w] && p.dm[w] > m) m = p.dm[w];
            }
        }
        for (int off = 8; off > 0; off >>= 1) {
            const uint32_t o = __shfl_xor(m, off, 64);
            m = o > m ? o : m;
        }
        if (live && sub == 0) {
            uint32_t b = p.dm[u] > m ? p.dm[u] : m;
            if (list) {
                // decrement bound: u at distance j from P loses at most the
                // vertices within h - j hops of P (P included)
                uint32_t j = 0, at = p.ctl->acnt[0];
                while (i >= at) at += p.ctl->acnt[++j];
                const uint32_t loss = ring_total(p, u, (int)p.h - (int)j);
                const uint32_t base = p.dirty[u] ? p.lbx[u] : p.d[u];
                const uint32_t x = base > loss ? base - loss : 0u;
                p.lbx[u] = x;
                b = b > x ? b : x;
            }
            p.lb[u] = b;
            if (mark_dirty) p.dirty[u] = 1;
        }
    }
}

// Work items of a heavy row in the affected BFS (rows of the next level).
__device__ __forceinline__ void add_aff_items(const PParams &p, uint32_t level, uint32_t y) {
    const uint64_t dy = p.row_ptr[y + 1] - p.row_ptr[y];
    if (dy <= kAffChunk) return;
    const uint32_t nch = (uint32_t)((dy + kAffChunk - 1) / kAffChunk);
    const uint32_t at = atomicAdd(&p.ctl->ahcnt[level], nch);
    uint64_t *items = p.ahq + (size_t)level * p.ahq_len;
    for (uint32_t c = 0; c < nch; ++c) items[at + c] = (uint64_t)y | ((uint64_t)c << 32);
}

// One level of the affected-set BFS (push from the previous level's rows,
// one wavefront per row or per kAffChunk arcs of a heavy row).
__device__ void affected_level(const PParams &p, uint32_t L) {
    uint32_t e_prev2 = 0, e_prev = 0;  // queue[e_prev2, e_prev) is level L-1
    for (uint32_t j = 0; j + 1 < L; ++j) e_prev2 += p.ctl->acnt[j];
    e_prev = e_prev2 + p.ctl->acnt[L - 1];
    const uint32_t nh = p.ctl->ahcnt[L - 1];
    const uint64_t *items = p.ahq + (size_t)(L - 1) * p.ahq_len;
    const uint32_t nl = e_prev - e_prev2;
    const int lane = threadIdx.x & 63;
    const size_t wave = gtid() >> 6, nwaves = gstride() >> 6;
    for (size_t it = wave; it < (size_t)nl + nh; it += nwaves) {
        uint32_t x;
        uint64_t ab, ae;
        if (it < nl) {
            x = p.queue[e_prev2 + it];
            ab = p.row_ptr[x];
            ae = p.row_ptr[x + 1];
            if (ae - ab > kAffChunk) continue;  // covered by its work items
        } else {
            const uint64_t v = items[it - nl];
            x = (uint32_t)v;
            ab = p.row_ptr[x] + (v >> 32) * kAffChunk;
            const uint64_t re = p.row_ptr[x + 1];
            ae = ab + kAffChunk < re ? ab + kAffChunk : re;
        }
        for (uint64_t a0 = ab; a0 < ae; a0 += 64) {
            const uint64_t a = a0 + lane;
            bool take = false;
            uint32_t y = 0;
            if (a < ae) {
                y = p.col[a];
                take = p.alive[y] && p.mark[y] == 0u && atomicCAS(&p.mark[y], 0u, 1u) == 0u;
            }
            const uint64_t m = __ballot(take);
            if (m) {
                const int leader = __builtin_ctzll(m);
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(&p.ctl->acnt[L], (uint32_t)__builtin_popcountll(m));
                base = __shfl(base, leader, 64);
                if (take) {
                    p.queue[e_prev + base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = y;
                    if (L < p.h) add_aff_items(p, L, y);
                }
            }
            ring_count(p, take, take ? graph_of(p, y) : 0u, L);
        }
    }
}

// Phases of the persistent kernel.  Every workgroup runs the same phase,
// then a grid barrier, then computes the next phase from values written
// before that barrier, so all workgroups follow the same sequence.
enum Phase : int {
    PH_INIT,
    PH_COMPACT,
    PH_LB_ALL,
    PH_KEYMIN,
    PH_LEVEL,
    PH_COLLECT,
    PH_CLEAN,
    PH_SELECT,
    PH_AFF,
    PH_KILL,
    PH_LBD,      // lower bounds and dirtiness of the affected set, unmark
    PH_UNMARK,
    PH_BFS_RESET,
    PH_BFS_SEED,
    PH_BFS_LEVEL,
    PH_BFS_SCATTER,
    PH_DONE
};
static_assert((int)PH_DONE + 1 == KHC_PERSIST_PHASES, "phase count of the profile");

// A bounded-BFS job: h-degrees (levels hops) of the n sources grouped by
// graph in p.list into out[] (clearing their dirty flags when clean is
// set), then continue with phase ret.  A split job also writes the
// (levels-1)-hop counts into p.dm: its levels add their totals to counts
// one by one, the last level into counts2.
struct Job {
    uint32_t n, levels;
    uint32_t *out;
    int ret;
    bool clean, split;
};

template <int W>
__global__ __launch_bounds__(kBlockThreads) void peel_persistent_kernel(PParams p) {
    __shared__ LevelLds<W> sh;
    __shared__ uint32_t s_gen, s_ok, s_ws[kBlockThreads / 64];
    if (threadIdx.x == 0) {
        s_gen = 0;
        // the grouped barrier needs workgroup b on XCD b % 8: check, and
        // abort before the first barrier completes if it is not so
        if (p.sync.grouped && (uint32_t)(__builtin_amdgcn_s_getreg(kHwregXccId) & 15) != blockIdx.x % kXcds)
            atomicCAS(p.sync.abort, 0u, (uint32_t)ABORT_PLACEMENT);
    }
    const uint32_t n = p.n, h = p.h;
    const bool bounded = p.bounded != 0, lazy = p.bounded == 2;
    PCtl *ctl = p.ctl;
    const uint32_t per = 64u * W;
    const int lane = threadIdx.x & 63;

    // uniform control state
    int phase = PH_INIT;
    Job job{0, 0, nullptr, PH_DONE, false, false};
    uint32_t batch = 0, lev = 0, aff_l = 0, np = 0, e_hm2 = 0, e_hm1 = 0, e_h = 0;
    auto start_job = [&](uint32_t cnt, uint32_t levels, uint32_t *out, int ret, bool clean, bool split) {
        job = Job{cnt, levels, out, ret, clean, split};
        batch = 0;
        return cnt ? (int)PH_BFS_RESET : ret;
    };

    uint64_t t_prev = wall_clock64();
    for (;;) {
        // ------------------------------------------------------------ work
        switch (phase) {
            case PH_INIT:
                for (size_t v = gtid(); v < n; v += gstride()) {
                    p.alive[v] = 1;
                    p.dirty[v] = 0;
                    p.mark[v] = 0;
                    p.core[v] = 0;
                    if (p.round) p.round[v] = 0;
                    p.d[v] = 0;
                    p.dm[v] = 0;
                }
                for (size_t g = gtid(); g < p.ngraphs; g += gstride()) {
                    p.K[g] = 0;
                    p.MIN[g] = 0xFFFFFFFFu;
                    p.seg_cnt[g] = 0;
                }
                if (gtid() == 0) {
                    ctl->left = n;
                    ctl->rn = 0;
                    ctl->round = 0;
                    ctl->nsrc = 0;
                    ctl->abort_reason = 0;
                    for (int i = 0; i < kMaxPersistH + 2; ++i) ctl->acnt[i] = ctl->ahcnt[i] = 0;
                    ctl->stat_hrec = ctl->stat_hm1 = ctl->stat_aff = ctl->stat_batches = 0;
                    for (int i = 0; i < KHC_PERSIST_PHASES; ++i) ctl->phase_ticks[i] = ctl->phase_count[i] = 0;
                }
                break;
            case PH_COMPACT:
                // sources of the initial degrees: vertices with a neighbour
                for (size_t v0 = gtid() - lane; v0 < n; v0 += gstride()) {
                    const size_t v = v0 + lane;
                    const bool take = v < n && p.row_ptr[v + 1] > p.row_ptr[v];
                    seg_append(p, take, (uint32_t)v, &ctl->nsrc);
                }
                if (gtid() == 0) {
                    ctl->stat_hrec += n;
                    if (bounded) ctl->stat_hm1 += n;
                }
                break;
            case PH_LB_ALL:
                lower_bounds(p, nullptr, 0, n, false);
                break;
            case PH_KEYMIN:
                // per-graph minimum key; a wavefront whose 64 vertices share
                // a graph (the usual case: graphs are contiguous) reduces first
                for (size_t v0 = gtid() - lane; v0 < n; v0 += gstride()) {
                    const size_t v = v0 + lane;
                    uint32_t key = 0xFFFFFFFFu, g = 0;
                    if (v < n) {
                        g = graph_of(p, (uint32_t)v);
                        if (p.alive[v]) key = (bounded && p.dirty[v]) ? p.lb[v] : p.d[v];
                    }
                    const uint32_t g0 = __shfl(g, 0, 64);
                    if (__ballot(v < n && g != g0) == 0ull) {
                        for (int off = 32; off > 0; off >>= 1) {
                            const uint32_t o = __shfl_xor(key, off, 64);
                            key = o < key ? o : key;
                        }
                        if (lane == 0 && key < p.MIN[g0]) atomicMin(&p.MIN[g0], key);
                    } else if (v < n && key < p.MIN[g]) {
                        atomicMin(&p.MIN[g], key);
                    }
                }
                break;
            case PH_LEVEL:
                for (size_t g = gtid(); g < p.ngraphs; g += gstride()) {
                    const uint32_t m = p.MIN[g];
                    if (m != 0xFFFFFFFFu && m > p.K[g]) p.K[g] = m;
                    p.MIN[g] = 0xFFFFFFFFu;
                    p.seg_cnt[g] = 0;
                }
                if (p.ngraphs > 1)
                    for (size_t i = gtid(); i < (size_t)p.ngraphs * (h + 1); i += gstride()) p.gring[i] = 0;
                if (gtid() == 0) {
                    ctl->rn = 0;
                    for (int i = 0; i < kMaxPersistH + 2; ++i) ctl->acnt[i] = ctl->ahcnt[i] = 0;
                }
                break;
            case PH_COLLECT:
                // dirty vertices whose lower bound reached their graph's level
                for (size_t v0 = gtid() - lane; v0 < n; v0 += gstride()) {
                    const size_t v = v0 + lane;
                    const bool take =
                        v < n && p.alive[v] && p.dirty[v] && p.lb[v] <= p.K[graph_of(p, (uint32_t)v)] &&
                        p.d[v] > p.K[graph_of(p, (uint32_t)v)];
                    seg_append(p, take, (uint32_t)v, &ctl->rn);
                }
                break;
            case PH_CLEAN:
                // the job's scatter cleared the recomputed vertices' dirty flags
                if (gtid() == 0) {
                    ctl->stat_hrec += ctl->rn;
                    if (lazy) ctl->stat_hm1 += ctl->rn;
                }
                break;
            case PH_SELECT: {
                // P: clean live vertices at or below their graph's level
                const uint32_t r = ctl->round;
                for (size_t v0 = gtid() - lane; v0 < n; v0 += gstride()) {
                    const size_t v = v0 + lane;
                    bool take = false;
                    // d is exact when clean and an upper bound when dirty
                    if (v < n && p.alive[v]) {
                        const uint32_t k = p.K[graph_of(p, (uint32_t)v)];
                        if (p.d[v] <= k) {
                            take = true;
                            p.core[v] = k;
                            if (p.round) p.round[v] = r;
                            p.mark[v] = 1;
                        }
                    }
                    const uint64_t m = __ballot(take);
                    if (m) {
                        const int leader = __builtin_ctzll(m);
                        uint32_t base = 0;
                        if (lane == leader) base = atomicAdd(&ctl->acnt[0], (uint32_t)__builtin_popcountll(m));
                        base = __shfl(base, leader, 64);
                        if (take) {
                            p.queue[base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = (uint32_t)v;
                            add_aff_items(p, 0, (uint32_t)v);
                        }
                    }
                    ring_count(p, take, take ? graph_of(p, (uint32_t)v) : 0u, 0);
                }
                break;
            }
            case PH_AFF:
                affected_level(p, aff_l);
                break;
            case PH_KILL: {
                np = ctl->acnt[0];
                e_hm2 = e_hm1 = e_h = 0;
                for (uint32_t j = 0; j <= h; ++j) {
                    if (j + 1 < h) e_hm2 += ctl->acnt[j];
                    if (j < h) e_hm1 += ctl->acnt[j];
                    e_h += ctl->acnt[j];
                }
                for (size_t i = gtid(); i < np; i += gstride()) p.alive[p.queue[i]] = 0;
                if (bounded)
                    // (h-1)-degree bounds: a vertex at distance j from P loses
                    // at most the vertices within h-1-j hops of P (P itself
                    // for the ring at distance h-1); schedule 1 recomputes
                    // the rings nearer P below instead
                    for (size_t i = (lazy ? np : e_hm2) + gtid(); i < e_hm1; i += gstride()) {
                        uint32_t j = 0, at = ctl->acnt[0];
                        while (i >= at) at += ctl->acnt[++j];
                        const uint32_t u = p.queue[i];
                        const uint32_t loss = ring_total(p, u, (int)h - 1 - (int)j);
                        p.dm[u] = p.dm[u] > loss ? p.dm[u] - loss : 0u;
                    }
                if (!lazy) {
                    // sources of the recompute job, grouped by graph: the
                    // (h-1)-degrees within h-2 hops of P (bounded) or the
                    // h-degrees of the whole affected set (plain)
                    const uint32_t span = (bounded ? e_hm2 : e_h) - np;
                    for (size_t i0 = gtid() - lane; i0 < span; i0 += gstride()) {
                        const size_t i = i0 + lane;
                        const bool take = i < span;
                        seg_append(p, take, take ? p.queue[np + i] : 0u, nullptr);
                    }
                }
                if (gtid() == 0) {
                    ctl->left -= np;
                    ctl->round += 1;
                    if (p.progress) {
                        __hip_atomic_store(&p.progress[0], (unsigned long long)ctl->round, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        __hip_atomic_store(&p.progress[1], (unsigned long long)(n - ctl->left), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                    }
                    ctl->stat_aff += e_h - np;
                    if (!bounded) ctl->stat_hrec += e_h - np;
                    else if (!lazy) ctl->stat_hm1 += e_hm2 - np;
                    if (np == 0) {
                        ctl->abort_reason = 1;
                        atomicExch(p.sync.abort, 1u);
                    }
                }
                break;
            }
            case PH_LBD:
                lower_bounds(p, p.queue, np, e_h, true);
                for (size_t i = gtid(); i < e_h; i += gstride()) p.mark[p.queue[i]] = 0;
                break;
            case PH_UNMARK:
                for (size_t i = gtid(); i < e_h; i += gstride()) p.mark[p.queue[i]] = 0;
                break;
            case PH_BFS_RESET:
                if (blockIdx.x == 0) {
                    for (uint32_t i = threadIdx.x; i <= job.levels; i += blockDim.x) {
                        p.bwork[i] = 0;
                        p.bqcnt[i] = 0;
                        p.bhcnt[i] = 0;
                        p.bqdeg[2 * i] = 0;
                        p.bqdeg[2 * i + 1] = 0;
                    }
                    for (uint32_t i = threadIdx.x; i < per; i += blockDim.x) p.counts[i] = p.counts2[i] = 0;
                    if (threadIdx.x == 0) ctl->stat_batches++;
                    if (batch == 0) scan_segments(p, s_ws);
                }
                break;
            case PH_BFS_SEED: {
                // lane l of the batch on its source, level-0 list entry l
                const uint32_t first = batch * per;
                const uint32_t cnt = job.n - first < per ? job.n - first : per;
                Frontier f0;
                f0.q = p.bq;
                f0.qcnt = p.bqcnt;
                f0.qdeg = p.bqdeg;
                f0.hq = p.bhq;
                f0.hcnt = p.bhcnt;
                if (gtid() == 0) {
                    // the graphs this batch covers (sources are grouped by graph)
                    BatchRange br{p.nnz, 0u, p.n_light, 0u, p.n_chunks};
                    if (p.vbase) {
                        const uint32_t ga = graph_of(p, job_source(p, first));
                        const uint32_t gb = graph_of(p, job_source(p, first + cnt - 1));
                        br.arcs = p.row_ptr[p.vbase[gb + 1]] - p.row_ptr[p.vbase[ga]];
                        br.light_lo = p.light_first[ga];
                        br.light_hi = p.light_first[gb + 1];
                        br.chunk_lo = p.gchunk_first[ga];
                        br.chunk_hi = p.gchunk_first[gb + 1];
                    }
                    *p.brange = br;
                }
                for (size_t l = gtid(); l < cnt; l += gstride()) {
                    const uint32_t s = job_source(p, first + (uint32_t)l);
                    f0.q[l] = s;
                    if (!p.alive[s]) continue;
                    const uint64_t bit = 1ull << (l & 63);
                    p.vis[(size_t)s * W + (l >> 6)] |= bit;
                    p.frt0[(size_t)s * W + (l >> 6)] |= bit;
                    atomicOr(&p.fnz[s >> 5], 1u << (s & 31));
                    const uint64_t ds = p.row_ptr[s + 1] - p.row_ptr[s];
                    atomicAdd(f0.qdeg, (unsigned long long)ds);
                    atomicAdd(f0.qdeg + 1, (unsigned long long)ds);
                    add_push_items(f0, s, ds);
                }
                if (gtid() == 0) *f0.qcnt = cnt;
                break;
            }
            case PH_BFS_LEVEL: {
                LevelParams lp;
                lp.row_ptr = p.row_ptr;
                lp.col = p.col;
                lp.alive = p.alive;
                lp.light_rows = p.light_rows;
                lp.heavy_rows = p.heavy_rows;
                lp.chunk_heavy = p.chunk_heavy;
                lp.chunk_first = p.chunk_first;
                lp.frt_in = frt_buf(p, (lev - 1) % 3);
                lp.frt_out = frt_buf(p, lev % 3);
                lp.frt_clr = frt_buf(p, (lev + 1) % 3);
                lp.vis = p.vis;
                lp.q_in = p.bq + (size_t)(lev - 1) * n;
                lp.hq_in = p.bhq + (size_t)(lev - 1) * p.hq_len;
                lp.qcnt_in = p.bqcnt + lev - 1;
                lp.hcnt_in = p.bhcnt + lev - 1;
                lp.qdeg_in = p.bqdeg + 2 * (lev - 1);
                lp.out.q = p.bq + (size_t)lev * n;
                lp.out.qcnt = p.bqcnt + lev;
                lp.out.qdeg = p.bqdeg + 2 * lev;
                lp.out.hq = p.bhq + (size_t)lev * p.hq_len;
                lp.out.hcnt = p.bhcnt + lev;
                lp.q_clr = lev >= 2 ? p.bq + (size_t)(lev - 2) * n : nullptr;
                lp.qcnt_clr = lev >= 2 ? p.bqcnt + lev - 2 : nullptr;
                lp.fnz_out = p.fnz + (size_t)(lev % 3) * p.fnz_words;
                lp.fnz_clr = p.fnz + (size_t)((lev + 1) % 3) * p.fnz_words;
                lp.hacc = p.hacc;
                lp.hdone = p.hdone;
                lp.work = p.bwork + lev;
                lp.counts = (job.split && lev == job.levels) ? p.counts2 : p.counts;
                lp.count_keep = job.split ? 0 : 1;
                lp.count_first = lev == 1;
                const BatchRange br = *p.brange;
                lp.nnz = br.arcs;
                lp.n = n;
                lp.push_cost = p.push_cost;
                lp.count_mask = nullptr;
                lp.light_lo = br.light_lo;
                lp.light_hi = br.light_hi;
                lp.chunk_lo = br.chunk_lo;
                lp.chunk_hi = br.chunk_hi;
                lp.gid = p.gid;
                lp.seg_pfx = p.gid ? p.seg_pfx : nullptr;
                lp.batch_base = batch * per;
                if (lev == job.levels)
                    level_body<W, true>(lp, sh);
                else
                    level_body<W, false>(lp, sh);
                break;
            }
            case PH_BFS_SCATTER: {
                // results, then clear what the batch touched
                const uint32_t first = batch * per;
                const uint32_t cnt = job.n - first < per ? job.n - first : per;
                for (size_t l = gtid(); l < cnt; l += gstride()) {
                    const uint32_t s = job_source(p, first + (uint32_t)l);
                    if (job.split) {
                        job.out[s] = p.counts[l] + p.counts2[l];
                        p.dm[s] = p.counts[l];
                    } else {
                        job.out[s] = p.counts[l];
                    }
                    if (job.clean) p.dirty[s] = 0;
                }
                for (uint32_t j = 0; j <= job.levels; ++j) {
                    const uint32_t c = p.bqcnt[j];
                    const uint32_t *q = p.bq + (size_t)j * n;
                    for (size_t i = gtid(); i < (size_t)c * W; i += gstride())
                        p.vis[(size_t)q[i / W] * W + (i % W)] = 0;
                }
                for (uint32_t j = job.levels - 1; j <= job.levels; ++j) {
                    const uint32_t c = p.bqcnt[j];
                    const uint32_t *q = p.bq + (size_t)j * n;
                    uint64_t *buf = frt_buf(p, j % 3);
                    uint32_t *fz = p.fnz + (size_t)(j % 3) * p.fnz_words;
                    for (size_t i = gtid(); i < (size_t)c * W; i += gstride())
                        buf[(size_t)q[i / W] * W + (i % W)] = 0;
                    for (size_t i = gtid(); i < c; i += gstride()) fz[q[i] >> 5] = 0;
                }
                break;
            }
            default:
                break;
        }
        if (!grid_sync(p.sync, &s_gen, &s_ok)) return;
        if (p.profile && gtid() == 0) {
            const uint64_t t = wall_clock64();
            ctl->phase_ticks[phase] += t - t_prev;
            ctl->phase_count[phase] += 1;
            t_prev = t;
        }

        // ------------------------------------------------------ next phase
        switch (phase) {
            case PH_INIT: phase = PH_COMPACT; break;
            case PH_COMPACT:
                // bounded: the initial (h-1)-degrees come from the same BFS
                phase = start_job(ctl->nsrc, h, p.d, bounded ? (int)PH_LB_ALL : (int)PH_KEYMIN, false, bounded);
                break;
            case PH_LB_ALL: phase = ctl->left ? PH_KEYMIN : PH_DONE; break;
            case PH_KEYMIN: phase = PH_LEVEL; break;
            case PH_LEVEL: phase = bounded ? PH_COLLECT : PH_SELECT; break;
            case PH_COLLECT: {
                const uint32_t rn = ctl->rn;
                phase = rn ? start_job(rn, h, p.d, PH_CLEAN, true, lazy) : (int)PH_SELECT;
                break;
            }
            case PH_CLEAN: phase = PH_KEYMIN; break;
            case PH_SELECT:
                aff_l = 1;
                phase = PH_AFF;
                break;
            case PH_AFF:
                if (aff_l < h) ++aff_l;
                else phase = PH_KILL;
                break;
            case PH_KILL:
                if (lazy)
                    phase = PH_LBD;
                else if (bounded)
                    phase = start_job(e_hm2 - np, h - 1, p.dm, PH_LBD, false, false);
                else
                    phase = start_job(e_h - np, h, p.d, PH_UNMARK, false, false);
                break;
            case PH_LBD:
            case PH_UNMARK:
                phase = (ctl->left && !(p.round_limit && ctl->round >= p.round_limit)) ? PH_KEYMIN : PH_DONE;
                break;
            case PH_BFS_RESET: phase = PH_BFS_SEED; break;
            case PH_BFS_SEED:
                lev = 1;
                phase = PH_BFS_LEVEL;
                break;
            case PH_BFS_LEVEL:
                if (lev < job.levels) ++lev;
                else phase = PH_BFS_SCATTER;
                break;
            case PH_BFS_SCATTER:
                if ((batch + 1) * per < job.n) {
                    ++batch;
                    phase = PH_BFS_RESET;
                } else {
                    phase = job.ret;
                    if (phase == PH_KEYMIN && !ctl->left) phase = PH_DONE;
                }
                break;
            default: phase = PH_DONE; break;
        }
        if (phase == PH_DONE) return;
    }
}

__global__ void sync_reset_kernel(uint32_t *words, uint32_t nwords) {
    for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) words[i] = 0;
}

template <int W>
int persistent_grid(khc_ctx *ctx) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, peel_persistent_kernel<W>, kBlockThreads, 0) !=
            hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        return -1;
    }
    const int want = (ctx->waves_per_cu + 3) / 4;
    return ctx->num_cu * (want < per_cu ? want : per_cu);
}

template <int W>
void launch_persistent(const PParams &p, int grid, hipStream_t st) {
    hipLaunchKernelGGL(peel_persistent_kernel<W>, dim3(grid), dim3(kBlockThreads), 0, st, p);
}

}  // namespace

// Runs the whole decomposition in one persistent kernel (captured in a
// hipGraph and replayed for identical arguments).
int persistent_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core,
                         uint32_t *peel_round, khc_stats *stats) {
    if (h > (uint32_t)kMaxPersistH)
        return set_error(ctx, KHC_EINVAL, "the persistent driver supports h <= 32");
    const auto t0 = std::chrono::steady_clock::now();
    const uint32_t n = g->n;
    const int W = ctx->persist_width;
    const bool bounded = (ctx->schedule == 1 || ctx->schedule == 3) && h >= 2;
    const uint32_t levels_max = h;
    const uint32_t nq = levels_max + 1;
    const size_t words = (size_t)n * W;
    const uint32_t fnz_words = (n + 31) / 32;
    const size_t hq_len = (size_t)n + g->nnz / 256 + 1;
    const size_t ahq_len = (size_t)n + g->nnz / kAffChunk + 1;
    void *vis, *f0, *f1, *f2, *fnz, *hacc, *hdone, *counts, *bq, *bhq, *bctr, *alive, *dirty, *d, *dm, *lb, *lbx,
        *mark, *queue, *list, *kg, *ming, *ahq, *ctl, *sync, *seg;
    int rc;
    if ((rc = ws_get(ctx, WS_VIS, words * 8, &vis)) || (rc = ws_get(ctx, WS_FRT0, words * 8, &f0)) ||
        (rc = ws_get(ctx, WS_FRT1, words * 8, &f1)) || (rc = ws_get(ctx, WS_FRT2, words * 8, &f2)) ||
        (rc = ws_get(ctx, WS_FNZ, (size_t)fnz_words * 3 * 4, &fnz)) ||
        (rc = ws_get(ctx, WS_HACC, ((size_t)g->n_heavy + 1) * W * 8, &hacc)) ||
        (rc = ws_get(ctx, WS_HDONE, ((size_t)g->n_heavy + 1) * 4, &hdone)) ||
        (rc = ws_get(ctx, WS_COUNTS, (size_t)2 * 64 * kMaxWidth * 4, &counts)) ||
        (rc = ws_get(ctx, WS_BQUEUE, (size_t)nq * n * 4 + 4, &bq)) ||
        (rc = ws_get(ctx, WS_HQUEUE, (size_t)nq * hq_len * 8, &bhq)) ||
        (rc = ws_get(ctx, WS_MISC, (size_t)nq * 32 + 64, &bctr)) ||
        (rc = ws_get(ctx, WS_ALIVE, (size_t)n + 8, &alive)) ||
        (rc = ws_get(ctx, WS_DIRTY, (size_t)n + 8, &dirty)) ||
        (rc = ws_get(ctx, WS_DEG, (size_t)n * 4 + 8, &d)) ||
        (rc = ws_get(ctx, WS_DHM1, (size_t)n * 4 + 8, &dm)) ||
        (rc = ws_get(ctx, WS_LB, (size_t)n * 4 + 8, &lb)) ||
        (rc = ws_get(ctx, WS_LBX, (size_t)n * 4 + 8, &lbx)) ||
        (rc = ws_get(ctx, WS_MARK, (size_t)n * 4 + 8, &mark)) ||
        (rc = ws_get(ctx, WS_QUEUE0, (size_t)n * 4 + 8, &queue)) ||
        (rc = ws_get(ctx, WS_QUEUE1, (size_t)n * 4 + 8, &list)) ||
        (rc = ws_get(ctx, WS_GRAPHK, (size_t)g->ngraphs * 8 + 8, &kg)) ||
        (rc = ws_get(ctx, WS_AHQ, (size_t)(h + 1) * ahq_len * 8, &ahq)) ||
        (rc = ws_get(ctx, WS_CTL, sizeof(PCtl), &ctl)) ||
        (rc = ws_get(ctx, WS_SYNC, (size_t)(32 + 32 * kXcds) * 4, &sync)) ||
        (rc = ws_get(ctx, WS_SEG, (size_t)g->ngraphs * 8 + 64 + 32 + (size_t)g->ngraphs * (h + 1) * 4, &seg)))
        return rc;
    ming = (uint32_t *)kg + g->ngraphs;
    PParams p;
    std::memset(&p, 0, sizeof(p));
    p.row_ptr = g->row_ptr;
    p.col = g->col;
    p.nnz = g->nnz;
    p.n = n;
    p.n_light = g->n_light_nz;
    p.push_cost = (uint32_t)ctx->push_cost;  // rows without arcs (a suffix) never gain a bit
    p.n_chunks = g->n_chunks;
    p.light_rows = g->light_rows;
    p.heavy_rows = g->heavy_rows;
    p.chunk_heavy = g->chunk_heavy;
    p.chunk_first = g->chunk_first;
    p.gid = g->gid;
    p.ngraphs = g->ngraphs;
    p.h = h;
    p.bounded = bounded ? (ctx->schedule == 3 ? 2 : 1) : 0;
    p.profile = ctx->profile ? 1 : 0;
    p.round_limit = ctx->round_limit;
    p.progress = ctx->persist_progress_dev;
    ctx->persist_progress[0] = ctx->persist_progress[1] = 0;
    p.alive = (uint8_t *)alive;
    p.dirty = (uint8_t *)dirty;
    p.d = (uint32_t *)d;
    p.dm = (uint32_t *)dm;
    p.lb = (uint32_t *)lb;
    p.lbx = (uint32_t *)lbx;
    p.mark = (uint32_t *)mark;
    p.queue = (uint32_t *)queue;
    p.list = (uint32_t *)list;
    p.core = core;
    p.round = peel_round;
    p.K = (uint32_t *)kg;
    p.MIN = (uint32_t *)ming;
    p.ahq = (uint64_t *)ahq;
    p.ahq_len = ahq_len;
    p.ctl = (PCtl *)ctl;
    p.vis = (uint64_t *)vis;
    p.frt0 = (uint64_t *)f0;
    p.frt1 = (uint64_t *)f1;
    p.frt2 = (uint64_t *)f2;
    p.fnz = (uint32_t *)fnz;
    p.fnz_words = fnz_words;
    p.hacc = (uint64_t *)hacc;
    p.hdone = (uint32_t *)hdone;
    p.counts = (uint32_t *)counts;
    p.counts2 = p.counts + 64 * kMaxWidth;
    p.bq = (uint32_t *)bq;
    p.bhq = (uint64_t *)bhq;
    p.hq_len = hq_len;
    p.bqdeg = (unsigned long long *)bctr;
    p.bwork = (uint32_t *)(p.bqdeg + 2 * nq);
    p.bqcnt = p.bwork + nq;
    p.bhcnt = p.bqcnt + nq;
    p.brange = (BatchRange *)seg;
    p.seg_cnt = (uint32_t *)((char *)seg + 32);
    p.seg_pfx = p.seg_cnt + g->ngraphs;
    p.gring = p.seg_pfx + g->ngraphs + 1;
    p.vbase = g->vtx_base;
    p.light_first = g->light_first;
    p.gchunk_first = g->graph_chunk_first;
    uint32_t *sp = (uint32_t *)sync;
    p.sync.count = sp;
    p.sync.gen = sp + 16;
    p.sync.abort = sp + 8;
    p.sync.groups = sp + 32;
    int grid = -1;
    switch (W) {
        case 8: grid = persistent_grid<8>(ctx); break;
        case 16: grid = persistent_grid<16>(ctx); break;
        default: grid = persistent_grid<32>(ctx); break;
    }
    if (grid < 1) return set_error(ctx, KHC_EHIP, "occupancy query for the persistent kernel failed");
    p.sync.nblocks = (uint32_t)grid;
    p.sync.ngroups = (uint32_t)grid < kXcds ? (uint32_t)grid : kXcds;
    const uint32_t sync_words = 32 + 32 * p.sync.ngroups;
    p.sync.timeout_ticks = (uint64_t)ctx->wall_clock_khz * 1000ull * (uint64_t)ctx->barrier_timeout_s;
    p.sync.grouped = ctx->xcd_grouped ? 1u : 0u;
    hipStream_t st = ctx->stream;

    // one graph per argument set, replayed on later calls
    khc_ctx::PersistGraph key{g,           h,         W,       grid, p.bounded, p.profile, p.round_limit,
                              core,        peel_round, p.sync.timeout_ticks, (int)p.sync.grouped, p.push_cost,
                              nullptr};
    hipGraphExec_t exec = nullptr;
    for (auto &e : ctx->persist_graphs)
        if (e.same_args(key)) exec = e.exec;
    if (!exec) {
        // captured on the context's private stream, launched on its work stream
        hipStream_t cs = ctx->capture_stream;
        if (!cs) return set_error(ctx, KHC_EHIP, "no capture stream");
        hipGraph_t graph;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return check_hip(ctx, e, "graph capture begin");
        hipLaunchKernelGGL(sync_reset_kernel, dim3(1), dim3(256), 0, cs, sp, sync_words);
        switch (W) {
            case 8: launch_persistent<8>(p, grid, cs); break;
            case 16: launch_persistent<16>(p, grid, cs); break;
            default: launch_persistent<32>(p, grid, cs); break;
        }
        e = hipStreamEndCapture(cs, &graph);
        if (e != hipSuccess) return check_hip(ctx, e, "graph capture end");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return check_hip(ctx, e, "graph instantiate");
        key.exec = exec;
        ctx->persist_graphs.push_back(key);
    }
    hipError_t e = hipGraphLaunch(exec, st);
    if (e != hipSuccess) return check_hip(ctx, e, "graph launch");
    if (ctx->progress_fn) {
        // report what the kernel publishes while it runs
        auto last = std::chrono::steady_clock::now();
        while ((e = hipStreamQuery(st)) == hipErrorNotReady) {
            std::this_thread::sleep_for(std::chrono::milliseconds(5));
            report_progress(ctx, &last, (uint32_t)ctx->persist_progress[0], ctx->persist_progress[1], 0u);
        }
        if (e != hipSuccess) return check_hip(ctx, e, "persistent decomposition");
    }
    PCtl host_ctl;
    uint32_t host_sync[3];
    e = hipMemcpyAsync(&host_ctl, ctl, sizeof(PCtl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(host_sync, sp + 8, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "persistent decomposition");
    if (host_sync[0] == ABORT_PLACEMENT && ctx->xcd_grouped) {
        // workgroups are not on XCD blockIdx % 8: rerun with the flat barrier
        ctx->xcd_grouped = 0;
        drop_persist_graphs(ctx, nullptr);
        return persistent_decompose(ctx, g, h, core, peel_round, stats);
    }
    if (host_sync[0]) {
        if (host_ctl.abort_reason == 1) return set_error(ctx, KHC_ELIMIT, "a round removed no vertex");
        return set_error(ctx, KHC_EHIP, "persistent decomposition aborted: a grid barrier wait exceeded " +
                                            std::to_string(ctx->barrier_timeout_s) + " s");
    }
    if (ctx->profile) {
        const double ms_per_tick = 1.0 / (double)ctx->wall_clock_khz;
        for (int i = 0; i < KHC_PERSIST_PHASES; ++i) {
            ctx->persist_phase_ms[i] += (double)host_ctl.phase_ticks[i] * ms_per_tick;
            ctx->persist_phase_count[i] += host_ctl.phase_count[i];
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->rounds = host_ctl.round;
        stats->h_recomputes = host_ctl.stat_hrec;
        stats->hm1_recomputes = host_ctl.stat_hm1;
        stats->bfs_batches = host_ctl.stat_batches;
        stats->affected_total = host_ctl.stat_aff;
        stats->width_words = (uint32_t)W;
        stats->wall_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return KHC_OK;
}

}  // namespace khc

extern "C" int khc_persist_profile_read(khc_ctx *ctx, double *ms, uint64_t *count, int reset) {
    if (!ctx) return KHC_EINVAL;
    for (int i = 0; i < KHC_PERSIST_PHASES; ++i) {
        if (ms) ms[i] = ctx->persist_phase_ms[i];
        if (count) count[i] = ctx->persist_phase_count[i];
        if (reset) {
            ctx->persist_phase_ms[i] = 0.0;
            ctx->persist_phase_count[i] = 0;
        }
    }
    return KHC_OK;
}

namespace khc {

void drop_persist_graphs(khc_ctx *ctx, const khc_graph *only) {
    auto &v = ctx->persist_graphs;
    for (size_t i = 0; i < v.size();) {
        if (!only || v[i].g == only) {
            (void)hipGraphExecDestroy(v[i].exec);
            v.erase(v.begin() + i);
        } else {
            ++i;
        }
    }
}

}  // namespace khc

using namespace khc;

extern "C" int khcore_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core,
                                uint32_t *peel_round, khc_stats *stats) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !core) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h == 0) return set_error(ctx, KHC_EINVAL, "h must be >= 1");
    (void)hipSetDevice(ctx->device);
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(*stats));
        return KHC_OK;
    }
    if (ctx->driver == 1 || g->ngraphs > 1) return persistent_decompose(ctx, g, h, core, peel_round, stats);
    return host_decompose(ctx, g, h, core, peel_round, stats);
}
