// Internal declarations shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <map>
#include <string>
#include <vector>

#include "khcore.h"

namespace khc {

// Rows with more arcs than this are split into chunks of kChunkArcs arcs
// that whole workgroups process; lighter rows go to one lane group each.
constexpr uint32_t kHeavyRowArcs = 512;
constexpr uint32_t kChunkArcs = 4096;
// Light rows with more arcs than this are scanned by lane groups in the
// affected-set search; the others by one lane each.
constexpr uint32_t kMidDeg = 16;
// A lower bound max(d^{h-1}(u), max over neighbours w of d^{h-1}(w)) reads
// at most this many neighbours of u: any subset of the neighbours still
// gives a lower bound, and hub rows stay cheap.
constexpr uint32_t kLbArcs = 512;
constexpr int kBlockThreads = 256;  // 4 wavefronts of 64 lanes
constexpr uint32_t kMaxRoundH = 1024;     // largest h of the host-driven peeling
constexpr size_t kHostScalarBytes = 16384;  // pinned per-round readback buffer
constexpr int kMaxWidth = 32;       // uint64 words per vertex per BFS batch

// Lane layout of one vertex row of W uint64 words inside a wavefront:
// each lane owns WPL consecutive words (one 16-byte load when WPL == 2) and
// LPR lanes cover a row, so a wavefront works on 64 / LPR rows at once.
template <int W>
struct RowLayout {
    static constexpr int WPL = (W >= 2) ? 2 : 1;
    static constexpr int LPR = W / WPL;
    static constexpr int RPW = 64 / LPR;
    static constexpr int GROUPS = kBlockThreads / LPR;  // lane groups per workgroup
};

// A device buffer that only grows.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Workspace;

}  // namespace khc

struct khc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    std::string err;
    int sticky = 0;
    // options
    int max_width = 32;
    int schedule = 3;
    uint64_t ws_limit = 0;
    int validate = 1;
    int waves_per_cu = 16;
    uint32_t round_limit = 0;  // 0: peel to the end
    int push_cost = 0;         // BFS push/pull rule (KHC_OPT_PUSH_COST)
    int tune_repeats = 3;      // autotuner trials per candidate
    int tune_cache_on = 1;     // autotuner reuses choices per size class
    std::map<uint64_t, std::pair<int, int>> tune_cache;  // size class -> (width, waves per CU)
    // workspace
    std::vector<khc::DevBuf> bufs;
    uint64_t ws_bytes = 0;
    // pinned host scalars for per-round readbacks
    uint32_t *host_scalars = nullptr;
    // kernel timing (KHC_OPT_PROFILE)
    int profile = 0;
    struct ProfRec {
        hipEvent_t a, b;
        int cls;
        double bytes;
    };
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    khc_profile prof_acc{};
    // persistent driver
    int driver = 0;             // 0 host-driven rounds, 1 one persistent kernel
    int persist_width = 32;     // source words per BFS batch in the persistent kernel
    int barrier_timeout_s = 20; // deadline of one grid-barrier wait
    int xcd_grouped = 1;        // 0 once a persistent run found a workgroup off XCD blockIdx % 8
    uint64_t wall_clock_khz = 100000;
    struct PersistGraph {
        const khc_graph *g;
        uint32_t h;
        int W, grid, bounded, profile;
        uint32_t round_limit;
        uint32_t *core, *round;
        uint64_t timeout_ticks;  // barrier deadline baked into the captured launch
        int grouped;             // XCD-grouped (1) or flat (0) barrier
        uint32_t push_cost;      // push/pull rule baked into the captured launch
        hipGraphExec_t exec;
        bool same_args(const PersistGraph &o) const {
            return g == o.g && h == o.h && W == o.W && grid == o.grid && bounded == o.bounded &&
                   profile == o.profile && round_limit == o.round_limit && core == o.core && round == o.round &&
                   timeout_ticks == o.timeout_ticks && grouped == o.grouped && push_cost == o.push_cost;
        }
    };
    std::vector<PersistGraph> persist_graphs;
    // [rounds done, vertices removed] of the running persistent kernel
    // (coherent pinned host memory the device writes; host and device views)
    volatile unsigned long long *persist_progress = nullptr;
    unsigned long long *persist_progress_dev = nullptr;
    // progress reports of the host-driven loops
    khc_progress_fn progress_fn = nullptr;
    void *progress_user = nullptr;
    uint32_t progress_ms = 1000;
    double persist_phase_ms[KHC_PERSIST_PHASES] = {};
    uint64_t persist_phase_count[KHC_PERSIST_PHASES] = {};
    hipStream_t capture_stream = nullptr;  // private stream the persistent launch is captured on
};

struct khc_graph {
    khc_ctx *ctx = nullptr;
    uint32_t n = 0;
    uint64_t nnz = 0;
    const uint64_t *row_ptr = nullptr;
    const uint32_t *col = nullptr;
    // row schedule (device)
    uint32_t *light_rows = nullptr;  // rows with <= kHeavyRowArcs arcs, by degree descending
    uint32_t n_light = 0;
    uint32_t n_light_mid = 0;  // light rows with more than kMidDeg arcs (a prefix)
    uint32_t n_light_nz = 0;   // light rows with at least one arc (a prefix)
    uint32_t *heavy_rows = nullptr;  // heavier rows, by degree descending
    uint32_t n_heavy = 0;
    uint32_t *chunk_heavy = nullptr;  // heavy-row index of each chunk
    uint32_t *chunk_first = nullptr;  // first chunk of each heavy row [n_heavy + 1]
    uint32_t n_chunks = 0;
    uint32_t max_degree = 0;
    // graphs packed together: light rows and chunks of graph g start at
    // light_first[g] and graph_chunk_first[g] (device, [ngraphs + 1])
    uint32_t *light_first = nullptr;
    uint32_t *graph_chunk_first = nullptr;
    // several graphs packed as one disjoint union: gid[v] = graph of v
    uint32_t ngraphs = 1;
    uint32_t *gid = nullptr;       // device, owned (null: one graph)
    uint32_t *col_owned = nullptr; // device, owned union column ids (batched graphs)
    uint64_t *vtx_base = nullptr;  // device, owned copy of the graph offsets [ngraphs + 1]
};

namespace khc {

int set_error(khc_ctx *ctx, int code, const std::string &msg);
// Kernel timing helpers: prof_begin returns a record index (or -1 when
// profiling is off); prof_end closes it.
int prof_begin(khc_ctx *ctx, int cls, double bytes);
void prof_end(khc_ctx *ctx, int rec);
int check_hip(khc_ctx *ctx, hipError_t e, const char *what);
// Workspace slot `slot` of at least `bytes` bytes (grown on demand).
int ws_get(khc_ctx *ctx, int slot, size_t bytes, void **out);

enum WsSlot {
    WS_VIS = 0,
    WS_FRT0,
    WS_FRT1,
    WS_FNZ,
    WS_HACC,
    WS_HDONE,
    WS_COUNTS,
    WS_SRCS,
    WS_MISC,
    WS_ALIVE,
    WS_DEG,
    WS_DHM1,
    WS_LB,
    WS_FLAGS,
    WS_QUEUE0,
    WS_QUEUE1,
    WS_MARK,
    WS_SCRATCH,
    WS_FRT2,
    WS_BQUEUE,
    WS_QPTRS,
    WS_TE,
    WS_HQUEUE,
    WS_DIRTY,
    WS_GRAPHK,
    WS_AHQ,
    WS_CTL,
    WS_SYNC,
    WS_APPROX_DJ,
    WS_APPROX_SCAL,
    WS_APPROX_X,
    WS_APPROX_Y,
    WS_MINPART,
    WS_ITEMS,
    WS_SEG,
    WS_LBX,
    WS_REGION,
    WS_ROWCNT,
    WS_GATE_LIST,
    WS_NUM_SLOTS
};

// A device region carved into buffers (256-byte aligned) instead of the
// context workspace: the entry point that allocates nothing.
struct Arena {
    char *base = nullptr;
    size_t bytes = 0, used = 0;
    void *take(size_t b) {
        const size_t at = (used + 255) & ~(size_t)255;
        if (at > bytes || b > bytes - at) return nullptr;
        used = at + b;
        return base + at;
    }
};

// Multi-source h-bounded BFS over up to 64*max_width sources per batch;
// writes deg_out[i] = d^h(srcs[i]) for i < nsrc (device list).  `alive` is
// a device uint8 mask or null.  With an arena, every buffer is carved from
// it (widths up to arena_width, no kernel timing) and nothing is allocated.
// Asynchronous.
int msbfs_degrees(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                  const uint32_t *srcs, uint32_t nsrc, uint32_t *deg_out, int scatter,
                  uint32_t *deg_full, Arena *arena = nullptr, int arena_width = 0);
// Like msbfs_degrees (scattered by source), but a source's count takes only
// the reached vertices v with count_mask[v] != 0.
int msbfs_masked_counts(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                        const uint32_t *srcs, uint32_t nsrc, const uint8_t *count_mask, uint32_t *deg_full);
// Row counts of the local h-degree update: after a BFS from sources listed
// by their distance from a removed set (lvl[j] of them at distance j, j =
// 0..h), acc[u] += the number of sources within h hops of u whose distance
// from the set is at most h - (mark[u] - 1), for every u in rows.
struct RowCount {
    const uint32_t *rows;
    uint32_t nrows;
    const uint32_t *mark;
    const uint32_t *lvl;
    uint32_t h;
    uint32_t *acc;
};
int msbfs_row_counts(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, const uint32_t *srcs,
                     uint32_t nsrc, const RowCount &rc);
// Bytes msbfs_degrees carves from an arena at width W (alignment included).
size_t msbfs_arena_bytes(const khc_graph *g, uint32_t h, int W);
// khdeg_compute after its argument checks; with an arena nothing is
// allocated (the source list and counter are carved from it as well).
int khdeg_compute_impl(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, uint32_t *deg,
                       Arena *arena, int arena_width);
// Address of this device's static scratch (set up by khc_create).
int noalloc_init(int device);

// te_full[s] = arcs a scalar bounded BFS from s examines (live degree summed
// over the vertices within h-1 hops of s, s included).  Asynchronous.
int msbfs_scanned_arcs(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                       const uint32_t *srcs, uint32_t nsrc, uint64_t *te_full);

// j-hop degrees of the sources for every j = 1..levels: level_out[j-1]
// (full-length device arrays, indexed by vertex).  Asynchronous.
int msbfs_all_levels(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t levels,
                     const uint32_t *srcs, uint32_t nsrc, uint32_t *const *level_out);
// Live sources (live vertices with a live neighbour) into the WS_SRCS
// workspace; returns their number in *count (synchronous).
int compact_sources(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t **srcs,
                    uint32_t *count);
void fill_u32(khc_ctx *ctx, uint32_t *p, uint32_t value, uint64_t count);

// Whole decomposition in one persistent kernel (khc_persist.hip).
int persistent_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core,
                         uint32_t *peel_round, khc_stats *stats);
// Learned recompute gate of the bounded schedule (khc_gate.hip).
struct GateArgs {
    const khc_mlp *mlp;  // null: no gate
    float margin;        // 0..1: soft key = lb + (estimate - lb) * (1 - margin)
};
int gate_pass(khc_ctx *ctx, const khc_graph *g, const khc_mlp *mlp, float margin, const uint8_t *alive,
              const uint32_t *dm, const uint32_t *list, uint32_t rn, uint32_t *lb, const uint32_t *d, uint8_t *dirty,
              const uint32_t *part, uint32_t *s, float *X, float *Y, uint32_t *out);
// Host-driven decomposition (khc_peel.hip); a non-null gate forces the
// bounded schedule and puts the learned gate in front of its recomputes.
int host_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core, uint32_t *peel_round,
                   khc_stats *stats, const GateArgs *gate = nullptr);
// Calls the progress callback when its interval has passed since *last.
void report_progress(khc_ctx *ctx, std::chrono::steady_clock::time_point *last, uint32_t rounds, uint64_t removed,
                     uint32_t level);
// Forget captured persistent launches (their arguments are stale).
void drop_persist_graphs(khc_ctx *ctx, const khc_graph *only);

}  // namespace khc
