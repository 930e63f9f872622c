/*
 * khcore.h -- C ABI of the MI355X (gfx950) h-degree / (k,h)-core library.
 *
 * The library computes h-hop degrees and distance-generalised core numbers
 * of a simple undirected unweighted graph G = (V, E) (Section II of
 * "Scaling Up Distance-generalized Core Decomposition", arXiv 2006.03372):
 *
 *   N_v^h(G(S)) = { u in S, u != v : dis_{G(S)}(u, v) <= h }   (S = live set)
 *   d_v^h(G(S)) = |N_v^h(G(S))|                                 (h-degree)
 *   core_h(v)   = largest k such that a (k,h)-core contains v   (Definition 2)
 *
 * Distances are hop counts inside the subgraph induced by the live
 * vertices: dead vertices are neither counted nor used as relays.
 *
 * Conventions for every entry point
 *   - Graph arrays, masks and outputs are DEVICE pointers (hipMalloc'd or
 *     torch CUDA tensors); the caller owns them.  A graph handle keeps the
 *     caller's CSR pointers (not copies): they must stay valid and
 *     unchanged until khc_graph_destroy.
 *   - Work runs on the stream given to khc_create (NULL: the null stream).
 *   - Every call returns 0 on success or a negative KHC_E* code; the text
 *     of the last error of a context is available from khc_last_error.
 *     Nothing throws across this interface.
 *   - One context per host thread; calls on one context must not overlap.
 */
#ifndef KHCORE_H
#define KHCORE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KHC_OK 0
#define KHC_EINVAL (-1) /* null pointer, h == 0, size mismatch, bad option */
#define KHC_EGRAPH (-2) /* CSR is not a simple undirected graph            */
#define KHC_ENOMEM (-3) /* device allocation failed or workspace cap hit   */
#define KHC_EHIP (-4)   /* HIP runtime error (sticky for the context)      */
#define KHC_ELIMIT (-5) /* round limit exceeded (internal consistency)     */

typedef struct khc_ctx khc_ctx;
typedef struct khc_graph khc_graph;

/* Simple undirected graph in CSR form, device pointers.
 *   n        number of vertices, n < 2^32 - 1
 *   nnz      number of arcs = 2 |E| (row_ptr[n] must equal nnz)
 *   row_ptr  uint64[n+1], row_ptr[0] == 0, non-decreasing
 *   col      uint32[nnz], each row strictly increasing, no self-loops, and
 *            arc u->v present iff arc v->u is present (Section II: an
 *            undirected unweighted graph). */
typedef struct {
    uint32_t n;
    uint64_t nnz;
    const uint64_t *row_ptr;
    const uint32_t *col;
} khc_csr;

/* Counters of one decomposition (host struct, filled on request). */
typedef struct {
    uint64_t rounds;          /* peeling rounds                                 */
    uint64_t h_recomputes;    /* h-degrees recomputed by bounded BFS            */
    uint64_t hm1_recomputes;  /* (h-1)-degrees recomputed (bounded schedule)    */
    uint64_t bfs_batches;     /* multi-source BFS batches launched              */
    uint64_t affected_total;  /* sum over rounds of the affected-set size       */
    uint32_t max_level;       /* largest core number                            */
    uint32_t width_words;     /* source-lane words per vertex of the last batch */
    double wall_ms;           /* host wall time of the call                     */
    uint64_t local_rounds;    /* rounds that updated h-degrees locally (schedule 2) */
    uint64_t local_sources;   /* BFS sources of those local updates             */
    uint64_t gate_deferrals;  /* recomputes the learned gate deferred           */
} khc_stats;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` that enqueues all work on
 * `hip_stream` (a hipStream_t; NULL = null stream). */
int khc_create(khc_ctx **out, int device, void *hip_stream);
int khc_destroy(khc_ctx *ctx);
/* Message for the last failing call on ctx (static storage of the ctx). */
const char *khc_last_error(const khc_ctx *ctx);

/* Options (khc_set_option).  Values are validated; unknown ids: KHC_EINVAL. */
#define KHC_OPT_MAX_WIDTH 1       /* max uint64 words per vertex per BFS batch (1..32, pow2; default 32) */
#define KHC_OPT_SCHEDULE 2        /* 0 = plain recompute of the affected set, 1 = bounded,
                                     2 = local update inside N^h[P] when it is the cheaper of the two,
                                     3 = bounded with the (h-1)-degree bounds lowered by the
                                     decrement bound instead of recomputed, and refreshed with every
                                     h-degree recompute (default) (the persistent driver treats
                                     2 as 0)                                                          */
#define KHC_OPT_WORKSPACE_LIMIT 3 /* cap on workspace bytes (0 = none)                                  */
#define KHC_OPT_VALIDATE 4        /* 1 = validate the CSR in khc_graph_create (default 1)               */
#define KHC_OPT_WAVES_PER_CU 5    /* wavefronts per CU for the BFS level kernels (4..32; default 16)     */
#define KHC_OPT_PROFILE 6         /* 1 = time every BFS kernel launch with HIP events (default 0)       */
#define KHC_OPT_DRIVER 7          /* single-graph decomposition driver: 0 = host loop over rounds
                                     (default), 1 = one persistent kernel captured in a hipGraph;
                                     batched graphs always use the persistent kernel                  */
#define KHC_OPT_PERSIST_WIDTH 8   /* uint64 words per vertex per BFS batch in the persistent driver
                                     (8, 16 or 32; default 32)                                        */
#define KHC_OPT_BARRIER_TIMEOUT 9 /* seconds a grid-barrier wait may take before the persistent kernel
                                     aborts with KHC_EHIP (default 20)                                */
#define KHC_OPT_ROUND_LIMIT 10    /* stop a decomposition after this many peeling rounds (0 = none,
                                     default): vertices not removed by then keep core 0; used by
                                     the autotuner's trial runs                                      */
#define KHC_OPT_PUSH_COST 11     /* push/pull choice of a BFS level: 0 = push while the frontier's total
                                     degree times a width-dependent factor is below the arc count;
                                     c in 1..4096 = push while (frontier arcs x non-zero source words)
                                     times c is below (arcs x width + 4 x rows), the pull's gathers */
#define KHC_OPT_TUNE_REPEATS 12  /* autotuner trials per candidate, the median kept (1..15; default 3)    */
#define KHC_OPT_TUNE_CACHE 13    /* 1 = khc_autotune reuses the choice made on this context for a graph of
                                     the same size class (default); 0 = always time, and forget the
                                     cached choices                                                   */
int khc_set_option(khc_ctx *ctx, int option, int64_t value);

/* Kernel timing collected while KHC_OPT_PROFILE is 1, per kernel class:
 * 0 batch clear, 1 first BFS level, 2 inner BFS levels, 3 last BFS level
 * (the counting level).  bytes[c] sums the algorithmic bytes of the pull
 * levels of that class whose live set is the whole graph:
 * n*(8 + 8W) + nnz*(4 + 8W) per launch (row offset + own words per row,
 * column id + gathered frontier words per arc); 0 where not known. */
typedef struct {
    uint64_t launches[4];
    double ms[4];
    double bytes[4];
} khc_profile;

/* Waits for the recorded launches, adds them into *out and, if reset != 0,
 * forgets them.  Timing is taken on the context stream with HIP events. */
int khc_profile_read(khc_ctx *ctx, khc_profile *out, int reset);

/* Progress of long decompositions: the host-driven peeling and the
 * approximate mode call fn(user, rounds done, vertices removed, current
 * level) on the calling thread, at most once every interval_ms
 * milliseconds.  fn == NULL turns reporting off.  The persistent driver
 * runs as one launch: it publishes its round count and removed vertices to
 * host memory as it goes and the waiting host thread reports them (level
 * 0: the levels are per graph). */
typedef void (*khc_progress_fn)(void *user, uint32_t rounds, uint64_t removed, uint32_t level);
int khc_set_progress(khc_ctx *ctx, khc_progress_fn fn, void *user, uint32_t interval_ms);

/* Phases of the persistent driver (khc_persist_profile_read order). */
#define KHC_PERSIST_PHASES 17
/* init, compact, lb_all, keymin, level, collect, clean, select, affected,
 * kill, lbd, unmark, bfs_reset, bfs_seed, bfs_level, bfs_scatter, done.
 * With KHC_OPT_PROFILE on, every persistent run adds, per phase, the
 * wall-clock milliseconds from the previous grid barrier to the end of the
 * phase's own barrier (as workgroup 0 sees it) and how often it ran.
 * ms (host double[KHC_PERSIST_PHASES]) and count (host
 * uint64_t[KHC_PERSIST_PHASES]) may be NULL; reset != 0 clears the sums. */
int khc_persist_profile_read(khc_ctx *ctx, double *ms, uint64_t *count, int reset);

/* ---- graph store ------------------------------------------------------ */

/* Wrap a device CSR (Section II's G) and build the row schedule used by
 * the BFS kernels (rows bucketed by degree).  With validation on, a graph
 * that is not simple and undirected gives KHC_EGRAPH.  Synchronous. */
int khc_graph_create(khc_ctx *ctx, const khc_csr *g, khc_graph **out);
int khc_graph_destroy(khc_graph *g);

/* Several independent graphs packed together (batched decomposition).
 * Graph g owns vertices [vtx_base[g], vtx_base[g+1]) of the concatenated
 * arrays; its rows keep graph-LOCAL column ids.
 *   G         number of graphs, >= 1
 *   vtx_base  device uint64[G+1]: vtx_base[0] = 0, non-decreasing,
 *             vtx_base[G] = total vertices (< 2^32 - 1)
 *   row_ptr   device uint64[total + 1]: offsets into col (absolute)
 *   col       device uint32[nnz]: graph-local ids 0..n_g-1, each graph a
 *             simple undirected graph (validated as a whole when validation
 *             is on; an id outside its own graph gives KHC_EGRAPH)
 * The handle holds its own union column array (global ids) and a graph id
 * per vertex; the caller's row_ptr must stay valid until khc_graph_destroy,
 * col may be released after the call.  khcore_decompose on such a handle
 * gives every vertex the core number it has in its own graph (core numbers
 * of a disjoint union are per component) and, as removal round, the round
 * of its own graph's peeling: all graphs advance one round per step of one
 * persistent kernel.  Synchronous. */
int khc_graph_create_batched(khc_ctx *ctx, uint32_t G, const uint64_t *vtx_base, const uint64_t *row_ptr,
                             const uint32_t *col, uint64_t nnz, khc_graph **out);

/* Validate a CSR without keeping it: 0 or KHC_EGRAPH (message says why). */
int khc_validate_csr(khc_ctx *ctx, const khc_csr *g);

/* ---- h-degrees -------------------------------------------------------- */

/* d_v^h(G(S)) for every vertex, S = { v : alive[v] != 0 } (alive == NULL:
 * S = V).  Section II definition of the h-hop degree; the per-vertex
 * computations are independent (Section IV-D runs them in parallel).
 *   alive  device uint8[n] or NULL
 *   h      >= 1
 *   deg    device uint32[n] output; dead vertices get 0
 * Returns once the kernels are enqueued, after one small readback (the
 * number of live vertices that need a BFS); deg is complete when the
 * context stream has drained. */
int khdeg_compute(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                  uint32_t *deg);

/* h-degrees of the listed vertices only: deg[i] = d^h of verts[i] (0 for
 * a dead vertex).
 *   verts  device uint32[count], each < n (else KHC_EINVAL before any
 *          kernel reads them); a vertex may be listed more than once
 *   alive  as above
 * Returns after a small readback (the id check); deg is complete when the
 * context stream has drained. */
int khdeg_compute_list(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                       const uint32_t *verts, uint32_t count, uint32_t *deg);

/* khdeg_compute for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, results and errors, but every scratch buffer comes from
 * one static 64 MiB device array of the library (held on each GPU the
 * library runs on until the process ends), so no hipMalloc, hipFree or
 * allocating routine is called.  The batch width is the widest power of
 * two up to KHC_OPT_MAX_WIDTH whose buffers fit; a graph whose buffers do
 * not fit even at width 1 (about 85 n + nnz / 8 bytes at h = 3) gives
 * KHC_ENOMEM.  All calls on one GPU share the array: calls that overlap on
 * one device (other contexts or threads) race and must not be made.
 * Kernel timing (KHC_OPT_PROFILE) is not recorded.  Returns after one small
 * readback; deg is complete when the context stream has drained. */
int khdeg_compute_noalloc(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                          uint32_t *deg);

/* Work measure for traversed-edges-per-second figures: te[v] = the number
 * of arcs a scalar bounded BFS from v examines, i.e. the live degree summed
 * over every live vertex within h-1 hops of v (v included).  Dead vertices
 * get 0.  The paper reports run times only; this count is the work unit
 * its BFS-based h-degree computation performs per vertex.
 *   te     device uint64[n] output.  Returns after one small readback;
 *          te is complete when the context stream has drained. */
int khdeg_scanned_arcs(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                       uint64_t *te);

/* ---- (k,h)-core decomposition ----------------------------------------- */

/* core_h(v) for every vertex (problem statement, Section II), by
 * level-synchronous peeling: each round removes every live vertex whose
 * h-degree is at most the level k = max(k, min live h-degree), gives it
 * core k, and recomputes the h-degree of the live vertices within h hops
 * of the removed ones (Algorithms 1-2, Observations 1-2).  The bounded
 * schedules (KHC_OPT_SCHEDULE 1, and 3, the default) recompute such a vertex only when
 * its lower bounds reach the level.  The bounds are structural ((h-1)-degrees
 * of it and its neighbours, after h-LB of Section III) and a decrement bound
 * (a vertex at distance j from the removed set loses at most the vertices
 * within h - j hops of that set).  Schedule 1 recomputes the (h-1)-degrees
 * near each removed set; schedule 3 lowers them by the same decrement bound
 * and refreshes them with every h-degree recompute.  All schedules give
 * identical results.
 *   h           1..1024 (1..32 with the persistent driver and for graphs
 *               made by khc_graph_create_batched); otherwise KHC_EINVAL
 *   core        device uint32[n] output (isolated vertices: 0)
 *   peel_round  device uint32[n] output or NULL: round of removal
 *   stats       host struct or NULL
 * Synchronous (reads a few scalars per round). */
int khcore_decompose(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t *core,
                     uint32_t *peel_round, khc_stats *stats);

/* Batched (k,h)-core decomposition: khc_graph_create_batched, then
 * khcore_decompose, then khc_graph_destroy (the "batched persistent" mode:
 * all graphs run in one persistent kernel captured in a hipGraph).
 *   core   device uint32[total vertices] output, vertex order of the input
 *   peel_round, stats  as in khcore_decompose
 * Synchronous. */
int khcore_decompose_batched(khc_ctx *ctx, uint32_t G, const uint64_t *vtx_base, const uint64_t *row_ptr,
                             const uint32_t *col, uint64_t nnz, uint32_t h, uint32_t *core,
                             uint32_t *peel_round, khc_stats *stats);

/* ---- sampling-based approximate mode ----------------------------------- */

/* The paper's sampling-based decomposition (Section IV-C, Algorithms 5-6)
 * in level-synchronous form, on a vertex sample S drawn by the caller.
 * Each vertex keeps its exact initial h-degree d0, the number sel0 of
 * sampled vertices within h hops at the start, and the number sel of
 * sampled vertices within h hops in the current graph; its estimated
 * h-degree is floor(sel * d0 / sel0), i.e. sel divided by the initial rate
 * sel0 / d0 (d0 when sel0 = 0).  Peeling runs on the estimate as
 * khcore_decompose runs on the h-degree.  After each round only vertices
 * that can lose a sampled vertex recount sel: a vertex at distance j from
 * the removed set P can only lose vertices within h - j hops of P, so with
 * r0 the distance from P of the nearest sampled vertex the live vertices
 * within h - r0 hops of P recount, and none when no sampled vertex lies
 * within h - 1 hops.  The estimate never grows under removal, so the
 * result does not depend on the removal order.
 *   sampled   device uint8[n]: nonzero marks a sampled vertex
 *   h         1..1024
 *   core      device uint32[n] output: the approximate core numbers
 *   estimate  device uint32[n] or NULL: each vertex's estimate when removed
 *   stats     host or NULL (h_recomputes counts the ball recounts)
 * Synchronous (reads a few scalars per round). */
int khcore_decompose_sampled(khc_ctx *ctx, const khc_graph *g, uint32_t h, const uint8_t *sampled,
                             uint32_t *core, uint32_t *estimate, khc_stats *stats);

/* ---- autotuner --------------------------------------------------------- */

/* Picks the BFS source-block width (uint64 words per vertex, 64 sources
 * each) and the wavefronts per CU for decompositions of g at h by timing
 * trials of each candidate: the decomposition cut after `rounds` peeling
 * rounds (KHC_OPT_ROUND_LIMIT), run on the driver khcore_decompose would use
 * for g, KHC_OPT_TUNE_REPEATS times, the median kept.  Candidates: widths 8,
 * 16, 32 and 4, 8, 16 wavefronts per CU.  The fastest candidate is set on
 * ctx (KHC_OPT_MAX_WIDTH or KHC_OPT_PERSIST_WIDTH, and
 * KHC_OPT_WAVES_PER_CU) and remembered for the graph's size class (driver,
 * h, rounds, and the powers of two at or above the vertex and arc counts);
 * a later call for the same class applies it without trials
 * (KHC_OPT_TUNE_CACHE).  Every median is reported in *out (host, or NULL).
 * Synchronous; allocates a trial output buffer when it times. */
#define KHC_TUNE_MAX 16
typedef struct {
    uint32_t width_words;              /* chosen width                              */
    uint32_t waves_per_cu;             /* chosen wavefronts per CU                  */
    uint32_t persistent;               /* 1: tuned for the persistent driver        */
    uint32_t candidates;               /* trials run                                */
    uint32_t cand_width[KHC_TUNE_MAX];
    uint32_t cand_waves[KHC_TUNE_MAX];
    double trial_ms[KHC_TUNE_MAX];     /* median wall time of each candidate's trials */
    uint32_t repeats;                  /* trials per candidate                      */
    uint32_t cached;                   /* 1: applied from the cache, no trials      */
} khc_tune;
int khc_autotune(khc_ctx *ctx, const khc_graph *g, uint32_t h, uint32_t rounds, khc_tune *out);

/* ---- learned approximate mode ----------------------------------------- */

/* A small MLP that estimates log-scaled h-degrees from eight cheap features
 * (the paper estimates updated h-degrees by sampling instead, Section
 * IV-C): 8 inputs -> 64 -> 64 (ReLU) -> 1, BF16 weights and activations in
 * MFMA with FP32 accumulation, FP32 biases and FP32 master weights trained
 * with Adam.  Parameter vector (4801 floats, this order): W1[64][8], b1[64],
 * W2[64][64], b2[64], W3[64], b3; layer l computes W_l x + b_l. */
typedef struct khc_mlp khc_mlp;

/* He-uniform weights from `seed`, zero biases. */
int khc_mlp_create(khc_ctx *ctx, uint64_t seed, khc_mlp **out);
int khc_mlp_destroy(khc_mlp *m);
/* Host float[4801] in/out (also resets the Adam state on set). */
int khc_mlp_set_params(khc_ctx *ctx, khc_mlp *m, const float *host_params);
int khc_mlp_get_params(khc_ctx *ctx, const khc_mlp *m, float *host_params, float *host_grad);
/* Adam state (Kingma and Ba, Algorithm 1): first and second moment
 * estimates m, v (host float[4801] each, either may be NULL) and the number
 * of Adam updates made since the parameters were last set (*host_step, may
 * be NULL).  Update t computes, per parameter, m = 0.9 m + 0.1 g,
 * v = 0.999 v + 0.001 g^2 and p -= lr (m / (1 - 0.9^t)) / (sqrt(v / (1 - 0.999^t))
 * + 1e-8) in float32.  Synchronous. */
int khc_mlp_get_moments(khc_ctx *ctx, const khc_mlp *m, float *host_m, float *host_v, uint64_t *host_step);
/* Parameters to / from a file: the 8 bytes "KHCMLP01", uint32 4801, then
 * the 4801 float32 parameters in the order above (little endian).  Loading
 * resets the Adam state; a file of another shape gives KHC_EINVAL.
 * Synchronous. */
int khc_mlp_save(khc_ctx *ctx, const khc_mlp *m, const char *path);
int khc_mlp_load(khc_ctx *ctx, khc_mlp *m, const char *path);
/* y[i] = network(X[i][0..8)), X device float[n][8], y device float[n].
 * Asynchronous. */
int khc_mlp_forward(khc_ctx *ctx, const khc_mlp *m, const float *X, uint32_t n, float *y);
/* Gradient of sum_i (y_i - target_i)^2 / n over all n rows into the
 * network's gradient (read it with khc_mlp_get_params); *host_loss gets the
 * mean squared error.  Synchronous. */
int khc_mlp_gradient(khc_ctx *ctx, khc_mlp *m, const float *X, const float *target, uint32_t n,
                     float *host_loss);
/* Adam training on (X, target) device arrays: `epochs` passes in a seeded
 * random order, minibatches of `batch` rows, learning rate lr.
 * host_epoch_loss (host float[epochs] or NULL) gets each epoch's mean
 * minibatch loss.  Gradients are summed in a fixed order, so the same
 * seeds, data and device give the same parameters bit for bit.
 * Synchronous. */
int khc_mlp_train(khc_ctx *ctx, khc_mlp *m, const float *X, const float *target, uint32_t n, uint32_t epochs,
                  uint32_t batch, float lr, uint64_t seed, float *host_epoch_loss);

/* Features of every vertex of G(alive) for the network: X device
 * float[n][8], each log1p(count) / 8 of exact counts with a = max(1, h-3),
 * b = max(1, h-2): d^a(v), d^b(v), d^{h-1}(v); min, mean, max over live
 * neighbours of d^{h-1}; mean over live neighbours of d^a and of d^b.
 * lb, ub (device uint32[n] or NULL): exact bounds on d^h(v) from d^{h-1}:
 * max(d^{h-1}(v), max_w d^{h-1}(w)) and min(live - 1, sum_w d^{h-1}(w)).
 * Dead vertices get zeros.  2 <= h <= 64.  Asynchronous. */
int khc_features(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, float *X,
                 uint32_t *lb, uint32_t *ub);

/* Approximate (k,h)-core numbers: the level-synchronous peeling of
 * khcore_decompose, with each affected vertex's h-degree replaced by the
 * network's estimate clamped to [lb, ub] and never raised; exact
 * (h-1)-hop degrees and features are maintained.  mlp == NULL uses lb as
 * the estimate.  estimate (device uint32[n] or NULL) gets each vertex's
 * estimate when it was removed.  2 <= h <= 64.  Synchronous. */
int khcore_decompose_approx(khc_ctx *ctx, const khc_graph *g, uint32_t h, const khc_mlp *mlp,
                            uint32_t *core, uint32_t *estimate, khc_stats *stats);

/* Features of the learned recompute gate for every vertex of G(alive):
 * X device float[n][8], each log1p(count) / 8 of: the live degree of v,
 * dm(v), min, mean and max over live neighbours w of dm(w), the mean full
 * degree of the live neighbours, min(live - 1, sum over live w of dm(w)),
 * live - 1.  dm (device uint32[n]) holds (h-1)-degrees or lower bounds on
 * them (khdeg_compute at h - 1 gives the exact ones); the network is
 * trained to predict log1p(d^h(v)) / 8 from them.  Dead vertices get
 * zeros.  2 <= h <= 1024.  Asynchronous. */
int khc_gate_features(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, const uint32_t *dm,
                      float *X);

/* Training samples for the network from one peeling state G(alive): the
 * features of every live vertex (kind 0: khc_features, for
 * khcore_decompose_approx; kind 1: khc_gate_features from exact
 * (h-1)-degrees, for khcore_decompose_gated) and the target
 * log1p(d^h(v)) / 8 with d^h the exact h-degree, compacted to the live
 * vertices in vertex order.
 *   X       device float[n][8] output; rows [0, *count) are written
 *   target  device float[n] output; entries [0, *count)
 *   count   host uint32 output: the number of live vertices
 * 2 <= h <= 64.  Synchronous (reads back the count). */
int khc_mlp_samples(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, int kind, float *X,
                    float *target, uint32_t *count);

/* Peeling state after round r0 of an exact decomposition: alive[v] = 1 iff
 * round[v] >= r0, with round the peel_round output of khcore_decompose
 * (device uint32[n]); alive is device uint8[n].  Asynchronous. */
int khc_alive_after(khc_ctx *ctx, uint32_t n, const uint32_t *round, uint32_t r0, uint8_t *alive);

/* Gated (k,h)-core decomposition: the bounded schedule of khcore_decompose
 * (host-driven rounds, Algorithms 1-2 in level-synchronous form) with a
 * learned gate in front of its recomputes (schedule 3 when KHC_OPT_SCHEDULE
 * is 3, else 1).  A dirty vertex whose exact
 * lower bound lb reached the level k (its stale h-degree d still above k)
 * is first estimated: e = clamp(expm1(8 y), lb, d) with y the network's
 * output on khc_gate_features; if lb + floor((e - lb) * (1 - margin)) > k
 * that value becomes its key and the recompute is deferred until the level
 * reaches it or a later removal affects the vertex.  Vertices still leave
 * only with an exact or stale h-degree <= k, so every returned core number
 * is at least the exact one.  mlp == NULL or margin == 1 defers nothing and
 * gives the exact core numbers and removal rounds of khcore_decompose.
 *   margin      0..1
 *   core        device uint32[n] output
 *   peel_round  device uint32[n] or NULL
 *   stats       host or NULL (gate_deferrals counts the deferrals)
 * 2 <= h <= 1024, one graph.  Synchronous. */
int khcore_decompose_gated(khc_ctx *ctx, const khc_graph *g, uint32_t h, const khc_mlp *mlp, float margin,
                           uint32_t *core, uint32_t *peel_round, khc_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* KHCORE_H */
