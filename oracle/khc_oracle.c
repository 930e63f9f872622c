/*
 * CPU oracle for h-hop degrees and (k,h)-core numbers.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code,
 * header or constant with the GPU library and is never linked into it.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * it.
 *
 * Everything here is integer-only and written directly from the
 * definitions of Section II of the paper.  The peel is single-threaded;
 * the per-vertex loops of oracle_hdeg_list and oracle_certificate may
 * split their independent vertices over OpenMP threads (each vertex still
 * gets the same scalar BFS):
 *   - N_v^h(G(S)) = { u in S, u != v : dis_{G(S)}(u, v) <= h }, distances
 *     measured in the subgraph induced by the current vertex set S;
 *   - d_v^h(G(S)) = |N_v^h(G(S))|;
 *   - the (k,h)-core is the maximal subgraph in which every vertex has
 *     h-degree >= k inside it (Definition 2), and core_h(v) is the largest
 *     such k over the cores containing v.
 *
 * The peeling routine follows the peeling idea of Algorithms 1 and 2 in
 * its level-synchronous form: every vertex whose h-degree is at most the
 * current level k is removed in the same round, the level is
 * k <- max(k, min degree), and only vertices within h hops of the removed
 * set (in the graph before removal) get their h-degree recomputed, from
 * scratch, by bounded BFS (Observations 1 and 2 of Section IV-A, taken for
 * a set of removed vertices).  Readings of the paper used here:
 *   - the level starts at 0, so vertices whose h-degree is 0 get core 0;
 *   - the line "k <- argmin d" of Algorithm 2 is read as the minimum value;
 *   - dead vertices are neither counted nor used as relays (induced
 *     subgraph semantics of Definition 2).
 *
 * Graph input: CSR with uint64 row offsets and uint32 column ids; rows are
 * expected to describe a simple undirected graph (both arc directions
 * present).  oracle_check_csr() verifies that.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
static int og_thread(void) { return omp_get_thread_num(); }
#else
static int og_thread(void) { return 0; }
#endif

typedef struct {
    uint32_t n;
    const uint64_t *row_ptr;
    const uint32_t *col;
} og_graph;

/* Bounded BFS scratch: epoch stamps avoid clearing the visited array. */
typedef struct {
    uint32_t *stamp;
    uint32_t *queue;
    uint32_t epoch;
} og_bfs;

static int og_bfs_init(og_bfs *b, uint32_t n) {
    b->stamp = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    b->queue = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    b->epoch = 0;
    return (b->stamp && b->queue) ? 0 : -1;
}

static void og_bfs_free(og_bfs *b) {
    free(b->stamp);
    free(b->queue);
}

static void og_next_epoch(og_bfs *b, uint32_t n) {
    b->epoch++;
    if (b->epoch == 0) { /* wrapped: reset stamps */
        memset(b->stamp, 0, (size_t)n * sizeof(uint32_t));
        b->epoch = 1;
    }
}

/*
 * Number of vertices u != v of the induced subgraph G({x : allowed(x)})
 * with hop distance <= h from v (Section II, h-hop neighbourhood).
 * allowed(x) is (mask == NULL || mask[x] != 0) when thr == NULL, and
 * thr[x] >= t otherwise (used by the certificate check).
 * If te != NULL it also accumulates the arcs this BFS scans: the alive
 * degree of every reached vertex at distance <= h-1.
 */
static uint32_t og_hdeg_one(const og_graph *g, const uint8_t *mask,
                            const uint32_t *thr, uint32_t t,
                            uint32_t h, uint32_t v, og_bfs *b, uint64_t *te) {
#define OG_ALLOWED(x) (thr ? (thr[(x)] >= t) : (mask == NULL || mask[(x)] != 0))
    og_next_epoch(b, g->n);
    uint32_t head = 0, tail = 0;
    b->queue[tail++] = v;
    b->stamp[v] = b->epoch;
    uint32_t level_end = tail;
    uint32_t depth = 0;
    while (head < tail && depth < h) {
        /* expand every vertex at distance `depth` */
        while (head < level_end) {
            uint32_t x = b->queue[head++];
            for (uint64_t e = g->row_ptr[x]; e < g->row_ptr[x + 1]; e++) {
                uint32_t y = g->col[e];
                if (!OG_ALLOWED(y)) continue;
                if (te) (*te)++;
                if (b->stamp[y] == b->epoch) continue;
                b->stamp[y] = b->epoch;
                b->queue[tail++] = y;
            }
        }
        level_end = tail;
        depth++;
    }
    return tail - 1; /* the count excludes v itself */
#undef OG_ALLOWED
}

/* 0 if the CSR is a simple undirected graph, else a negative code:
 * -1 bad offsets, -2 column out of range, -3 self-loop, -4 row not strictly
 * increasing (unsorted or duplicate), -5 missing reverse arc. */
int oracle_check_csr(uint32_t n, const uint64_t *row_ptr, const uint32_t *col) {
    if (row_ptr[0] != 0) return -1;
    for (uint32_t v = 0; v < n; v++)
        if (row_ptr[v + 1] < row_ptr[v]) return -1;
    for (uint32_t v = 0; v < n; v++) {
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            uint32_t u = col[e];
            if (u >= n) return -2;
            if (u == v) return -3;
            if (e > row_ptr[v] && col[e - 1] >= u) return -4;
        }
    }
    for (uint32_t v = 0; v < n; v++) {
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            uint32_t u = col[e];
            /* binary search v in row u */
            uint64_t lo = row_ptr[u], hi = row_ptr[u + 1];
            int found = 0;
            while (lo < hi) {
                uint64_t mid = lo + (hi - lo) / 2;
                if (col[mid] == v) { found = 1; break; }
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (!found) return -5;
        }
    }
    return 0;
}

/*
 * h-degree of every vertex in the subgraph induced by the alive vertices
 * (alive == NULL: all).  Dead vertices get 0.  Returns 0, or -1 on
 * allocation failure.
 */
int oracle_hdeg(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                const uint8_t *alive, uint32_t h, uint32_t *deg) {
    og_graph g = {n, row_ptr, col};
    og_bfs b;
    if (og_bfs_init(&b, n)) return -1;
    for (uint32_t v = 0; v < n; v++)
        deg[v] = (alive && !alive[v]) ? 0 : og_hdeg_one(&g, alive, NULL, 0, h, v, &b, NULL);
    og_bfs_free(&b);
    return 0;
}

/* One BFS scratch per thread for the loops over independent vertices. */
static og_bfs *og_bfs_pool(uint32_t n, int threads) {
    og_bfs *pool = (og_bfs *)calloc((size_t)threads, sizeof(og_bfs));
    if (!pool) return NULL;
    for (int t = 0; t < threads; t++) {
        if (og_bfs_init(&pool[t], n)) {
            for (int u = 0; u <= t; u++) og_bfs_free(&pool[u]);
            free(pool);
            return NULL;
        }
    }
    return pool;
}

static void og_bfs_pool_free(og_bfs *pool, int threads) {
    for (int t = 0; t < threads; t++) og_bfs_free(&pool[t]);
    free(pool);
}

/*
 * h-degree of the listed vertices only (deg_out[i] for verts[i]), plus the
 * number of arcs each of those bounded BFS runs scans (te_out, optional).
 * A listed dead vertex gets 0.  The vertices are independent: with
 * threads > 1 they are split over that many OpenMP threads, each running
 * the same scalar BFS on its own scratch.
 */
int oracle_hdeg_list(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                     const uint8_t *alive, uint32_t h, const uint32_t *verts,
                     uint64_t count, uint32_t *deg_out, uint64_t *te_out, int threads) {
    og_graph g = {n, row_ptr, col};
    if (threads < 1) threads = 1;
    og_bfs *pool = og_bfs_pool(n, threads);
    if (!pool) return -1;
    #pragma omp parallel for num_threads(threads) schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)count; i++) {
        og_bfs *b = &pool[og_thread()];
        uint32_t v = verts[i];
        uint64_t te = 0;
        if (alive && !alive[v]) {
            deg_out[i] = 0;
        } else {
            deg_out[i] = og_hdeg_one(&g, alive, NULL, 0, h, v, b, te_out ? &te : NULL);
        }
        if (te_out) te_out[i] = te;
    }
    og_bfs_pool_free(pool, threads);
    return 0;
}

/*
 * Level-synchronous peeling with from-scratch recomputation (plain
 * schedule).  Outputs core[v] and round[v] (the round in which v was
 * removed).  Per-round trace, if the arrays are given (capacity
 * trace_cap rounds): trace_k[r] = level k, trace_p[r] = |P_r| (vertices
 * removed), trace_a[r] = |A_r| (vertices recomputed).  *rounds_out gets the
 * number of rounds.  Returns 0, -1 on allocation failure, -2 if the trace
 * capacity is too small (results are still complete).
 */
int oracle_peel(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                uint32_t h, uint32_t *core, uint32_t *round,
                uint32_t *trace_k, uint32_t *trace_p, uint32_t *trace_a,
                uint64_t trace_cap, uint64_t *rounds_out) {
    og_graph g = {n, row_ptr, col};
    og_bfs b, ab;
    uint8_t *alive = (uint8_t *)malloc(n ? n : 1);
    uint32_t *d = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *P = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *A = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *dist = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    int rc = 0;
    if (!alive || !d || !P || !A || !dist || og_bfs_init(&b, n) || og_bfs_init(&ab, n)) {
        free(alive); free(d); free(P); free(A); free(dist);
        return -1;
    }
    memset(alive, 1, n);
    /* initial h-degrees (Algorithm 1, lines 2-3) */
    for (uint32_t v = 0; v < n; v++) d[v] = og_hdeg_one(&g, alive, NULL, 0, h, v, &b, NULL);

    uint64_t left = n, r = 0;
    uint32_t k = 0;
    while (left > 0) {
        /* level: k <- max(k, min over alive of d) */
        uint32_t m = UINT32_MAX;
        for (uint32_t v = 0; v < n; v++)
            if (alive[v] && d[v] < m) m = d[v];
        if (m > k) k = m;
        /* P = alive vertices with d <= k; they all get core k */
        uint32_t np = 0;
        for (uint32_t v = 0; v < n; v++) {
            if (alive[v] && d[v] <= k) {
                P[np++] = v;
                core[v] = k;
                round[v] = (uint32_t)r;
            }
        }
        /* A = alive vertices within h hops of P in the graph before removal,
         * excluding P: one multi-source BFS of depth h. */
        og_next_epoch(&ab, n);
        uint32_t head = 0, tail = 0;
        for (uint32_t i = 0; i < np; i++) {
            ab.stamp[P[i]] = ab.epoch;
            ab.queue[tail++] = P[i];
            dist[P[i]] = 0;
        }
        while (head < tail) {
            uint32_t x = ab.queue[head++];
            if (dist[x] >= h) continue;
            for (uint64_t e = row_ptr[x]; e < row_ptr[x + 1]; e++) {
                uint32_t y = col[e];
                if (!alive[y] || ab.stamp[y] == ab.epoch) continue;
                ab.stamp[y] = ab.epoch;
                dist[y] = dist[x] + 1;
                ab.queue[tail++] = y;
            }
        }
        uint32_t na = 0;
        for (uint32_t i = np; i < tail; i++) A[na++] = ab.queue[i];
        /* remove P */
        for (uint32_t i = 0; i < np; i++) alive[P[i]] = 0;
        left -= np;
        /* recompute the h-degree of every affected vertex from scratch */
        for (uint32_t i = 0; i < na; i++)
            d[A[i]] = og_hdeg_one(&g, alive, NULL, 0, h, A[i], &b, NULL);
        if (r < trace_cap) {
            if (trace_k) trace_k[r] = k;
            if (trace_p) trace_p[r] = np;
            if (trace_a) trace_a[r] = na;
        } else if (trace_k || trace_p || trace_a) {
            rc = -2;
        }
        r++;
    }
    if (rounds_out) *rounds_out = r;
    og_bfs_free(&b); og_bfs_free(&ab);
    free(alive); free(d); free(P); free(A); free(dist);
    return rc;
}

/*
 * Peeling-order certificate for claimed core numbers c and removal rounds
 * rho.  With C_k = {u : c(u) >= k} and R_j = {u : rho(u) >= j}:
 *   (i)   d^h_v(G(C_{c(v)})) >= c(v)     (each C_k is a (k,h)-feasible set)
 *   (ii)  d^h_v(G(R_{rho(v)})) <= c(v)   (v was removable when it was removed)
 *   (iii) rho(u) <= rho(v)  =>  c(u) <= c(v).
 * Together they imply c = core_h (by the monotonicity of h-degrees under
 * vertex removal and the uniqueness of the (k,h)-core, Section II); the
 * output of any correct level-synchronous peel satisfies them.
 * (i) and (ii) are checked for the listed vertices (verts == NULL: all),
 * (iii) for all vertices.  fail_out[0..2] receive the number of violations
 * of each condition.  Returns 0 or -1 on allocation failure.
 */
int oracle_certificate(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                       uint32_t h, const uint32_t *c, const uint32_t *rho,
                       const uint32_t *verts, uint64_t count, uint64_t *fail_out, int threads) {
    og_graph g = {n, row_ptr, col};
    if (threads < 1) threads = 1;
    og_bfs *pool = og_bfs_pool(n, threads);
    if (!pool) return -1;
    uint64_t f0 = 0, f1 = 0;
    int64_t total = verts ? (int64_t)count : (int64_t)n;
    /* (i) and (ii) per vertex, independent of each other */
    #pragma omp parallel for num_threads(threads) schedule(dynamic, 4) reduction(+ : f0, f1)
    for (int64_t i = 0; i < total; i++) {
        og_bfs *b = &pool[og_thread()];
        uint32_t v = verts ? verts[i] : (uint32_t)i;
        if (c[v] > 0 && og_hdeg_one(&g, NULL, c, c[v], h, v, b, NULL) < c[v]) f0++;
        if (og_hdeg_one(&g, NULL, rho, rho[v], h, v, b, NULL) > c[v]) f1++;
    }
    og_bfs_pool_free(pool, threads);
    fail_out[0] = f0;
    fail_out[1] = f1;
    fail_out[2] = 0;
    /* (iii): for every round value, the claimed cores must be a single
     * value, and non-decreasing in the round.  Bucket by round. */
    uint32_t maxr = 0;
    for (uint32_t v = 0; v < n; v++) if (rho[v] > maxr) maxr = rho[v];
    uint64_t nr = (uint64_t)maxr + 1;
    uint32_t *lo = (uint32_t *)malloc(nr * sizeof(uint32_t));
    uint32_t *hi = (uint32_t *)malloc(nr * sizeof(uint32_t));
    uint8_t *seen = (uint8_t *)calloc(nr, 1);
    if (!lo || !hi || !seen) { free(lo); free(hi); free(seen); return -1; }
    for (uint32_t v = 0; v < n; v++) {
        uint32_t r = rho[v];
        if (!seen[r]) { seen[r] = 1; lo[r] = hi[r] = c[v]; }
        else { if (c[v] < lo[r]) lo[r] = c[v]; if (c[v] > hi[r]) hi[r] = c[v]; }
    }
    int have = 0;
    uint32_t prev_hi = 0;
    for (uint64_t r = 0; r < nr; r++) {
        if (!seen[r]) continue;
        if (lo[r] != hi[r]) fail_out[2]++;
        if (have && lo[r] < prev_hi) fail_out[2]++;
        prev_hi = hi[r];
        have = 1;
    }
    free(lo); free(hi); free(seen);
    return 0;
}

/*
 * Sampling-based peeling (Section IV-C, the KHCoreSamp / UpdateHNbrSamp
 * pair) in level-synchronous form.  sampled[v] != 0 marks the vertex
 * sample S (drawn by the caller).  For every vertex:
 *   d0[v]   = exact initial h-degree,
 *   sel[v]  = |N_v^h(G(alive)) cap S|, the sampled vertices within h hops
 *             in the current graph (kept exact: the paper subtracts exactly
 *             the sampled vertices a removal cuts off),
 *   rate[v] = sel0[v] / d0[v], fixed at the start (sel0 = initial sel),
 *   est[v]  = sel[v] / rate[v], read here as floor(sel * d0 / sel0) in
 *             integer arithmetic (the paper's worked example truncates);
 *             a vertex with sel0 = 0 has no sampled vertex to scale by and
 *             keeps est = d0.
 * Peeling then runs on est exactly as oracle_peel runs on the exact
 * degree: k <- max(k, min est), P = {est <= k}, core[P] = k, and est is
 * recomputed for the live vertices within h hops of P in the graph before
 * removal (only their balls can lose sampled vertices).  est never grows
 * under removal, so the result does not depend on the removal order.
 * est_out (optional) gets each vertex's estimate when it was removed.
 * Returns 0 or -1 on allocation failure.
 */
static uint32_t og_sampled_in_ball(const og_graph *g, const uint8_t *alive, const uint8_t *sampled,
                                   uint32_t h, uint32_t v, og_bfs *b) {
    uint32_t reached = og_hdeg_one(g, alive, NULL, 0, h, v, b, NULL);
    uint32_t sel = 0;
    /* the BFS queue holds v and then every vertex it reached */
    for (uint32_t i = 1; i <= reached; i++) sel += sampled[b->queue[i]] ? 1u : 0u;
    return sel;
}

static uint32_t og_estimate(uint32_t sel, uint32_t sel0, uint32_t d0) {
    if (sel0 == 0) return d0;
    return (uint32_t)(((uint64_t)sel * d0) / sel0);
}

int oracle_peel_sampled(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                        uint32_t h, const uint8_t *sampled, uint32_t *core, uint32_t *est_out) {
    og_graph g = {n, row_ptr, col};
    og_bfs b, ab;
    uint8_t *alive = (uint8_t *)malloc(n ? n : 1);
    uint32_t *d0 = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *sel0 = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *est = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *P = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *dist = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!alive || !d0 || !sel0 || !est || !P || !dist || og_bfs_init(&b, n) || og_bfs_init(&ab, n)) {
        free(alive); free(d0); free(sel0); free(est); free(P); free(dist);
        return -1;
    }
    memset(alive, 1, n);
    for (uint32_t v = 0; v < n; v++) {
        d0[v] = og_hdeg_one(&g, alive, NULL, 0, h, v, &b, NULL);
        sel0[v] = og_sampled_in_ball(&g, alive, sampled, h, v, &b);
        est[v] = d0[v];
    }
    uint64_t left = n;
    uint32_t k = 0;
    while (left > 0) {
        uint32_t m = UINT32_MAX;
        for (uint32_t v = 0; v < n; v++)
            if (alive[v] && est[v] < m) m = est[v];
        if (m > k) k = m;
        uint32_t np = 0;
        for (uint32_t v = 0; v < n; v++) {
            if (alive[v] && est[v] <= k) {
                P[np++] = v;
                core[v] = k;
                if (est_out) est_out[v] = est[v];
            }
        }
        /* vertices within h hops of P before removal */
        og_next_epoch(&ab, n);
        uint32_t head = 0, tail = 0;
        for (uint32_t i = 0; i < np; i++) {
            ab.stamp[P[i]] = ab.epoch;
            ab.queue[tail++] = P[i];
            dist[P[i]] = 0;
        }
        while (head < tail) {
            uint32_t x = ab.queue[head++];
            if (dist[x] >= h) continue;
            for (uint64_t e = row_ptr[x]; e < row_ptr[x + 1]; e++) {
                uint32_t y = col[e];
                if (!alive[y] || ab.stamp[y] == ab.epoch) continue;
                ab.stamp[y] = ab.epoch;
                dist[y] = dist[x] + 1;
                ab.queue[tail++] = y;
            }
        }
        for (uint32_t i = 0; i < np; i++) alive[P[i]] = 0;
        left -= np;
        for (uint32_t i = np; i < tail; i++) {
            uint32_t u = ab.queue[i];
            est[u] = og_estimate(og_sampled_in_ball(&g, alive, sampled, h, u, &b), sel0[u], d0[u]);
        }
    }
    og_bfs_free(&b); og_bfs_free(&ab);
    free(alive); free(d0); free(sel0); free(est); free(P); free(dist);
    return 0;
}
