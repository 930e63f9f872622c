"""Literal Python oracle for h-degrees and (k,h)-core numbers.

TEST INFRASTRUCTURE ONLY: this module is the slow, obviously correct
reference used by the tests, the smoke check and the benchmark's CPU
baseline.  It shares no code with the GPU library.

Written from Section II (definitions) and Section III (Algorithm 1) of the
paper.  Graphs are given as (n, row_ptr, col) CSR arrays of a simple
undirected graph; vertex sets as boolean/uint8 masks.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def _rows(n, row_ptr, col):
    rp = [int(x) for x in row_ptr]
    cl = [int(x) for x in col]
    return [cl[rp[v]:rp[v + 1]] for v in range(n)]


def h_neighbourhood(adj, alive, h, v):
    """N_v^h(G(S)): vertices u != v in S with dis_{G(S)}(u, v) <= h.

    Distances are shortest-path hop counts inside the subgraph induced by
    S = {x : alive[x]} (Section II); dead vertices are never relays.
    """
    dist = {v: 0}
    q = deque([v])
    while q:
        x = q.popleft()
        if dist[x] == h:
            continue
        for y in adj[x]:
            if alive[y] and y not in dist:
                dist[y] = dist[x] + 1
                q.append(y)
    del dist[v]
    return set(dist)


def hdeg(n, row_ptr, col, alive, h):
    """d_v^h(G(S)) for every v in S; 0 for vertices outside S."""
    adj = _rows(n, row_ptr, col)
    alive = [True] * n if alive is None else [bool(a) for a in alive]
    return np.array([len(h_neighbourhood(adj, alive, h, v)) if alive[v] else 0
                     for v in range(n)], dtype=np.int64)


def brute_core(n, row_ptr, col, h):
    """core_h(v) straight from Definition 2, by enumerating every vertex set.

    core_h(v) = max over S containing v of min_{u in S} d_u^h(G(S)): every
    S whose minimum h-degree is k lies inside the (k,h)-core, and the
    (k,h)-core itself is such a set.  Exponential; n <= 12 only.
    """
    if n > 12:
        raise ValueError("brute force is limited to n <= 12")
    adj = _rows(n, row_ptr, col)
    best = [0] * n
    for mask in range(1, 1 << n):
        alive = [(mask >> i) & 1 == 1 for i in range(n)]
        members = [i for i in range(n) if alive[i]]
        k = min(len(h_neighbourhood(adj, alive, h, u)) for u in members)
        for u in members:
            if k > best[u]:
                best[u] = k
    return np.array(best, dtype=np.int64)


def alg1_peel(n, row_ptr, col, h):
    """The basic peeling algorithm (Algorithm 1), one vertex at a time.

    Buckets B[d] hold vertices by current h-degree; the level k runs upward
    from 0 (a vertex with h-degree 0 gets core 0); the vertex picked from
    B[k] is the smallest id (any choice gives the same result).  After a
    removal every u in N_v^h(G) has its h-degree recomputed in G(V minus v)
    and moves to bucket max(k, d).  Returns (core, removal order).
    """
    adj = _rows(n, row_ptr, col)
    alive = [True] * n
    d = [len(h_neighbourhood(adj, alive, h, v)) for v in range(n)]
    buckets = [set() for _ in range(n + 1)]
    for v in range(n):
        buckets[d[v]].add(v)
    core = [0] * n
    order = []
    for k in range(0, n + 1):
        while buckets[k]:
            v = min(buckets[k])
            buckets[k].remove(v)
            core[v] = k
            order.append(v)
            ball = h_neighbourhood(adj, alive, h, v)
            alive[v] = False
            for u in ball:
                nd = len(h_neighbourhood(adj, alive, h, u))
                buckets[d[u]].discard(u)
                d[u] = max(k, nd)
                buckets[d[u]].add(u)
    return np.array(core, dtype=np.int64), order


def bz_kcore(n, row_ptr, col):
    """Classical core numbers (h = 1) by the linear bin-sort peeling.

    Vertices are kept in an array sorted by current degree with bin start
    positions; removing the minimum-degree vertex decrements each remaining
    neighbour of larger degree and swaps it to the front of its bin.
    """
    adj = _rows(n, row_ptr, col)
    deg = [len(a) for a in adj]
    md = max(deg) if n else 0
    bin_count = [0] * (md + 1)
    for x in deg:
        bin_count[x] += 1
    start = [0] * (md + 1)
    s = 0
    for k in range(md + 1):
        start[k] = s
        s += bin_count[k]
    pos = [0] * n
    vert = [0] * n
    nxt = list(start)
    for v in range(n):
        pos[v] = nxt[deg[v]]
        vert[pos[v]] = v
        nxt[deg[v]] += 1
    for i in range(n):
        v = vert[i]
        for u in adj[v]:
            if deg[u] > deg[v]:
                du = deg[u]
                pu = pos[u]
                pw = start[du]
                w = vert[pw]
                if u != w:
                    vert[pu], vert[pw] = w, u
                    pos[u], pos[w] = pw, pu
                start[du] += 1
                deg[u] -= 1
    return np.array(deg, dtype=np.int64)


def level_sync_peel(n, row_ptr, col, h):
    """Level-synchronous peeling with from-scratch recomputation.

    Each round: k <- max(k, min alive d); P = alive vertices with d <= k all
    get core k; the vertices within h hops of P in the graph before removal
    (Observations 1-2, for a removed set) have their h-degree recomputed in
    the graph after removal.  Returns (core, round, trace) with
    trace = [(k, |P|, |A|) per round].
    """
    adj = _rows(n, row_ptr, col)
    alive = [True] * n
    d = [len(h_neighbourhood(adj, alive, h, v)) for v in range(n)]
    core = [0] * n
    rnd = [0] * n
    trace = []
    k, r, left = 0, 0, n
    while left:
        k = max(k, min(d[v] for v in range(n) if alive[v]))
        P = [v for v in range(n) if alive[v] and d[v] <= k]
        affected = set()
        for p in P:
            core[p], rnd[p] = k, r
            affected |= h_neighbourhood(adj, alive, h, p)
        affected -= set(P)
        for p in P:
            alive[p] = False
        for u in affected:
            d[u] = len(h_neighbourhood(adj, alive, h, u))
        trace.append((k, len(P), len(affected)))
        left -= len(P)
        r += 1
    return np.array(core, dtype=np.int64), np.array(rnd, dtype=np.int64), trace



def brute_core_sampled(n, row_ptr, col, h, sampled):
    """Core numbers of the sampling-based estimate (Section IV-C), straight
    from the core definition over every vertex set (small n only).

    With d0 and sel0 the exact h-degree and the number of sampled vertices
    within h hops in the whole graph, a vertex u of a set T has estimated
    degree est(u, T) = floor(sel(u, T) * d0(u) / sel0(u)), where sel(u, T)
    counts the sampled vertices within h hops of u in G(T) (est = d0 when
    sel0 = 0).  est only shrinks as T shrinks, so the estimated cores nest
    and core(v) = max over T containing v of min over u in T of est(u, T).
    """
    adj = _rows(n, row_ptr, col)
    full = [True] * n
    d0 = [len(h_neighbourhood(adj, full, h, v)) for v in range(n)]
    sel0 = [sum(1 for u in h_neighbourhood(adj, full, h, v) if sampled[u]) for v in range(n)]
    best = [0] * n
    for mask in range(1, 1 << n):
        alive = [(mask >> v) & 1 == 1 for v in range(n)]
        members = [v for v in range(n) if alive[v]]
        lo = None
        for u in members:
            sel = sum(1 for w in h_neighbourhood(adj, alive, h, u) if sampled[w])
            e = d0[u] if sel0[u] == 0 else (sel * d0[u]) // sel0[u]
            lo = e if lo is None or e < lo else lo
        for v in members:
            if lo > best[v]:
                best[v] = lo
    return np.array(best, dtype=np.uint32)


def bitmap_update(n, row_ptr, col, alive, h, v):
    """h-degree update after deleting one vertex v by reachability inside
    the ball of v (Section IV-A/B: Observations 1-2, Theorem 1, and the
    bitmap dynamic programme of Algorithms 3-4), written from the paper's
    description.

    Returns (labels, region_edges, bitmaps, new_degree):
      labels       the ball R = N_v^h(G(alive)) relabelled u_0, u_1, ...:
                   the vertices at distance < h from v first (these own a
                   bit), each group by increasing vertex id;
      region_edges the edges of G(R) as (i, j) label pairs, i < j;
      bitmaps      the reach bitmaps (int, bit j = u_j) after the
                   initialisation and after each of the h iterations; the
                   two buffers of the iteration are kept apart (the
                   programme reads one and writes the other, and both start
                   from the initial bitmaps);
      new_degree   {u: h-degree of u in G(alive minus v)} for u in R, from
                   d(u) - 1 - |{w in R : dist(v, w) <= h - dist(v, u),
                   w not reachable from u}|.
    """
    adj = _rows(n, row_ptr, col)
    al = [bool(x) for x in alive]
    dist = {v: 0}
    q = deque([v])
    while q:
        x = q.popleft()
        if dist[x] == h:
            continue
        for y in adj[x]:
            if al[y] and y not in dist:
                dist[y] = dist[x] + 1
                q.append(y)
    ball = [u for u in dist if u != v]
    inner = sorted(u for u in ball if dist[u] < h)
    outer = sorted(u for u in ball if dist[u] == h)
    labels = inner + outer
    idx = {u: i for i, u in enumerate(labels)}
    edges = sorted({(min(idx[a], idx[b]), max(idx[a], idx[b]))
                    for a in labels for b in adj[a] if b in idx})
    init = [(1 << i) if i < len(inner) else 0 for i in range(len(labels))]
    buf = [list(init), list(init)]
    history = [list(init)]
    p, qq = 1, 0
    for _ in range(h):
        qq, p = p, 1 - p
        for i, j in edges:
            buf[qq][i] |= buf[p][j]
            buf[qq][j] |= buf[p][i]
        history.append(list(buf[qq]))
    final = buf[qq]
    old = hdeg(n, row_ptr, col, al, h)
    new = {}
    for u in labels:
        s = dist[u]
        lost = 1 + sum(1 for w in labels if dist[w] <= h - s and not (final[idx[u]] >> idx[w]) & 1)
        new[u] = int(old[u]) - lost
    return labels, edges, history, new


def set_local_update(n, row_ptr, col, alive, h, removed):
    """New h-degrees of the live vertices within h hops of a removed SET P,
    computed only inside the region N^h[P] (the set form of the update
    above, used by the library's local-update rounds).

    With t(w) = dist(P, w) before removal and s = t(u) for an affected u,
    every vertex u loses exactly the vertices w with t(w) <= h - s that it
    reaches within h hops before removal but not after; every shortest path
    of length <= h between such u and w stays inside N^h[P] (before
    removal) or N^h[P] minus P (after), so both reach tests are made inside
    the region.  Returns {u: new h-degree}.
    """
    adj = _rows(n, row_ptr, col)
    al = [bool(x) for x in alive]
    P = set(int(x) for x in removed)
    t = {p: 0 for p in P}
    q = deque(P)
    while q:
        x = q.popleft()
        if t[x] == h:
            continue
        for y in adj[x]:
            if al[y] and y not in t:
                t[y] = t[x] + 1
                q.append(y)
    region_pre = [x in t for x in range(n)]
    region_post = [x in t and x not in P for x in range(n)]
    old = hdeg(n, row_ptr, col, al, h)
    new = {}
    for u, s in t.items():
        if u in P:
            continue
        pre = h_neighbourhood(adj, region_pre, h, u)
        post = h_neighbourhood(adj, region_post, h, u)
        lost = sum(1 for w in pre if t[w] <= h - s and w not in post)
        new[u] = int(old[u]) - lost
    return new
