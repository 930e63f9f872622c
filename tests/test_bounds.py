"""CPU pins of the bounds the bounded peeling schedule relies on, checked by
brute force with the oracle's h-degrees on small random graphs and random
removed sets P:

* structural lower bound: d^h(u) >= d^{h-1}(u) and d^h(u) >= d^{h-1}(w) for
  every live neighbour w (also over any subset of the neighbours);
* decrement bound: removing P, a live vertex u at distance j (1 <= j <= h)
  from P loses at most |{v : dist(P, v) <= h - j}| vertices of its h-ball
  (P counted); vertices farther than h keep their h-degree;
* the same at radius h - 1: a vertex at distance h - 1 from P loses at most
  |P| from its (h-1)-ball;
* the sampling mode's recount rule: a vertex at distance j from P loses
  only sampled vertices within h - j hops of P, so its sampled count is
  unchanged when there are none.
"""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_2006_03372_amd import synth


def _dist_from_set(g, alive, P):
    """BFS distances from the set P over live vertices (inf when unreached)."""
    INF = np.iinfo(np.int64).max
    dist = np.full(g.n, INF, dtype=np.int64)
    frontier = [int(p) for p in P]
    for p in frontier:
        dist[p] = 0
    d = 0
    while frontier:
        d += 1
        nxt = []
        for x in frontier:
            for y in g.col[g.row_ptr[x]:g.row_ptr[x + 1]]:
                y = int(y)
                if alive[y] and dist[y] == INF:
                    dist[y] = d
                    nxt.append(y)
        frontier = nxt
    return dist


def _graph(kind, n, seed):
    if kind == "er":
        return synth.erdos_renyi(n, 4.0 / max(n - 1, 1), seed)
    return synth.chung_lu(n, 4.0, 2.5, seed)


@settings(max_examples=60, deadline=None)
@given(kind=st.sampled_from(["er", "cl"]), n=st.integers(8, 60), h=st.integers(1, 4),
       seed=st.integers(0, 10_000), frac=st.floats(0.02, 0.3))
def test_decrement_bound(kind, n, h, seed, frac):
    g = _graph(kind, n, seed)
    rng = np.random.default_rng(seed + 1)
    alive = (rng.random(g.n) < 0.9).astype(np.uint8)
    live = np.flatnonzero(alive)
    if live.size == 0:
        return
    P = rng.choice(live, size=max(1, int(frac * live.size)), replace=False)
    after = alive.copy()
    after[P] = 0
    dist = _dist_from_set(g, alive.astype(bool), P)
    for r in (h, h - 1):
        if r < 1:
            continue
        before = oracle.hdeg(g, r, alive).astype(np.int64)
        now = oracle.hdeg(g, r, after).astype(np.int64)
        ring = np.array([int(np.sum(dist[alive.astype(bool)] <= t)) for t in range(r + 1)])
        for u in np.flatnonzero(after):
            j = dist[u]
            if j > r:
                assert now[u] == before[u], (u, r)
            else:
                assert before[u] - now[u] <= ring[r - j], (u, r, j)
                if j == r:  # the outermost ring loses P at most
                    assert before[u] - now[u] <= P.size, (u, r)


def _ball(g, alive, u, h):
    """Vertices other than u within h hops of u over live vertices."""
    seen = {int(u)}
    frontier = [int(u)]
    for _ in range(h):
        nxt = []
        for x in frontier:
            for y in g.col[g.row_ptr[x]:g.row_ptr[x + 1]]:
                y = int(y)
                if alive[y] and y not in seen:
                    seen.add(y)
                    nxt.append(y)
        frontier = nxt
    seen.discard(int(u))
    return seen


@settings(max_examples=40, deadline=None)
@given(kind=st.sampled_from(["er", "cl"]), n=st.integers(8, 50), h=st.integers(1, 4),
       seed=st.integers(0, 10_000), frac=st.floats(0.02, 0.3), rate=st.floats(0.05, 0.5))
def test_sampled_recount_rule(kind, n, h, seed, frac, rate):
    g = _graph(kind, n, seed)
    rng = np.random.default_rng(seed + 2)
    alive = (rng.random(g.n) < 0.9).astype(np.uint8)
    sampled = rng.random(g.n) < rate
    live = np.flatnonzero(alive)
    if live.size == 0:
        return
    P = rng.choice(live, size=max(1, int(frac * live.size)), replace=False)
    after = alive.copy()
    after[P] = 0
    dist = _dist_from_set(g, alive.astype(bool), P)
    for u in np.flatnonzero(after):
        j = int(min(dist[u], h + 1))
        lost = {x for x in _ball(g, alive, u, h) - _ball(g, after, u, h) if sampled[x]}
        # every lost sampled vertex lies within h - j hops of P
        assert all(dist[x] <= h - j for x in lost), (u, j, lost)
        if not np.any(sampled & (dist <= h - j) & alive.astype(bool)):
            assert not lost


@pytest.mark.parametrize("h", [2, 3, 4])
def test_structural_lower_bound(h):
    for seed in range(6):
        g = synth.chung_lu(300, 5.0, 2.5, seed)
        alive = synth.random_alive(g.n, 0.85, seed + 7)
        d = oracle.hdeg(g, h, alive).astype(np.int64)
        dm = oracle.hdeg(g, h - 1, alive).astype(np.int64)
        for u in np.flatnonzero(alive):
            nb = [w for w in g.col[g.row_ptr[u]:g.row_ptr[u + 1]] if alive[w]]
            assert d[u] >= dm[u]
            for w in nb[:3]:  # any subset of the neighbours gives a bound
                assert d[u] >= dm[w]
            if nb:
                assert d[u] >= max(dm[w] for w in nb)
