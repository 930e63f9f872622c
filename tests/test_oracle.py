"""Pins for the CPU oracle: closed forms, brute force, textbook routines,
the paper's running example and invariants.  CPU only."""
import math
import os
from collections import deque

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from oracle import reference as R
from paper_2006_03372_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def py_hdeg(g, h, alive=None):
    return R.hdeg(g.n, g.row_ptr, g.col, alive, h)


# ----------------------------------------------------------- closed forms

@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_hdeg_closed_forms(oracle_lib, h):
    for n in (1, 2, 5, 9):
        assert (oracle.hdeg(synth.complete(n), h) == n - 1).all()
    for n in (3, 4, 7, 10, 13):
        assert (oracle.hdeg(synth.cycle(n), h) == min(2 * h, n - 1)).all()
    for n in (1, 2, 6, 11):
        i = np.arange(n)
        expect = np.minimum(i, h) + np.minimum(n - 1 - i, h)
        assert (oracle.hdeg(synth.path(n), h) == expect).all()
    for m in (1, 3, 8):
        d = oracle.hdeg(synth.star(m), h)
        assert d[0] == m
        assert (d[1:] == (1 if h == 1 else m)).all()
    for a, b in ((1, 1), (2, 3), (4, 5)):
        d = oracle.hdeg(synth.complete_bipartite(a, b), h)
        if h == 1:
            assert (d[:a] == b).all() and (d[a:] == a).all()
        else:
            assert (d == a + b - 1).all()
    p = oracle.hdeg(synth.petersen(), h)
    assert (p == (3 if h == 1 else 9)).all()
    for dim in (3, 5):
        q = oracle.hdeg(synth.hypercube(dim), h)
        assert (q == sum(math.comb(dim, i) for i in range(1, h + 1))).all()
    # interior of the infinite grid: 2h(h+1) vertices within L1 distance h
    t = oracle.hdeg(synth.torus(2 * h + 3, 2 * h + 5), h)
    assert (t == 2 * h * (h + 1)).all()


def test_hdeg_large_h_is_component_size(oracle_lib):
    g = synth.disjoint_union([synth.path(7), synth.cycle(5), synth.star(4)])
    d = oracle.hdeg(g, 50)
    assert (d[:7] == 6).all() and (d[7:12] == 4).all() and (d[12:] == 4).all()


@pytest.mark.parametrize("h", [1, 2, 3, 5])
def test_core_closed_forms(oracle_lib, h):
    for n in (2 * h + 1, 2 * h + 4, 17):
        c, _ = oracle.peel(synth.cycle(n), h)
        assert (c == 2 * h).all()
    for n in (3, 5, 2 * h):
        if n >= 3:
            c, _ = oracle.peel(synth.cycle(n), h)
            assert (c == min(2 * h, n - 1)).all()
    for n in (1, 4, 8):
        c, _ = oracle.peel(synth.complete(n), h)
        assert (c == n - 1).all()
    for n in (2, 5, 12):
        c, _ = oracle.peel(synth.path(n), h)
        assert (c == min(h, n - 1)).all()
    c, _ = oracle.peel(synth.star(6), h)
    assert (c == (1 if h == 1 else 6)).all()
    # isolated vertices have core 0
    c, _ = oracle.peel(synth.from_edges(5, [0], [1]), h)
    assert list(c) == [1, 1, 0, 0, 0]


# ----------------------------------------------------- running example

def _golden():
    lines = [ln.split() for ln in open(os.path.join(GOLDEN, "running_example.txt"))
             if ln.strip() and not ln.startswith("#")]
    edges = [tuple(int(x) - 1 for x in e.split("-")) for e in lines[0][1:]]
    e = np.array(edges)
    g = synth.from_edges(14, e[:, 0], e[:, 1])
    return g, lines[1:]


def _remove_mask(spec):
    alive = np.ones(14, dtype=np.uint8)
    for x in spec.split("=")[1].split(","):
        alive[int(x) - 1] = 0
    return alive


def test_running_example(oracle_lib):
    g, facts = _golden()
    assert oracle.check_csr(g) == 0
    seen = set()
    for f in facts:
        h = int(f[1].split("=")[1])
        if f[0] == "core":
            expect = np.array([int(x) for x in f[2:]])
            c, r = oracle.peel(g, h)
            assert (c == expect).all()
            c_py, _ = R.alg1_peel(g.n, g.row_ptr, g.col, h)
            assert (c_py == expect).all()
        elif f[0] == "mindeg":
            d = oracle.hdeg(g, h)
            v, k = int(f[2]) - 1, int(f[3])
            assert d[v] == k == d.min()
        elif f[0] == "ball":
            adj = R._rows(g.n, g.row_ptr, g.col)
            ball = R.h_neighbourhood(adj, [True] * 14, h, int(f[2]) - 1)
            assert ball == {int(x) - 1 for x in f[3:]}
        elif f[0] == "after_remove":
            alive = _remove_mask(f[2])
            d = oracle.hdeg(g, h, alive)
            for item in f[3:]:
                v, k = item.split(":")
                assert d[int(v) - 1] == int(k)
        elif f[0] == "ball_in":
            alive = _remove_mask(f[2])
            d = oracle.hdeg(g, h, alive)
            v = int(f[3]) - 1
            live = np.flatnonzero(alive)
            assert d[v] == d[live].min() == len(f[4:])
            adj = R._rows(g.n, g.row_ptr, g.col)
            ball = R.h_neighbourhood(adj, [bool(a) for a in alive], h, v)
            assert ball == {int(x) - 1 for x in f[4:]}
        seen.add(f[0])
    assert seen == {"core", "mindeg", "ball", "after_remove", "ball_in"}


# ------------------------------------------------ brute force / textbook

def _graph_strategy(max_n):
    @st.composite
    def graphs(draw):
        n = draw(st.integers(1, max_n))
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
        mask = draw(st.lists(st.booleans(), min_size=len(pairs), max_size=len(pairs)))
        e = [p for p, m in zip(pairs, mask) if m]
        u = [a for a, _ in e]
        v = [b for _, b in e]
        return synth.from_edges(n, u, v)
    return graphs()


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(g=_graph_strategy(8), h=st.integers(1, 4))
def test_brute_force_equals_peels(oracle_lib, g, h):
    brute = R.brute_core(g.n, g.row_ptr, g.col, h)
    alg1, _ = R.alg1_peel(g.n, g.row_ptr, g.col, h)
    lvl, rnd, _ = R.level_sync_peel(g.n, g.row_ptr, g.col, h)
    c, r = oracle.peel(g, h)
    assert (brute == alg1).all()
    assert (brute == lvl).all()
    assert (brute == c).all()
    assert (rnd == r).all()


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(g=_graph_strategy(14), h=st.integers(1, 4), seed=st.integers(0, 1000))
def test_c_hdeg_equals_python(oracle_lib, g, h, seed):
    alive = synth.random_alive(g.n, 0.7, seed)
    assert (oracle.hdeg(g, h, alive) == py_hdeg(g, h, alive)).all()
    assert (oracle.hdeg(g, h) == py_hdeg(g, h)).all()


def test_h1_equals_kcore(oracle_lib):
    import networkx as nx
    for seed in range(4):
        g = synth.chung_lu(600, 6.0, 2.5, seed)
        c, _ = oracle.peel(g, 1)
        bz = R.bz_kcore(g.n, g.row_ptr, g.col)
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from(zip(*synth.edge_list(g)))
        nxc = nx.core_number(G)
        assert (c == bz).all()
        assert all(c[v] == nxc[v] for v in range(g.n))


def _bfs_dist(adj, alive, src):
    dist = {src: 0}
    q = deque([src])
    while q:
        x = q.popleft()
        for y in adj[x]:
            if alive[y] and y not in dist:
                dist[y] = dist[x] + 1
                q.append(y)
    return dist


@pytest.mark.parametrize("h", [2, 3])
def test_observation2_identity(oracle_lib, h):
    """d_u^h(G) - d_u^h(G minus v) = 1 + |F_u| for every u in N_v^h(G)
    (Observation 2, Section IV-A), with F_u computed from BFS distances."""
    g = synth.erdos_renyi(40, 0.08, seed=3)
    adj = R._rows(g.n, g.row_ptr, g.col)
    full = [True] * g.n
    d0 = oracle.hdeg(g, h)
    for v in range(0, g.n, 3):
        alive = np.ones(g.n, dtype=np.uint8)
        alive[v] = 0
        d1 = oracle.hdeg(g, h, alive)
        dv = _bfs_dist(adj, full, v)
        for u, s in dv.items():
            if u == v or s > h:
                continue
            du = _bfs_dist(adj, [bool(a) for a in alive], u)
            F = [w for w, t in dv.items() if w != v and t <= h - s and du.get(w, h + 1) > h]
            assert d0[u] - d1[u] == 1 + len(F)


def test_invariants(oracle_lib):
    g = synth.chung_lu(400, 6.0, 2.5, 11)
    prev = None
    for h in (1, 2, 3, 4):
        d = oracle.hdeg(g, h)
        assert int(d.sum()) % 2 == 0
        c, r = oracle.peel(g, h)
        assert (c <= d).all()
        if prev is not None:
            assert (prev <= c).all()
        prev = c


def test_disjoint_union_componentwise(oracle_lib):
    parts = [synth.chung_lu(n, 5.0, 2.5, s) for n, s in ((120, 1), (80, 2), (200, 3))]
    u = synth.disjoint_union(parts)
    for h in (2, 3):
        c, _ = oracle.peel(u, h)
        off = 0
        for p in parts:
            cp, _ = oracle.peel(p, h)
            assert (c[off:off + p.n] == cp).all()
            off += p.n


# ------------------------------------------------------------- certificate

def test_certificate_accepts_and_rejects(oracle_lib):
    rng = np.random.default_rng(0)
    for h in (1, 2, 3):
        g = synth.chung_lu(150, 5.0, 2.5, 21 + h)
        c, r = oracle.peel(g, h)
        assert oracle.certificate(g, h, c, r).sum() == 0
        for _ in range(15):
            v = int(rng.integers(g.n))
            for delta in (-1, 1):
                if int(c[v]) + delta < 0:
                    continue
                c2 = c.astype(np.int64)
                c2[v] += delta
                assert oracle.certificate(g, h, c2, r).sum() > 0
        # a wrong removal order is caught too
        v = int(np.argmax(c))
        r2 = r.copy()
        r2[v] = 0
        if c[v] != c[r == 0].max():
            assert oracle.certificate(g, h, c, r2).sum() > 0


def test_te_counts(oracle_lib):
    # K_n: h=1 scans the n-1 arcs of the source, h=2 every arc of the graph
    g = synth.complete(6)
    _, te = oracle.hdeg_list(g, 1, [0, 3])
    assert list(te) == [5, 5]
    _, te = oracle.hdeg_list(g, 2, [0])
    assert list(te) == [30]
    # long cycle: 2h-1 vertices within h-1 hops, 2 arcs each
    g = synth.cycle(50)
    for h in (1, 2, 3):
        d, te = oracle.hdeg_list(g, h, [7])
        assert d[0] == 2 * h and te[0] == 2 * (2 * h - 1)


# ----------------------------------------------------------- inputs / CSR

def test_csr_validation_codes(oracle_lib):
    good = synth.cycle(5)
    assert oracle.check_csr(good) == 0
    bad = synth.CSR(n=3, row_ptr=np.array([0, 1, 1, 1], np.uint64), col=np.array([1], np.uint32))
    assert oracle.check_csr(bad) == -5
    loop = synth.CSR(n=2, row_ptr=np.array([0, 1, 1], np.uint64), col=np.array([0], np.uint32))
    assert oracle.check_csr(loop) == -3
    rng_bad = synth.CSR(n=2, row_ptr=np.array([0, 1, 2], np.uint64), col=np.array([5, 0], np.uint32))
    assert oracle.check_csr(rng_bad) == -2
    dup = synth.CSR(n=2, row_ptr=np.array([0, 2, 4], np.uint64), col=np.array([1, 1, 0, 0], np.uint32))
    assert oracle.check_csr(dup) == -4


def test_generators_deterministic_and_simple(oracle_lib):
    a = synth.rmat(10, 8, seed=5)
    b = synth.rmat(10, 8, seed=5)
    assert (a.row_ptr == b.row_ptr).all() and (a.col == b.col).all()
    assert oracle.check_csr(a) == 0
    c1 = synth.chung_lu(500, 8.0, 2.5, 9)
    c2 = synth.chung_lu(500, 8.0, 2.5, 9)
    assert (c1.col == c2.col).all()
    assert oracle.check_csr(c1) == 0
    assert 3.0 < c1.nnz / c1.n / 1.0 < 12.0


# ---------------------------------------------------------------- sampling

def test_sampled_peel_with_every_vertex_sampled_is_exact():
    """With S = V the sampled count is the h-degree and the rate is 1, so
    the sampling-based peel gives the exact core numbers."""
    for g, h in ((synth.chung_lu(300, 6.0, 2.5, seed=3), 2), (synth.rmat(8, 8, seed=2), 3),
                 (synth.petersen(), 2), (synth.cycle(11), 2)):
        c, est = oracle.peel_sampled(g, h, np.ones(g.n, np.uint8))
        assert (c == oracle.peel(g, h)[0]).all()


@settings(max_examples=25, deadline=None)
@given(st.integers(5, 9), st.floats(0.2, 0.7), st.integers(0, 10 ** 6), st.integers(1, 3), st.floats(0.2, 0.8))
def test_sampled_peel_matches_brute_force(n, p, seed, h, rate):
    g = synth.erdos_renyi(n, p, seed)
    sampled = (np.random.default_rng(seed + 1).random(n) < rate).astype(np.uint8)
    c, _ = oracle.peel_sampled(g, h, sampled)
    ref = R.brute_core_sampled(g.n, g.row_ptr, g.col, h, sampled)
    assert (c == ref).all(), (c, ref)


def test_sampled_estimate_never_grows_and_starts_exact():
    """The estimate at removal is at most the initial h-degree (sel <= sel0),
    and a vertex removed in the first round keeps its exact degree."""
    g = synth.chung_lu(800, 8.0, 2.5, seed=9)
    sampled = (np.random.default_rng(4).random(g.n) < 0.2).astype(np.uint8)
    c, est = oracle.peel_sampled(g, 2, sampled)
    d0 = oracle.hdeg(g, 2)
    assert (est <= d0).all()
    first = c == c.min()
    assert (est[first & (c == d0.min())] == d0[first & (c == d0.min())]).all()


# ------------------------------------------------ local h-degree update

def test_table2_bitmaps():
    """Table 2 / Example 3: relabelling, region edges and every bitmap row."""
    g, _ = _golden()
    rows = {ln.split()[0] + ("" if ln.split()[0] != "bitmaps" else " " + ln.split()[1]): ln.split()[1:]
            for ln in open(os.path.join(GOLDEN, "table2_bitmaps.txt")) if ln.strip() and not ln.startswith("#")}
    alive = np.ones(14, dtype=np.uint8)
    for x in rows["remove"]:
        alive[int(x) - 1] = 0
    v, h = int(rows["vertex"][0]) - 1, int(rows["h"][0])
    labels, edges, hist, new = R.bitmap_update(g.n, g.row_ptr, g.col, alive, h, v)
    assert [u + 1 for u in labels] == [int(x) for x in rows["relabel"]]
    assert edges == sorted(tuple(int(a) for a in e.split("-")) for e in rows["region_edges"])
    assert hist[0] == [int(x) for x in rows["bitmaps init"][1:]]
    assert hist[1] == [int(x) for x in rows["bitmaps iter1"][1:]]
    assert hist[2] == [int(x) for x in rows["bitmaps iter2"][1:]]
    # and the updated degrees are the recomputed ones (Observation 2)
    after = alive.copy()
    after[v] = 0
    d = oracle.hdeg(g, h, after)
    assert all(d[u] == k for u, k in new.items())


def test_example2_by_bitmap_update():
    """Example 2: deleting v1 (h = 2) leaves v2, v3, v4, v6 with 2-hop
    degrees 3, 3, 7, 7."""
    g, _ = _golden()
    _, _, _, new = R.bitmap_update(g.n, g.row_ptr, g.col, np.ones(14, np.uint8), 2, 0)
    assert {u + 1: k for u, k in new.items()} == {2: 3, 3: 3, 4: 7, 6: 7}


@settings(max_examples=40, deadline=None)
@given(st.integers(6, 30), st.floats(0.08, 0.5), st.integers(0, 10 ** 6), st.integers(1, 4))
def test_bitmap_update_equals_recompute(n, p, seed, h):
    """Theorem 1 / Observation 2: the update inside the ball equals the
    h-degrees recomputed on the whole graph without v."""
    g = synth.erdos_renyi(n, p, seed)
    rng = np.random.default_rng(seed)
    alive = (rng.random(n) < 0.85).astype(np.uint8)
    live = np.flatnonzero(alive)
    if live.size == 0:
        return
    v = int(rng.choice(live))
    _, _, _, new = R.bitmap_update(g.n, g.row_ptr, g.col, alive, h, v)
    after = alive.copy()
    after[v] = 0
    d = oracle.hdeg(g, h, after)
    assert all(d[u] == k for u, k in new.items())


@settings(max_examples=40, deadline=None)
@given(st.integers(6, 30), st.floats(0.08, 0.5), st.integers(0, 10 ** 6), st.integers(1, 4), st.integers(1, 5))
def test_set_local_update_equals_recompute(n, p, seed, h, k):
    """The set form: removing several vertices at once, the region-only
    update equals the recomputed h-degrees of every affected vertex."""
    g = synth.erdos_renyi(n, p, seed)
    rng = np.random.default_rng(seed + 7)
    alive = (rng.random(n) < 0.9).astype(np.uint8)
    live = np.flatnonzero(alive)
    if live.size == 0:
        return
    P = rng.choice(live, size=min(k, live.size), replace=False)
    new = R.set_local_update(g.n, g.row_ptr, g.col, alive, h, P)
    after = alive.copy()
    after[P] = 0
    d = oracle.hdeg(g, h, after)
    assert all(d[u] == k2 for u, k2 in new.items())
    # a dropped term (the pre-removal reach test) would count vertices that
    # were never within h hops: on some case the plain difference differs
