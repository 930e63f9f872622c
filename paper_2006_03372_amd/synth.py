"""Seeded synthetic graph inputs and the CSR container.

This module only builds inputs: it draws random graphs from a seed and
packs them as simple undirected CSR graphs (rows sorted, no self-loops, no
duplicate edges, every edge stored in both directions).  It holds none of
the h-degree or core-number arithmetic, so both the GPU library's tests and
the CPU oracle may use it.

Graph model: an undirected unweighted graph G=(V,E) (Section II of the
paper).  The paper's real datasets are replaced by two seeded stand-ins
with the same power-law shape:

* Chung-Lu: expected degrees drawn from a power law with density exponent
  beta (Pareto shape beta-1), rescaled to a target mean; each pair i<j is an
  edge independently with probability min(1, w_i w_j / sum(w)).  Sampled
  exactly in O(n + m) with the Miller-Hagberg skipping method, vectorised
  over all rows at once.
* R-MAT: ef * 2^scale edge samples, each choosing one of four quadrants per
  bit level with probabilities a, b, c, d; then symmetrised, self-loops and
  duplicates removed, and vertex ids permuted by a seeded permutation.
"""
from __future__ import annotations

import dataclasses
import numpy as np


@dataclasses.dataclass
class CSR:
    """Simple undirected graph in compressed sparse row form (host arrays).

    row_ptr: uint64[n+1], monotone, row_ptr[0] == 0, row_ptr[n] == nnz.
    col:     uint32[nnz], neighbours of each row sorted ascending.
    Every undirected edge {u, v} appears as arc u->v and arc v->u.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def num_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def from_edges(n: int, u, v) -> CSR:
    """Build a simple undirected CSR from an (unordered) edge list.

    Self-loops are dropped, both directions are added, duplicates removed.
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.shape != v.shape:
        raise ValueError("edge endpoint arrays differ in length")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * np.int64(n) + dst)
    src = key // n
    dst = key - src * n
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n=n, row_ptr=row_ptr, col=dst.astype(np.uint32))


def edge_list(g: CSR):
    """Return (u, v) arrays with u < v, one entry per undirected edge."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    dst = g.col.astype(np.int64)
    m = src < dst
    return src[m], dst[m]


def induced(g: CSR, keep) -> tuple[CSR, np.ndarray]:
    """Induced subgraph on the vertices where keep is true, relabelled 0..k-1.

    Returns (subgraph, old_ids) with old_ids[new] = old.
    """
    keep = np.asarray(keep, dtype=bool)
    old = np.flatnonzero(keep)
    new_id = -np.ones(g.n, dtype=np.int64)
    new_id[old] = np.arange(old.size)
    u, v = edge_list(g)
    m = keep[u] & keep[v]
    return from_edges(old.size, new_id[u[m]], new_id[v[m]]), old


def disjoint_union(graphs) -> CSR:
    """Disjoint union: graph i's vertex j becomes offset_i + j."""
    us, vs, off = [], [], 0
    for g in graphs:
        u, v = edge_list(g)
        us.append(u + off)
        vs.append(v + off)
        off += g.n
    if not us:
        return from_edges(0, [], [])
    return from_edges(off, np.concatenate(us), np.concatenate(vs))


# ---------------------------------------------------------------- generators

def chung_lu(n: int, mean_degree: float = 10.0, beta: float = 2.5, seed: int = 1) -> CSR:
    """Chung-Lu power-law graph with exact per-pair Bernoulli sampling.

    Weights w_i = (1-U_i)^(-1/(beta-1)) (power-law density exponent beta),
    rescaled so that mean(w) == mean_degree.  Pair {i, j}, i != j, is an
    edge with probability min(1, w_i w_j / S), S = sum(w).  Sampled with the
    Miller-Hagberg geometric skipping over rows in descending weight order;
    all rows advance together in vectorised steps.
    """
    if n <= 0:
        return from_edges(0, [], [])
    rng = np.random.default_rng(seed)
    w = (1.0 - rng.random(n)) ** (-1.0 / (beta - 1.0))
    w *= mean_degree / w.mean()
    order = np.argsort(-w, kind="stable")
    ws = w[order]
    S = ws.sum()
    # per-row cursor: candidate column index (into ws), current bound p
    rows = np.arange(n - 1, dtype=np.int64)
    v = rows + 1
    p = np.minimum(ws[rows] * ws[v] / S, 1.0)
    out_u, out_v = [], []
    active = np.flatnonzero(p > 0)
    rows, v, p = rows[active], v[active], p[active]
    while rows.size:
        r = rng.random(rows.size)
        skip = np.zeros(rows.size, dtype=np.int64)
        frac = p < 1.0
        with np.errstate(divide="ignore"):
            skip[frac] = np.floor(np.log(r[frac]) / np.log1p(-p[frac])).astype(np.int64)
        v = v + skip
        live = v < n
        rows, v, p = rows[live], v[live], p[live]
        if not rows.size:
            break
        q = np.minimum(ws[rows] * ws[v] / S, 1.0)
        r2 = rng.random(rows.size)
        acc = r2 < q / p
        out_u.append(rows[acc])
        out_v.append(v[acc])
        p = q
        v = v + 1
        live = (v < n) & (p > 0)
        rows, v, p = rows[live], v[live], p[live]
    if out_u:
        uu = order[np.concatenate(out_u)]
        vv = order[np.concatenate(out_v)]
    else:
        uu = vv = np.zeros(0, dtype=np.int64)
    return from_edges(n, uu, vv)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, permute: bool = True,
         chunk: int = 1 << 22) -> CSR:
    """R-MAT graph on 2^scale vertices from edge_factor * 2^scale samples.

    Each sample picks, per bit level, quadrant (0,0) with probability a,
    (0,1) with b, (1,0) with c and (1,1) with d = 1-a-b-c.  No noise.  The
    result is symmetrised and deduplicated with self-loops dropped; with
    permute=True vertex ids are relabelled by a seeded random permutation.
    """
    n = 1 << scale
    m = edge_factor * n
    rng = np.random.default_rng(seed)
    ab = a + b
    c_norm = c / (1.0 - ab)
    a_norm = a / ab
    us, vs = [], []
    done = 0
    while done < m:
        k = min(chunk, m - done)
        u = np.zeros(k, dtype=np.int64)
        v = np.zeros(k, dtype=np.int64)
        for bit in range(scale):
            r1 = rng.random(k)
            r2 = rng.random(k)
            ubit = r1 > ab
            vbit = np.where(ubit, r2 > c_norm, r2 > a_norm)
            u |= ubit.astype(np.int64) << bit
            v |= vbit.astype(np.int64) << bit
        us.append(u)
        vs.append(v)
        done += k
    u = np.concatenate(us)
    v = np.concatenate(vs)
    if permute:
        perm = rng.permutation(n)
        u = perm[u]
        v = perm[v]
    return from_edges(n, u, v)


def batch_chung_lu(count: int = 256, n_lo: int = 500, n_hi: int = 20000,
                   mean_lo: float = 4.0, mean_hi: float = 16.0, beta: float = 2.5,
                   seed: int = 7):
    """A list of independent Chung-Lu graphs of uneven size.

    Graph i uses n ~ integer-uniform [n_lo, n_hi], mean degree ~ uniform
    [mean_lo, mean_hi], and its own seed seed + i.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    means = rng.uniform(mean_lo, mean_hi, size=count)
    return [chung_lu(int(ns[i]), float(means[i]), beta, seed + i) for i in range(count)]


def random_alive(n: int, frac: float, seed: int) -> np.ndarray:
    """uint8 mask with each vertex alive independently with probability frac."""
    rng = np.random.default_rng(seed)
    return (rng.random(n) < frac).astype(np.uint8)


def erdos_renyi(n: int, p: float, seed: int) -> CSR:
    """G(n, p) on small n (dense pair enumeration)."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    m = rng.random(iu.size) < p
    return from_edges(n, iu[m], ju[m])


# ------------------------------------------------------ closed-form families

def complete(n: int) -> CSR:
    iu, ju = np.triu_indices(n, 1)
    return from_edges(n, iu, ju)


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n)


def path(n: int) -> CSR:
    i = np.arange(max(n - 1, 0))
    return from_edges(n, i, i + 1)


def star(m: int) -> CSR:
    """Centre 0 joined to leaves 1..m."""
    return from_edges(m + 1, np.zeros(m, dtype=np.int64), np.arange(1, m + 1))


def complete_bipartite(a: int, b: int) -> CSR:
    u = np.repeat(np.arange(a), b)
    v = a + np.tile(np.arange(b), a)
    return from_edges(a + b, u, v)


def petersen() -> CSR:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    e = np.array(outer + spokes + inner)
    return from_edges(10, e[:, 0], e[:, 1])


def hypercube(d: int) -> CSR:
    n = 1 << d
    us, vs = [], []
    for bit in range(d):
        x = np.arange(n)
        m = (x >> bit) & 1 == 0
        us.append(x[m])
        vs.append(x[m] | (1 << bit))
    return from_edges(n, np.concatenate(us), np.concatenate(vs))


def torus(rows: int, cols: int) -> CSR:
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    idx = r * cols + c
    right = r * cols + (c + 1) % cols
    down = ((r + 1) % rows) * cols + c
    return from_edges(rows * cols, np.concatenate([idx.ravel(), idx.ravel()]),
                      np.concatenate([right.ravel(), down.ravel()]))
