"""GPU parity of khdeg_compute / khdeg_compute_list with the CPU oracle.

Integer results: every comparison is bit-exact.
"""
import numpy as np
import pytest

import oracle
from paper_2006_03372_amd import synth

pytestmark = pytest.mark.gpu

WIDTHS = [1, 2, 4, 8, 16, 32]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2006_03372_amd import khcore
    c = khcore.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _gpu_hdeg(ctx, g, h, alive=None, width=16):
    import torch
    from paper_2006_03372_amd import khcore
    ctx.set_option(khcore.OPT_MAX_WIDTH, width)
    gr = ctx.graph(g)
    a = None if alive is None else torch.from_numpy(alive).to(gr.device)
    d = _u32(ctx.hdeg(gr, h, a))
    gr.close()
    return d


def _check(ctx, g, h, alive=None, widths=(16,)):
    ref = oracle.hdeg(g, h, alive)
    for w in widths:
        print(f"hdeg n={g.n} nnz={g.nnz} h={h} width={w} alive={'all' if alive is None else int(alive.sum())}",
              flush=True)
        d = _gpu_hdeg(ctx, g, h, alive, w)
        assert (d == ref).all(), (w, np.flatnonzero(d != ref)[:10], d[d != ref][:10], ref[d != ref][:10])


@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_closed_form_families(ctx, h):
    for g in (synth.complete(9), synth.cycle(13), synth.path(11), synth.star(7),
              synth.complete_bipartite(4, 5), synth.petersen(), synth.hypercube(5),
              synth.torus(2 * h + 3, 2 * h + 5)):
        _check(ctx, g, h, widths=(1, 16))


@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_chung_lu_all_widths(ctx, h):
    g = synth.chung_lu(2000, 10.0, 2.5, seed=1)
    _check(ctx, g, h, widths=WIDTHS)


@pytest.mark.parametrize("h", [2, 3])
def test_random_alive_masks(ctx, h):
    g = synth.chung_lu(3000, 8.0, 2.5, seed=4)
    for seed, frac in ((1, 0.9), (2, 0.5), (3, 0.1)):
        alive = synth.random_alive(g.n, frac, seed)
        _check(ctx, g, h, alive, widths=(1, 4, 16))


def test_heavy_rows_and_chunks(ctx):
    # a hub with 9000 arcs is cut into three chunks; 600-arc hubs are heavy
    # single-chunk rows; rows are ragged around the lane-group sizes
    parts = [synth.star(9000), synth.star(600), synth.chung_lu(1500, 6.0, 2.5, seed=9),
             synth.complete(40)]
    g = synth.disjoint_union(parts)
    u, v = synth.edge_list(g)
    # tie the hubs together so heavy rows feed each other's frontiers
    extra_u = np.array([0, 0, 9001, 9001 + 601])
    extra_v = np.array([9001, 9001 + 601 + 5, 9001 + 601 + 100, 9001 + 601 + 1500 + 3])
    g = synth.from_edges(g.n, np.concatenate([u, extra_u]), np.concatenate([v, extra_v]))
    for h in (1, 2, 3):
        _check(ctx, g, h, widths=(1, 2, 16, 32))
    alive = synth.random_alive(g.n, 0.7, 5)
    alive[0] = 1
    _check(ctx, g, 3, alive, widths=(4, 16))


@pytest.mark.parametrize("scale", [10, 12])
def test_rmat(ctx, scale):
    g = synth.rmat(scale, 8, seed=1)
    for h in (1, 2, 3, 4):
        _check(ctx, g, h, widths=(16,))


def test_edge_cases(ctx):
    # single vertex, isolated vertices only, one edge, all dead, n not a multiple of 64
    _check(ctx, synth.from_edges(1, [], []), 2)
    _check(ctx, synth.from_edges(70, [], []), 3)
    _check(ctx, synth.from_edges(2, [0], [1]), 1)
    g = synth.chung_lu(333, 5.0, 2.5, seed=2)
    _check(ctx, g, 2, np.zeros(g.n, dtype=np.uint8))
    _check(ctx, g, 2, np.ones(g.n, dtype=np.uint8), widths=(1, 32))
    # h far beyond the diameter gives component size - 1
    _check(ctx, synth.disjoint_union([synth.path(30), synth.cycle(17)]), 40, widths=(1,))


def test_list_variant(ctx):
    import torch
    g = synth.chung_lu(2500, 9.0, 2.5, seed=3)
    alive = synth.random_alive(g.n, 0.8, 6)
    rng = np.random.default_rng(0)
    verts = rng.choice(g.n, size=700, replace=False).astype(np.uint32)
    ref, _ = oracle.hdeg_list(g, 3, verts, alive)
    gr = ctx.graph(g)
    out = ctx.hdeg_list(gr, 3, torch.from_numpy(verts.view(np.int32)).to(gr.device),
                        torch.from_numpy(alive).to(gr.device))
    d = _u32(out)
    assert (d == ref).all()
    # dead listed vertices report 0
    assert (d[alive[verts] == 0] == 0).all()
    gr.close()


def test_deterministic(ctx):
    g = synth.rmat(12, 8, seed=3)
    a = _gpu_hdeg(ctx, g, 3)
    b = _gpu_hdeg(ctx, g, 3)
    assert (a == b).all()


@pytest.mark.parametrize("h", [1, 2, 3])
def test_scanned_arcs(ctx, h):
    g = synth.chung_lu(2000, 10.0, 2.5, seed=1)
    alive = synth.random_alive(g.n, 0.85, 7)
    import torch
    for a in (None, alive):
        verts = np.arange(g.n, dtype=np.uint32)
        _, te_ref = oracle.hdeg_list(g, h, verts, a)
        gr = ctx.graph(g)
        te = ctx.scanned_arcs(gr, h, None if a is None else torch.from_numpy(a).to(gr.device))
        got = te.cpu().numpy().view(np.uint64)
        gr.close()
        assert (got == te_ref).all()
