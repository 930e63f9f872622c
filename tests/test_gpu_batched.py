"""GPU parity of the batched decomposition (many graphs, one persistent
kernel): every graph's core numbers and removal rounds equal the oracle's
for that graph alone."""
import numpy as np
import pytest

import oracle
from paper_2006_03372_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2006_03372_amd import khcore
    c = khcore.Context(0)
    c.set_option(khcore.OPT_BARRIER_TIMEOUT, 10)
    yield c
    torch.cuda.synchronize()
    c.close()


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _graphs(count, lo, hi, seed):
    rng = np.random.default_rng(seed)
    ns = rng.integers(lo, hi + 1, size=count)
    ms = rng.uniform(3.0, 10.0, size=count)
    return [synth.chung_lu(int(ns[i]), float(ms[i]), 2.5, seed * 1000 + i) for i in range(count)]


def _run(ctx, graphs, h, schedule=1, width=16):
    from paper_2006_03372_amd import khcore
    ctx.set_option(khcore.OPT_SCHEDULE, schedule)
    ctx.set_option(khcore.OPT_PERSIST_WIDTH, width)
    b = ctx.batch(graphs)
    c, r, st = ctx.core(b, h, with_round=True)
    out = _u32(c), _u32(r), st, b.vtx_base_host
    b.close()
    return out


@pytest.mark.parametrize("h", [2, 3])
def test_batch_matches_oracle_per_graph(ctx, h):
    graphs = _graphs(24, 30, 700, seed=5 + h)
    graphs.append(synth.from_edges(7, [], []))          # isolated vertices only
    graphs.append(synth.cycle(2 * h + 3))               # closed form: all 2h
    graphs.insert(3, synth.complete(9))                 # closed form: all 8
    for sched in (0, 1, 3):
        for width in (8, 32):
            print(f"batch h={h} schedule={sched} width={width} graphs={len(graphs)}", flush=True)
            c, r, st, vb = _run(ctx, graphs, h, sched, width)
            for i, g in enumerate(graphs):
                lo, hi = int(vb[i]), int(vb[i + 1])
                c_ref, r_ref = oracle.peel(g, h)
                assert (c[lo:hi] == c_ref).all(), (i, sched, width)
                assert (r[lo:hi] == r_ref).all(), (i, sched, width)
            assert st["rounds"] == max(int(oracle.peel(g, h)[1].max()) + 1 for g in graphs if g.n)


def test_batch_equals_single_graph_runs(ctx):
    from paper_2006_03372_amd import khcore
    graphs = _graphs(12, 200, 3000, seed=11)
    c, r, st, vb = _run(ctx, graphs, 3)
    ctx.set_option(khcore.OPT_DRIVER, 1)
    for i, g in enumerate(graphs):
        gr = ctx.graph(g)
        cs, rs, _ = ctx.core(gr, 3, with_round=True)
        gr.close()
        lo, hi = int(vb[i]), int(vb[i + 1])
        assert (c[lo:hi] == _u32(cs)).all()
        assert (r[lo:hi] == _u32(rs)).all()
    # deterministic
    c2, r2, _, _ = _run(ctx, graphs, 3)
    assert (c == c2).all() and (r == r2).all()


def test_batch_schedule3_matches_schedule1(ctx):
    """Schedule 3 in the persistent kernel (decremented (h-1)-degree bounds,
    refreshed by the cleaning BFS) removes the same vertices in the same
    rounds as schedule 1, and computes (h-1)-degrees only for the vertices
    whose h-degree it recomputes."""
    graphs = _graphs(16, 300, 4000, seed=23)
    for h in (3, 4):
        print(f"batch schedule 1 vs 3 h={h} graphs={len(graphs)}", flush=True)
        c1, r1, st1, _ = _run(ctx, graphs, h, 1, 16)
        c3, r3, st3, _ = _run(ctx, graphs, h, 3, 16)
        assert (c1 == c3).all() and (r1 == r3).all(), h
        assert st1["rounds"] == st3["rounds"]
        # the initial pass computes both degrees of every vertex; later
        # (h-1)-degrees come only with the cleaning recomputes
        assert st3["hm1_recomputes"] == st3["h_recomputes"]


def test_batch_rejects_foreign_column(ctx):
    import torch
    from paper_2006_03372_amd import khcore
    g0 = synth.path(4)
    g1 = synth.path(3)
    vb = torch.tensor([0, 4, 7], dtype=torch.int64, device="cuda")
    rp = np.concatenate([g0.row_ptr[:-1], g1.row_ptr + g0.row_ptr[-1]]).astype(np.uint64)
    col = np.concatenate([g0.col, g1.col]).astype(np.uint32)
    col[0] = 5  # vertex 0 of graph 0 points outside graph 0
    rpt = torch.from_numpy(rp.view(np.int64)).cuda()
    ct = torch.from_numpy(col.view(np.int32)).cuda()
    import ctypes
    h = ctypes.c_void_p()
    rc = ctx.lib.khc_graph_create_batched(ctx.handle, 2, ctypes.c_void_p(vb.data_ptr()),
                                          ctypes.c_void_p(rpt.data_ptr()), ctypes.c_void_p(ct.data_ptr()),
                                          int(rp[-1]), ctypes.byref(h))
    assert rc == khcore.KHC_EGRAPH


def test_batch_deep_h_and_closed_forms(ctx):
    """h = 5 on small graphs, including closed forms (cycles: 2h; complete: n-1)."""
    graphs = _graphs(6, 20, 200, seed=11) + [synth.cycle(13), synth.cycle(40), synth.complete(7), synth.path(9)]
    c, r, st, vb = _run(ctx, graphs, 5, 1, 8)
    for i, g in enumerate(graphs):
        lo, hi = int(vb[i]), int(vb[i + 1])
        c_ref, r_ref = oracle.peel(g, 5)
        assert (c[lo:hi] == c_ref).all(), i
        assert (r[lo:hi] == r_ref).all(), i
    assert (c[int(vb[7]):int(vb[8])] == 10).all()   # cycle of 40 at h = 5
    assert (c[int(vb[8]):int(vb[9])] == 6).all()    # K7


def test_batch_with_multi_chunk_hub(ctx):
    """A star with 9000 leaves (rows of several 4096-arc chunks, pulled and
    pushed inside its graph's word window) next to small graphs."""
    graphs = _graphs(5, 100, 1500, seed=12)
    graphs.insert(2, synth.star(9000))
    for width in (8, 32):
        c, r, st, vb = _run(ctx, graphs, 2, 1, width)
        for i, g in enumerate(graphs):
            lo, hi = int(vb[i]), int(vb[i + 1])
            c_ref, r_ref = oracle.peel(g, 2)
            assert (c[lo:hi] == c_ref).all(), (i, width)
            assert (r[lo:hi] == r_ref).all(), (i, width)
