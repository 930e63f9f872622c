"""GPU parity at the benchmark configurations' own sizes.

* R-MAT scale 16 (ef 8) at h = 2, 3, 4: the peeling-order certificate over
  EVERY vertex (conditions (i)-(iii) on all vertices prove the core numbers
  exact: each C_k is a (k,h)-feasible set, so c <= core; and the first
  removed member of any denser core would contradict (ii) and (iii)), the
  host-driven and persistent drivers give identical cores and rounds, and
  sampled h-degrees of the whole graph match the oracle.
* The 256-graph Chung-Lu batch at h = 3 in one persistent launch: the
  oracle's full peel on the 32 smallest graphs and the certificate on a
  sample of every other graph (a sampled certificate is a spot check, not
  a proof: it tests (i) and (ii) on the sampled vertices only).
* The plain schedule's affected sets: the sum over rounds of |A_r| and the
  round count equal the oracle's trace.
* R-MAT scale 20 (ef 16), the benchmark's graph, in the benchmark's launch
  configuration: h-degrees at h = 2, 3, 4 on sampled vertices equal the
  oracle's, with and without an alive mask; the exact decomposition at
  h = 4 (default schedule) passes the certificate on sampled vertices and
  the hubs (a spot check).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2006_03372_amd import synth

pytestmark = pytest.mark.gpu

THREADS = min(16, oracle.host_threads())


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2006_03372_amd import khcore
    c = khcore.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def rmat16():
    return synth.rmat(16, 8, seed=1)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _core(ctx, gr, h, driver=0, schedule=1):
    from paper_2006_03372_amd import khcore
    ctx.set_option(khcore.OPT_DRIVER, driver)
    ctx.set_option(khcore.OPT_SCHEDULE, schedule)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_PERSIST_WIDTH, 32)
    ctx.set_option(khcore.OPT_BARRIER_TIMEOUT, 30)
    c, r, st = ctx.core(gr, h, with_round=True)
    out = _u32(c), _u32(r), st
    ctx.set_option(khcore.OPT_DRIVER, 0)
    ctx.set_option(khcore.OPT_SCHEDULE, 1)
    return out


def test_rmat16_hdeg_sampled(ctx, rmat16):
    g = rmat16
    gr = ctx.graph(g)
    verts = np.random.default_rng(16).choice(g.n, 2000, replace=False).astype(np.uint32)
    for h in (2, 3, 4):
        d = _u32(ctx.hdeg(gr, h))
        ref, _ = oracle.hdeg_list(g, h, verts, threads=THREADS)
        assert (d[verts] == ref).all(), h
    gr.close()


def test_rmat20_hdeg_sampled_bench_launch(ctx):
    """khdeg_compute over all of R-MAT scale 20 (ef 16, seed 1) with width 32
    and 16 wavefronts per CU, as the benchmark times it: 256 random
    vertices, the 16 highest-degree hubs and 16 isolated vertices match the
    oracle bit for bit at h = 2, 3, 4, and at h = 3 under a random alive
    mask (dead vertices 0)."""
    import torch
    from paper_2006_03372_amd import khcore
    g = synth.rmat(20, 16, seed=1)
    deg = g.degrees()
    rng = np.random.default_rng(20)
    hubs = np.argsort(deg, kind="stable")[-16:]
    isolated = rng.choice(np.flatnonzero(deg == 0), 16, replace=False)
    verts = np.unique(np.concatenate([rng.choice(g.n, 256, replace=False), hubs, isolated])).astype(np.uint32)
    print(f"R-MAT-20 n={g.n} nnz={g.nnz}, {verts.size} sampled vertices", flush=True)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)
    gr = ctx.graph(g)
    for h in (2, 3, 4):
        print(f"R-MAT-20 h={h}", flush=True)
        d = _u32(ctx.hdeg(gr, h))
        ref, _ = oracle.hdeg_list(g, h, verts, threads=THREADS)
        assert (d[verts] == ref).all(), h
        assert (d[isolated] == 0).all()
    alive = synth.random_alive(g.n, 0.9, 21)
    print("R-MAT-20 h=3 with an alive mask", flush=True)
    d = _u32(ctx.hdeg(gr, 3, alive=torch.from_numpy(alive).cuda()))
    ref, _ = oracle.hdeg_list(g, 3, verts, alive=alive, threads=THREADS)
    assert (d[verts] == ref).all()
    assert (d[alive == 0] == 0).all()
    gr.close()


def test_rmat20_h4_decomposition_certificate(ctx):
    """The exact (k,4)-core decomposition of R-MAT scale 20 (ef 16, seed 1)
    with the default schedule and host-driven rounds, width 32: conditions
    (i) and (ii) of the peeling-order certificate hold on 200 random
    vertices and the 16 highest-degree hubs, (iii) on every vertex."""
    from paper_2006_03372_amd import khcore
    g = synth.rmat(20, 16, seed=1)
    deg = g.degrees()
    rng = np.random.default_rng(22)
    verts = np.unique(np.concatenate([rng.choice(g.n, 200, replace=False),
                                      np.argsort(deg, kind="stable")[-16:]])).astype(np.uint32)
    ctx.set_option(khcore.OPT_DRIVER, 0)
    ctx.set_option(khcore.OPT_SCHEDULE, 3)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)
    gr = ctx.graph(g)
    print(f"R-MAT-20 h=4 decomposition n={g.n} nnz={g.nnz}", flush=True)
    c, r, st = ctx.core(gr, 4, with_round=True)
    c, r = _u32(c), _u32(r)
    gr.close()
    ctx.set_option(khcore.OPT_SCHEDULE, 1)
    print(f"rounds {st['rounds']}; certificate on {verts.size} vertices", flush=True)
    fail = oracle.certificate(g, 4, c, r, verts, threads=THREADS)
    assert fail.sum() == 0, fail
    assert (c[deg == 0] == 0).all()


@pytest.mark.parametrize("h", [2, 3, 4])
def test_rmat16_certificate_all_vertices(ctx, rmat16, h):
    g = rmat16
    gr = ctx.graph(g)
    c, r, st = _core(ctx, gr, h)
    print(f"R-MAT-16 h={h}: {st['rounds']} rounds, max core {c.max()}", flush=True)
    fail = oracle.certificate(g, h, c, r, threads=THREADS)
    assert fail.sum() == 0, fail
    # the persistent driver gives the same cores and rounds
    c2, r2, _ = _core(ctx, gr, h, driver=1)
    assert (c2 == c).all() and (r2 == r).all()
    if h == 2:
        # and so does the plain schedule (every affected vertex recomputed)
        c3, r3, _ = _core(ctx, gr, h, schedule=0)
        assert (c3 == c).all() and (r3 == r).all()
    gr.close()


def test_batch256_h3(ctx):
    """One persistent launch over the 256 graphs of the batched
    configuration; oracle peel on the 32 smallest, certificate samples on
    the others."""
    from paper_2006_03372_amd import khcore
    graphs = synth.batch_chung_lu(256)
    bg = ctx.batch(graphs)
    ctx.set_option(khcore.OPT_PERSIST_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 4)
    ctx.set_option(khcore.OPT_BARRIER_TIMEOUT, 60)
    c, r, st = ctx.core(bg, 3, with_round=True)
    c, r = _u32(c), _u32(r)
    bg.close()
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    np.cumsum([g.n for g in graphs], out=off[1:])
    order = np.argsort([g.n for g in graphs], kind="stable")
    small, rest = order[:32], order[32:]
    print(f"batch: {st['rounds']} rounds; 32 smallest graphs n <= {graphs[small[-1]].n}", flush=True)

    def full(i):
        cr, rr = oracle.peel(graphs[i], 3)
        return i, bool((c[off[i]:off[i + 1]] == cr).all() and (r[off[i]:off[i + 1]] == rr).all())

    def sampled(i):
        g = graphs[i]
        verts = np.random.default_rng(int(i)).choice(g.n, min(8, g.n), replace=False).astype(np.uint32)
        fail = oracle.certificate(g, 3, c[off[i]:off[i + 1]], r[off[i]:off[i + 1]], verts)
        return i, int(fail.sum())

    with ThreadPoolExecutor(THREADS) as ex:
        res_full = list(ex.map(full, small))
        res_cert = list(ex.map(sampled, rest))
    assert all(ok for _, ok in res_full), [i for i, ok in res_full if not ok]
    assert all(f == 0 for _, f in res_cert), [i for i, f in res_cert if f]


@pytest.mark.parametrize("h", [2, 3])
def test_plain_schedule_affected_sets_match_trace(ctx, h):
    g = synth.chung_lu(2000, 10.0, 2.5, seed=1)
    gr = ctx.graph(g)
    c, r, st = _core(ctx, gr, h, schedule=0)
    gr.close()
    c_ref, r_ref, trace = oracle.peel(g, h, trace=True)
    assert (c == c_ref).all() and (r == r_ref).all()
    assert st["rounds"] == trace.shape[0]
    assert st["affected_total"] == int(trace[:, 2].astype(np.int64).sum())
    assert st["h_recomputes"] == g.n + int(trace[:, 2].astype(np.int64).sum())
