"""GPU parity of khcore_decompose with the CPU oracle (bit-exact core numbers
and removal rounds)."""
import os

import numpy as np
import pytest

import oracle
from paper_2006_03372_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def _gpu_core(ctx, g, h, schedule=1, width=16, driver=1):
    from paper_2006_03372_amd import khcore
    ctx.set_option(khcore.OPT_SCHEDULE, schedule)
    ctx.set_option(khcore.OPT_MAX_WIDTH, width)
    ctx.set_option(khcore.OPT_DRIVER, driver)
    ctx.set_option(khcore.OPT_PERSIST_WIDTH, max(width, 8))
    ctx.set_option(khcore.OPT_BARRIER_TIMEOUT, 10)
    gr = ctx.graph(g)
    c, r, st = ctx.core(gr, h, with_round=True)
    out = _u32(c), _u32(r), st
    gr.close()
    return out


def _check(ctx, g, h, schedules=(0, 1, 3), widths=(16,), drivers=(0, 1)):
    c_ref, r_ref = oracle.peel(g, h)
    for drv in drivers:
        for s in schedules:
            for w in widths:
                print(f"core n={g.n} nnz={g.nnz} h={h} driver={drv} schedule={s} width={w}", flush=True)
                c, r, st = _gpu_core(ctx, g, h, s, w, drv)
                assert (c == c_ref).all(), (drv, s, w, np.flatnonzero(c != c_ref)[:10])
                assert (r == r_ref).all(), (drv, s, w, np.flatnonzero(r != r_ref)[:10])


@pytest.mark.parametrize("h", [1, 2, 3, 5])
def test_closed_forms(ctx, h):
    for n in (2 * h + 1, 2 * h + 4, 17):
        c, _, _ = _gpu_core(ctx, synth.cycle(n), h)
        assert (c == 2 * h).all()
    c, _, _ = _gpu_core(ctx, synth.complete(8), h)
    assert (c == 7).all()
    c, _, _ = _gpu_core(ctx, synth.path(12), h)
    assert (c == min(h, 11)).all()
    c, _, _ = _gpu_core(ctx, synth.from_edges(5, [0], [1]), h)
    assert list(c) == [1, 1, 0, 0, 0]


def test_running_example(ctx):
    lines = [ln.split() for ln in open(os.path.join(GOLDEN, "running_example.txt"))
             if ln.strip() and not ln.startswith("#")]
    e = np.array([tuple(int(x) - 1 for x in t.split("-")) for t in lines[0][1:]])
    g = synth.from_edges(14, e[:, 0], e[:, 1])
    for f in lines[1:]:
        if f[0] == "core":
            h = int(f[1].split("=")[1])
            c, _, _ = _gpu_core(ctx, g, h)
            assert list(c) == [int(x) for x in f[2:]]


@pytest.mark.parametrize("h", [1, 2, 3, 4])
def test_chung_lu_2000(ctx, h):
    g = synth.chung_lu(2000, 10.0, 2.5, seed=1)
    _check(ctx, g, h, widths=(8, 32))


@pytest.mark.parametrize("h", [2, 3, 4])
def test_rmat_12(ctx, h):
    g = synth.rmat(12, 8, seed=1)
    _check(ctx, g, h)


def test_disjoint_union_and_isolated(ctx):
    parts = [synth.chung_lu(n, m, 2.5, s) for n, m, s in ((300, 5.0, 1), (700, 9.0, 2), (50, 3.0, 3))]
    g = synth.disjoint_union(parts + [synth.from_edges(9, [], [])])
    _check(ctx, g, 3)


def test_certificate_rmat14_h3(ctx):
    """R-MAT scale 14, h=3: the peeling-order certificate on sampled
    vertices plus exact oracle h-degrees of sampled vertices."""
    g = synth.rmat(14, 8, seed=1)
    c, r, st = _gpu_core(ctx, g, 3)
    rng = np.random.default_rng(0)
    verts = rng.choice(g.n, size=300, replace=False)
    fail = oracle.certificate(g, 3, c, r, verts)
    assert fail.sum() == 0, fail


def _with_hubs(g, hubs, deg, seed):
    """g plus `hubs` new vertices, each joined to `deg` random vertices of g."""
    rng = np.random.default_rng(seed)
    src, dst = synth.edge_list(g)
    extra_s, extra_d = [src], [dst]
    for i in range(hubs):
        nb = rng.choice(g.n, size=deg, replace=False)
        extra_s.append(np.full(deg, g.n + i))
        extra_d.append(nb)
    return synth.from_edges(g.n + hubs, np.concatenate(extra_s), np.concatenate(extra_d))


@pytest.mark.parametrize("h", [2, 3])
def test_multi_chunk_hubs(ctx, h):
    """Rows longer than one 4096-arc chunk (pulled by several wavefronts,
    pushed as several items): both drivers and schedules agree, and the
    certificate holds on sampled vertices and on the hubs."""
    g = _with_hubs(synth.chung_lu(6000, 4.0, 2.5, seed=3), 2, 5000, seed=4)
    assert np.diff(g.row_ptr).max() > 4096
    runs = [_gpu_core(ctx, g, h, s, 16, drv) for drv in (0, 1) for s in (0, 1)]
    c, r, _ = runs[0]
    for c2, r2, _ in runs[1:]:
        assert (c2 == c).all() and (r2 == r).all()
    rng = np.random.default_rng(1)
    verts = np.concatenate([rng.choice(g.n, size=200, replace=False), [g.n - 2, g.n - 1]])
    fail = oracle.certificate(g, h, c, r, verts)
    assert fail.sum() == 0, fail


def test_progress_reports(ctx):
    """With a zero interval the host-driven loop reports after every round;
    the last report has every vertex removed."""
    from paper_2006_03372_amd import khcore
    g = synth.chung_lu(1500, 8.0, 2.5, seed=5)
    seen = []
    ctx.set_progress(lambda r, removed, level: seen.append((r, removed, level)), 0)
    try:
        c, r, st = _gpu_core(ctx, g, 2, 1, 16, 0)
    finally:
        ctx.set_progress(None)
    assert len(seen) == st["rounds"]
    assert [x[0] for x in seen] == list(range(1, st["rounds"] + 1))
    assert seen[-1][1] == g.n and seen[-1][2] == c.max()
    assert all(a[1] < b[1] and a[2] <= b[2] for a, b in zip(seen, seen[1:]))


def test_persistent_progress_reports(ctx):
    """The persistent kernel publishes its progress to host memory while it
    runs; reports are monotone and never ahead of the final statistics."""
    g = synth.rmat(12, 8, seed=1)
    seen = []
    ctx.set_progress(lambda r, removed, level: seen.append((r, removed)), 0)
    try:
        c, r, st = _gpu_core(ctx, g, 3, 1, 16, 1)
    finally:
        ctx.set_progress(None)
    print("reports", len(seen), "wall ms", st["wall_ms"], flush=True)
    if st["wall_ms"] > 100:
        assert seen
    assert all(a[0] <= b[0] and a[1] <= b[1] for a, b in zip(seen, seen[1:]))
    assert all(x[0] <= st["rounds"] and x[1] <= g.n for x in seen)
