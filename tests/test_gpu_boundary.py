"""GPU tests of the C ABI's error paths and less used entry points: every
class of invalid CSR gives KHC_EGRAPH, the workspace cap gives KHC_ENOMEM
(and the context stays usable), h = 0 gives KHC_EINVAL, out-of-range ids of
khdeg_compute_list are refused before any kernel reads them, a vertex
listed twice gets its h-degree on both entries, and khcore_decompose_batched
called directly matches the oracle per graph."""
import ctypes

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
    yield c
    torch.cuda.synchronize()
    c.close()


def _dev(a, dtype):
    import torch
    a = np.ascontiguousarray(a, dtype=dtype)
    view = {np.uint64: np.int64, np.uint32: np.int32}[dtype]
    return torch.from_numpy(a.view(view)).cuda()


def _raw_csr(ctx, n, row_ptr, col, nnz=None):
    """(validate code, graph_create code) for a CSR given as host arrays."""
    from paper_2006_03372_amd import khcore
    rp = _dev(row_ptr, np.uint64)
    cl = _dev(col if len(col) else [0], np.uint32)
    s = khcore.CSRStruct(n, int(row_ptr[-1]) if nnz is None else nnz, ctypes.c_void_p(rp.data_ptr()),
                         ctypes.c_void_p(cl.data_ptr()))
    rc_v = ctx.lib.khc_validate_csr(ctx.handle, ctypes.byref(s))
    h = ctypes.c_void_p()
    rc_g = ctx.lib.khc_graph_create(ctx.handle, ctypes.byref(s), ctypes.byref(h))
    if rc_g == 0:
        ctx.lib.khc_graph_destroy(h)
    return rc_v, rc_g, ctx.lib.khc_last_error(ctx.handle).decode()


# a path 0-1-2-3 and the ways to spoil it
GOOD = (4, [0, 1, 3, 5, 6], [1, 0, 2, 1, 3, 2])
BAD = {
    "asymmetric": (4, [0, 1, 3, 5, 6], [1, 0, 2, 1, 3, 1]),       # 3->1 without 1->3
    "self_loop": (4, [0, 2, 4, 6, 7], [0, 1, 0, 2, 1, 3, 2]),      # 0->0
    "unsorted": (4, [0, 1, 3, 5, 6], [1, 2, 0, 1, 3, 2]),          # row 1 is (2, 0)
    "duplicate_arc": (4, [0, 2, 4, 6, 7], [1, 1, 0, 0, 2, 3, 2]),  # 0->1 twice
    "column_out_of_range": (4, [0, 1, 3, 5, 6], [1, 0, 2, 1, 7, 2]),
    "row_ptr_decreasing": (4, [0, 3, 1, 5, 6], [1, 0, 2, 1, 3, 2]),
    "row_ptr0_nonzero": (4, [1, 1, 3, 5, 6], [1, 0, 2, 1, 3, 2]),
}


def test_valid_csr_is_accepted(ctx):
    rc_v, rc_g, _ = _raw_csr(ctx, *GOOD)
    assert (rc_v, rc_g) == (0, 0)


@pytest.mark.parametrize("case", sorted(BAD))
def test_invalid_csr_gives_egraph(ctx, case):
    from paper_2006_03372_amd import khcore
    n, rp, col = BAD[case]
    assert oracle.check_csr(synth.CSR(n, np.array(rp, np.uint64), np.array(col, np.uint32))) != 0
    rc_v, rc_g, msg = _raw_csr(ctx, n, rp, col)
    print(case, rc_v, rc_g, msg, flush=True)
    assert rc_v == khcore.KHC_EGRAPH and rc_g == khcore.KHC_EGRAPH


def test_nnz_mismatch_gives_egraph(ctx):
    from paper_2006_03372_amd import khcore
    n, rp, col = GOOD
    rc_v, rc_g, _ = _raw_csr(ctx, n, rp, col, nnz=5)
    assert rc_v == khcore.KHC_EGRAPH and rc_g == khcore.KHC_EGRAPH


def test_workspace_limit_gives_enomem_and_context_recovers(ctx):
    import torch
    from paper_2006_03372_amd import khcore
    g = synth.rmat(12, 8, seed=5)
    gr = ctx.graph(g)
    # a fresh context so the cap is hit by growth, not by buffers sized earlier
    with khcore.Context(0) as c2:
        g2 = c2.graph(g)
        c2.set_option(khcore.OPT_WORKSPACE_LIMIT, 64 << 10)
        with pytest.raises(khcore.KhcError) as e:
            c2.hdeg(g2, 3)
        assert e.value.code == khcore.KHC_ENOMEM
        c2.set_option(khcore.OPT_WORKSPACE_LIMIT, 0)
        d = c2.hdeg(g2, 3)
        torch.cuda.synchronize()
        assert (d.cpu().numpy().view(np.uint32) == oracle.hdeg(g, 3)).all()
        g2.close()
    gr.close()


def test_h_zero_is_rejected(ctx):
    from paper_2006_03372_amd import khcore
    gr = ctx.graph(synth.cycle(9))
    for call in (lambda: ctx.hdeg(gr, 0), lambda: ctx.core(gr, 0), lambda: ctx.scanned_arcs(gr, 0)):
        with pytest.raises(khcore.KhcError) as e:
            call()
        assert e.value.code == khcore.KHC_EINVAL
    gr.close()


def test_hdeg_list_rejects_out_of_range_ids(ctx):
    import torch
    from paper_2006_03372_amd import khcore
    g = synth.chung_lu(500, 6.0, 2.5, seed=3)
    gr = ctx.graph(g)
    verts = torch.tensor([3, 7, g.n, 11], dtype=torch.int32, device="cuda")
    with pytest.raises(khcore.KhcError) as e:
        ctx.hdeg_list(gr, 2, verts)
    assert e.value.code == khcore.KHC_EINVAL
    verts = torch.tensor([0, 0xFFFFFFFF - (1 << 32)], dtype=torch.int32, device="cuda")  # id 2^32 - 1
    with pytest.raises(khcore.KhcError):
        ctx.hdeg_list(gr, 2, verts)
    gr.close()


@pytest.mark.parametrize("h", [1, 2, 3])
def test_hdeg_list_with_repeated_vertices(ctx, h):
    """Repeated ids (within one 64-lane word and across words and batches)
    all get the exact h-degree, on a random live mask."""
    import torch
    g = synth.chung_lu(3000, 8.0, 2.5, seed=12)
    alive = synth.random_alive(g.n, 0.85, 4)
    rng = np.random.default_rng(h)
    base = rng.choice(g.n, size=300, replace=False).astype(np.uint32)
    verts = np.concatenate([base, base[:50], base[:50], rng.choice(base, size=5000)]).astype(np.uint32)
    gr = ctx.graph(g)
    for width in (1, 4, 32):
        from paper_2006_03372_amd import khcore
        ctx.set_option(khcore.OPT_MAX_WIDTH, width)
        d = ctx.hdeg_list(gr, h, torch.from_numpy(verts.view(np.int32)).cuda(),
                          alive=torch.from_numpy(alive).cuda())
        torch.cuda.synchronize()
        ref, _ = oracle.hdeg_list(g, h, verts, alive)
        got = d.cpu().numpy().view(np.uint32)
        assert (got == ref).all(), (width, np.flatnonzero(got != ref)[:10])
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    gr.close()


def test_decompose_batched_entry_point(ctx):
    """khcore_decompose_batched, called directly through the C ABI on packed
    arrays, gives every graph the oracle's core numbers and rounds."""
    import torch
    from paper_2006_03372_amd import khcore
    parts = [synth.chung_lu(n, m, 2.5, seed=s) for n, m, s in ((400, 5.0, 41), (900, 8.0, 42), (250, 4.0, 43))]
    parts.append(synth.star(40))
    vb = np.zeros(len(parts) + 1, np.uint64)
    np.cumsum([p.n for p in parts], out=vb[1:])
    arc = np.zeros(len(parts) + 1, np.uint64)
    np.cumsum([p.nnz for p in parts], out=arc[1:])
    rp = np.concatenate([p.row_ptr[:-1].astype(np.uint64) + arc[i] for i, p in enumerate(parts)] + [arc[-1:]])
    col = np.concatenate([p.col for p in parts]).astype(np.uint32)
    vb_d, rp_d, col_d = _dev(vb, np.uint64), _dev(rp, np.uint64), _dev(col, np.uint32)
    total = int(vb[-1])
    for h in (2, 3):
        core = torch.zeros(total, dtype=torch.int32, device="cuda")
        rnd = torch.zeros(total, dtype=torch.int32, device="cuda")
        st = khcore.Stats()
        rc = ctx.lib.khcore_decompose_batched(ctx.handle, len(parts), ctypes.c_void_p(vb_d.data_ptr()),
                                              ctypes.c_void_p(rp_d.data_ptr()), ctypes.c_void_p(col_d.data_ptr()),
                                              int(arc[-1]), h, ctypes.c_void_p(core.data_ptr()),
                                              ctypes.c_void_p(rnd.data_ptr()), ctypes.byref(st))
        assert rc == 0, ctx.lib.khc_last_error(ctx.handle)
        c = core.cpu().numpy().view(np.uint32)
        r = rnd.cpu().numpy().view(np.uint32)
        for i, p in enumerate(parts):
            c_ref, r_ref = oracle.peel(p, h)
            assert (c[vb[i]:vb[i + 1]] == c_ref).all(), (h, i)
            assert (r[vb[i]:vb[i + 1]] == r_ref).all(), (h, i)
    # a column id outside its own graph is refused
    bad = col.copy()
    bad[int(arc[1])] = parts[1].n + 5
    bad_d = _dev(bad, np.uint32)
    core = torch.zeros(total, dtype=torch.int32, device="cuda")
    rc = ctx.lib.khcore_decompose_batched(ctx.handle, len(parts), ctypes.c_void_p(vb_d.data_ptr()),
                                          ctypes.c_void_p(rp_d.data_ptr()), ctypes.c_void_p(bad_d.data_ptr()),
                                          int(arc[-1]), 2, ctypes.c_void_p(core.data_ptr()), None, None)
    assert rc == khcore.KHC_EGRAPH
