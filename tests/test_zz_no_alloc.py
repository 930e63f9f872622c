"""khdeg_compute_noalloc (the entry point for callers that cannot allocate)
against khdeg_compute, bit for bit, on two calls in a row, the second on a
smaller input; a graph beyond the static scratch is refused with
KHC_ENOMEM."""
import numpy as np
import pytest

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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_noalloc_matches_khdeg_compute_twice(ctx):
    import torch
    big = synth.rmat(16, 8, seed=3)
    small = synth.chung_lu(2000, 10.0, 2.5, seed=1)
    alive = torch.from_numpy(synth.random_alive(small.n, 0.8, 5)).cuda()
    cases = [(big, 3, None), (small, 2, alive)]
    for g, h, a in cases:
        gr = ctx.graph(g)
        print(f"noalloc n={g.n} nnz={g.nnz} h={h} alive={'mask' if a is not None else 'all'}", flush=True)
        ref = _u32(ctx.hdeg(gr, h, alive=a))
        out = torch.full((g.n,), -1, dtype=torch.int32, device="cuda")
        ctx.hdeg_noalloc(gr, h, alive=a, out=out)
        torch.cuda.synchronize()
        got = _u32(out)
        assert (got == ref).all(), np.flatnonzero(got != ref)[:10]
        gr.close()


def test_noalloc_rejects_graph_beyond_scratch(ctx):
    from paper_2006_03372_amd import khcore
    g = synth.path(1 << 20)
    gr = ctx.graph(g)
    with pytest.raises(khcore.KhcError) as e:
        ctx.hdeg_noalloc(gr, 3)
    assert e.value.code == khcore.KHC_ENOMEM
    gr.close()
