"""GPU parity of the local-update schedule (KHC_OPT_SCHEDULE 2): rounds
whose region N^h[P] is small update the affected h-degrees inside it (the
set form of Section IV-A's update, two bounded BFS from the vertices within
h-1 hops of P, before and after removal), the others recompute; core
numbers and removal rounds must equal the oracle's bit for bit."""
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
    c.set_option(khcore.OPT_SCHEDULE, 1)
    c.close()


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


CASES = [
    ("chung-lu 2000", lambda: synth.chung_lu(2000, 10.0, 2.5, seed=1), (2, 3)),
    ("chung-lu 3000 mean 4", lambda: synth.chung_lu(3000, 4.0, 2.5, seed=8), (2, 3, 4)),
    ("r-mat 12", lambda: synth.rmat(12, 8, seed=2), (2, 3)),
    ("torus 30x30", lambda: synth.torus(30, 30), (1, 2, 3)),
    ("running example", lambda: synth.from_edges(14, *np.array(
        [(0, 1), (0, 2), (1, 3), (2, 5), (3, 4), (4, 5), (4, 6), (3, 7), (6, 7), (5, 8), (6, 8), (7, 9), (7, 10),
         (8, 9), (8, 12), (9, 10), (9, 11), (9, 12), (9, 13), (10, 11), (12, 13)]).T), (1, 2, 3)),
]


@pytest.mark.parametrize("name,make,hs", CASES)
def test_local_schedule_matches_oracle(ctx, name, make, hs):
    from paper_2006_03372_amd import khcore
    g = make()
    gr = ctx.graph(g)
    ctx.set_option(khcore.OPT_SCHEDULE, 2)
    ctx.set_option(khcore.OPT_DRIVER, 0)
    for h in hs:
        for width in (1, 32):
            ctx.set_option(khcore.OPT_MAX_WIDTH, width)
            c, r, st = ctx.core(gr, h, with_round=True)
            c_ref, r_ref = oracle.peel(g, h)
            print(f"{name} h={h} width={width}: {st['rounds']} rounds, {st['local_rounds']} local, "
                  f"{st['h_recomputes']} recomputes", flush=True)
            assert (_u32(c) == c_ref).all(), np.flatnonzero(_u32(c) != c_ref)[:10]
            assert (_u32(r) == r_ref).all()
    ctx.set_option(khcore.OPT_SCHEDULE, 1)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    gr.close()


def test_local_rounds_are_used(ctx):
    """On a sparse graph at h = 2 most rounds take the local update."""
    from paper_2006_03372_amd import khcore
    g = synth.chung_lu(5000, 4.0, 2.5, seed=21)
    gr = ctx.graph(g)
    ctx.set_option(khcore.OPT_SCHEDULE, 2)
    c, r, st = ctx.core(gr, 2, with_round=True)
    ctx.set_option(khcore.OPT_SCHEDULE, 1)
    gr.close()
    c_ref, r_ref = oracle.peel(g, 2)
    assert (_u32(c) == c_ref).all() and (_u32(r) == r_ref).all()
    assert st["local_rounds"] > st["rounds"] // 4, st
