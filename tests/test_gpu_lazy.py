"""GPU parity of schedule 3 (KHC_OPT_SCHEDULE 3): the bounded schedule with
the (h-1)-degree bounds of the vertices near each removed set lowered by
the decrement bound instead of recomputed, and refreshed exactly whenever
the vertex's h-degree is recomputed.  Core numbers and removal rounds must
equal the oracle's bit for bit (the bounds stay valid lower bounds)."""
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
    c.set_option(khcore.OPT_MAX_WIDTH, 32)
    c.close()


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


CASES = [
    ("chung-lu 2000", lambda: synth.chung_lu(2000, 10.0, 2.5, seed=1), (2, 3, 4)),
    ("chung-lu 3000 mean 4", lambda: synth.chung_lu(3000, 4.0, 2.5, seed=8), (2, 3, 5)),
    ("r-mat 12", lambda: synth.rmat(12, 8, seed=2), (2, 3, 4)),
    ("torus 30x30", lambda: synth.torus(30, 30), (2, 3)),
]


@pytest.mark.parametrize("name,make,hs", CASES)
def test_lazy_schedule_matches_oracle(ctx, name, make, hs):
    from paper_2006_03372_amd import khcore
    g = make()
    gr = ctx.graph(g)
    ctx.set_option(khcore.OPT_SCHEDULE, 3)
    try:
        for h in hs:
            c_ref, r_ref = oracle.peel(g, h)
            for width in (1, 32):
                ctx.set_option(khcore.OPT_MAX_WIDTH, width)
                c, r, st = ctx.core(gr, h, with_round=True)
                print(f"{name} h={h} width={width}: {st['rounds']} rounds, {st['h_recomputes']} h-recomputes, "
                      f"{st['hm1_recomputes']} (h-1)-refreshes", flush=True)
                assert (_u32(c) == c_ref).all(), np.flatnonzero(_u32(c) != c_ref)[:10]
                assert (_u32(r) == r_ref).all()
    finally:
        ctx.set_option(khcore.OPT_SCHEDULE, 1)
        ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
        gr.close()


def test_lazy_schedule_at_scale_matches_bounded(ctx):
    """R-MAT-16 at h = 3 and 4: schedule 3 gives the bounded schedule's cores
    and rounds (both certified elsewhere against the oracle)."""
    from paper_2006_03372_amd import khcore
    g = synth.rmat(16, 8, seed=1)
    gr = ctx.graph(g)
    try:
        for h in (3, 4):
            ctx.set_option(khcore.OPT_SCHEDULE, 1)
            c1, r1, _ = ctx.core(gr, h, with_round=True)
            ctx.set_option(khcore.OPT_SCHEDULE, 3)
            c3, r3, st = ctx.core(gr, h, with_round=True)
            print(f"r-mat 16 h={h}: {st}", flush=True)
            assert (_u32(c1) == _u32(c3)).all() and (_u32(r1) == _u32(r3)).all()
    finally:
        ctx.set_option(khcore.OPT_SCHEDULE, 1)
        gr.close()
