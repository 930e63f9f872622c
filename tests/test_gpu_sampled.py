"""GPU parity of the sampling-based mode (Section IV-C) with the CPU
oracle: for a fixed vertex sample the mode is deterministic (exact sampled
counts, integer estimate), so core numbers and removal estimates must match
bit for bit; with every vertex sampled it is the exact decomposition."""
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _sample(n, rate, seed):
    return (np.random.default_rng(seed).random(n) < rate).astype(np.uint8)


CASES = [
    ("chung-lu 2000", lambda: synth.chung_lu(2000, 10.0, 2.5, seed=1), 2, 0.1),
    ("chung-lu 2000", lambda: synth.chung_lu(2000, 10.0, 2.5, seed=1), 3, 0.3),
    ("r-mat 12", lambda: synth.rmat(12, 8, seed=2), 2, 0.2),
    ("r-mat 12", lambda: synth.rmat(12, 8, seed=2), 3, 0.05),
    ("star 700", lambda: synth.star(700), 2, 0.1),
    ("r-mat 12", lambda: synth.rmat(12, 8, seed=2), 1, 0.1),
    ("chung-lu 3000 mean 4", lambda: synth.chung_lu(3000, 4.0, 2.5, seed=8), 2, 0.02),
    ("chung-lu 3000 mean 4", lambda: synth.chung_lu(3000, 4.0, 2.5, seed=8), 4, 0.02),
]


@pytest.mark.parametrize("name,make,h,rate", CASES)
def test_sampled_matches_oracle(ctx, name, make, h, rate):
    import torch
    from paper_2006_03372_amd import khcore
    g = make()
    s = _sample(g.n, rate, 11)
    gr = ctx.graph(g)
    for width in (4, 32):
        ctx.set_option(khcore.OPT_MAX_WIDTH, width)
        c, est, st = ctx.core_sampled(gr, h, torch.from_numpy(s).cuda(), with_estimate=True)
        c_ref, est_ref = oracle.peel_sampled(g, h, s)
        print(f"{name} h={h} rate={rate} width={width}: {st['rounds']} rounds", flush=True)
        assert (_u32(c) == c_ref).all(), np.flatnonzero(_u32(c) != c_ref)[:10]
        assert (_u32(est) == est_ref).all()
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    gr.close()


def test_everything_sampled_is_exact(ctx):
    import torch
    g = synth.chung_lu(1500, 8.0, 2.5, seed=5)
    gr = ctx.graph(g)
    c, _, _ = ctx.core_sampled(gr, 2, torch.ones(g.n, dtype=torch.uint8, device="cuda"))
    exact, _, _ = ctx.core(gr, 2)
    gr.close()
    assert (_u32(c) == _u32(exact)).all()
    assert (_u32(c) == oracle.peel(g, 2)[0]).all()


def test_sparse_sample_skips_recounts(ctx):
    """A vertex at distance j from the removed set can only lose sampled
    vertices within h - j hops of it: with a sparse sample most affected
    vertices keep their counts, and the result still equals the oracle's
    (which recounts every affected vertex)."""
    import torch
    g = synth.chung_lu(5000, 6.0, 2.5, seed=3)
    s = _sample(g.n, 0.03, 5)
    gr = ctx.graph(g)
    c, est, st = ctx.core_sampled(gr, 2, torch.from_numpy(s).cuda(), with_estimate=True)
    gr.close()
    c_ref, est_ref = oracle.peel_sampled(g, 2, s)
    assert (_u32(c) == c_ref).all() and (_u32(est) == est_ref).all()
    print(st, flush=True)
    # h_recomputes also counts the two initial passes over every vertex with a neighbour
    recounts = st["h_recomputes"] - 2 * int(np.count_nonzero(g.degrees()))
    assert 0 <= recounts < st["affected_total"] // 2, st
