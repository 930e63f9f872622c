"""GPU: round-limited decompositions and the width / waves-per-CU autotuner."""
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


@pytest.mark.parametrize("driver", [0, 1])
def test_round_limit_is_a_prefix(ctx, driver):
    """Cut after R rounds: the vertices removed in rounds < R have their
    final core numbers, the others 0."""
    from paper_2006_03372_amd import khcore
    g = synth.chung_lu(2000, 10.0, 2.5, seed=1)
    c_ref, r_ref = oracle.peel(g, 2)
    ctx.set_option(khcore.OPT_DRIVER, driver)
    gr = ctx.graph(g)
    try:
        for R in (1, 7, 50):
            ctx.set_option(khcore.OPT_ROUND_LIMIT, R)
            c, r, st = ctx.core(gr, 2, with_round=True)
            c, r = _u32(c), _u32(r)
            done = r_ref < R
            assert st["rounds"] == R
            assert (c[done] == c_ref[done]).all()
            assert (c[~done] == 0).all()
            assert (r[done] == r_ref[done]).all()
    finally:
        ctx.set_option(khcore.OPT_ROUND_LIMIT, 0)
        ctx.set_option(khcore.OPT_DRIVER, 0)
        gr.close()


def test_autotune_single_graph(ctx):
    from paper_2006_03372_amd import khcore
    g = synth.chung_lu(2000, 10.0, 2.5, seed=1)
    gr = ctx.graph(g)
    t = ctx.autotune(gr, 3, rounds=16)
    print("tune", t, flush=True)
    assert not t["persistent"]
    assert len(t["trials"]) == 9
    best = min(t["trials"], key=lambda x: x[2])
    assert (t["width_words"], t["waves_per_cu"]) == best[:2]
    # the decomposition after tuning (full length) still matches the oracle
    c, r, st = ctx.core(gr, 3, with_round=True)
    gr.close()
    assert st["width_words"] == t["width_words"]
    c_ref, r_ref = oracle.peel(g, 3)
    assert (_u32(c) == c_ref).all() and (_u32(r) == r_ref).all()
    ctx.set_option(khcore.OPT_MAX_WIDTH, 16)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)


def test_autotune_batched(ctx):
    from paper_2006_03372_amd import khcore
    graphs = synth.batch_chung_lu(6, n_lo=300, n_hi=1500)
    bg = ctx.batch(graphs)
    t = ctx.autotune(bg, 3, rounds=8)
    print("tune", t, flush=True)
    assert t["persistent"] and len(t["trials"]) == 9
    c, r, st = ctx.core(bg, 3, with_round=True)
    bg.close()
    assert st["width_words"] == t["width_words"]
    c = _u32(c)
    off = 0
    for g in graphs:
        c_ref, _ = oracle.peel(g, 3)
        assert (c[off:off + g.n] == c_ref).all()
        off += g.n
    ctx.set_option(khcore.OPT_PERSIST_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)


def test_autotune_median_and_cache(ctx):
    """Each candidate is timed OPT_TUNE_REPEATS times (the median kept); a
    second graph of the same size class gets the cached choice without
    trials, and turning the cache off times again."""
    from paper_2006_03372_amd import khcore
    a = ctx.graph(synth.chung_lu(3000, 8.0, 2.5, seed=31))
    b = ctx.graph(synth.chung_lu(3000, 8.0, 2.5, seed=32))
    try:
        ctx.set_option(khcore.OPT_TUNE_REPEATS, 5)
        ta = ctx.autotune(a, 2, rounds=12)
        assert not ta["cached"] and ta["repeats"] == 5 and len(ta["trials"]) == 9
        best = min(ta["trials"], key=lambda x: x[2])
        assert (ta["width_words"], ta["waves_per_cu"]) == best[:2]
        # same vertex count, arc counts below the same power of two: cached
        assert a.n == b.n
        ctx.set_option(khcore.OPT_MAX_WIDTH, 1)
        tb = ctx.autotune(b, 2, rounds=12)
        assert tb["cached"] and tb["trials"] == []
        assert (tb["width_words"], tb["waves_per_cu"]) == (ta["width_words"], ta["waves_per_cu"])
        c, _, st = ctx.core(b, 2)
        assert st["width_words"] == ta["width_words"]
        # another h is another class
        assert not ctx.autotune(b, 3, rounds=12)["cached"]
        ctx.set_option(khcore.OPT_TUNE_CACHE, 0)
        assert not ctx.autotune(b, 2, rounds=12)["cached"]
    finally:
        ctx.set_option(khcore.OPT_TUNE_CACHE, 1)
        ctx.set_option(khcore.OPT_TUNE_REPEATS, 3)
        ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
        ctx.set_option(khcore.OPT_WAVES_PER_CU, 16)
        a.close()
        b.close()
