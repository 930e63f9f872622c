"""GPU tests of the learned recompute gate (khcore_decompose_gated): its
features against values computed here from the oracle's h-degrees; without
a network, or with margin 1, the exact core numbers and removal rounds of
the oracle bit for bit; with any network, core numbers never below the exact
ones (a vertex leaves only when an exact or stale h-degree is at most the
level, so no member of a (k,h)-core leaves below k); and with a trained
network fewer recomputes than the exact schedule."""
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


def _gate_reference(g, h, alive, dm):
    live = alive.astype(bool)
    n_live = int(live.sum())
    deg_full = np.diff(g.row_ptr).astype(np.float64)
    X = np.zeros((g.n, 8))
    for v in range(g.n):
        if not live[v]:
            continue
        nb = np.array([w for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if live[w]], dtype=np.int64)
        f = np.zeros(8)
        f[0] = nb.size
        f[1] = dm[v]
        if nb.size:
            c = dm[nb].astype(np.float64)
            f[2], f[3], f[4] = c.min(), c.mean(), c.max()
            f[5] = deg_full[nb].mean()
            f[6] = min(n_live - 1, c.sum())
        else:
            f[6] = 0.0
        f[7] = n_live - 1
        X[v] = np.log1p(f) / 8.0
    return X


@pytest.mark.parametrize("h", [2, 3, 4])
def test_gate_features_match_reference(ctx, h):
    import torch
    g = synth.chung_lu(1500, 8.0, 2.5, seed=4)
    alive = synth.random_alive(g.n, 0.8, 9)
    dm = oracle.hdeg(g, h - 1, alive).astype(np.uint32)
    gr = ctx.graph(g)
    a = torch.from_numpy(alive).cuda()
    X = ctx.gate_features(gr, h, torch.from_numpy(dm.view(np.int32)).cuda(), a).cpu().numpy()
    # arbitrary lower bounds work the same way
    lowered = (dm // 2).astype(np.uint32)
    X2 = ctx.gate_features(gr, h, torch.from_numpy(lowered.view(np.int32)).cuda(), a).cpu().numpy()
    gr.close()
    assert np.allclose(X, _gate_reference(g, h, alive, dm), rtol=1e-5, atol=1e-6)
    assert np.allclose(X2, _gate_reference(g, h, alive, lowered), rtol=1e-5, atol=1e-6)


CASES = [
    ("chung-lu 2000", lambda: synth.chung_lu(2000, 10.0, 2.5, seed=1), (2, 3)),
    ("r-mat 12", lambda: synth.rmat(12, 8, seed=2), (2, 3, 4)),
    ("torus 20x20", lambda: synth.torus(20, 20), (2, 3)),
]


@pytest.mark.parametrize("name,make,hs", CASES)
def test_gate_without_network_is_exact(ctx, name, make, hs):
    g = make()
    gr = ctx.graph(g)
    net = ctx.mlp(seed=3)
    for h in hs:
        c_ref, r_ref = oracle.peel(g, h)
        c, r, st = ctx.core_gated(gr, h, None, 0.0, with_round=True)
        assert (_u32(c) == c_ref).all() and (_u32(r) == r_ref).all()
        assert st["gate_deferrals"] == 0
        # margin 1 puts every soft key at the lower bound: nothing is deferred
        c, r, st = ctx.core_gated(gr, h, net, 1.0, with_round=True)
        assert (_u32(c) == c_ref).all() and (_u32(r) == r_ref).all()
        assert st["gate_deferrals"] == 0
    net.close()
    gr.close()


@pytest.mark.parametrize("h", [2, 3])
def test_gate_never_below_exact(ctx, h):
    """Any network, even an untrained one: core numbers at least the exact."""
    g = synth.chung_lu(3000, 6.0, 2.5, seed=12)
    gr = ctx.graph(g)
    c_ref, _ = oracle.peel(g, h)
    for seed, margin in ((1, 0.0), (2, 0.3)):
        net = ctx.mlp(seed=seed)
        c, _, st = ctx.core_gated(gr, h, net, margin)
        net.close()
        print(f"h={h} seed={seed} margin={margin}: {st['gate_deferrals']} deferrals", flush=True)
        assert (_u32(c) >= c_ref).all()
    gr.close()


@pytest.mark.parametrize("h", [2, 3])
def test_trained_gate_saves_recomputes(ctx, h):
    """Trained on peeling states of small Chung-Lu graphs, the gate defers
    recomputes on an unseen graph of the family and the run needs fewer of
    them than the exact schedule.  Deferred vertices mostly come back for
    their recompute once the level nears them, so the saving is small
    (measured 19,429 -> 17,704 at h = 2 and 23,609 -> 21,725 at h = 3).  The
    exact fraction has no guarantee (the deferrals rest on estimates); it
    measured 0.997 at h = 2 and 0.866 at h = 3 on this graph at margin 0.2,
    and 0.8 only guards against a gate that defers blindly."""
    from paper_2006_03372_amd import learned
    train = [synth.chung_lu(3000, 6.0, 2.5, 300 + i) for i in range(6)]
    X, t = learned.gate_training_set(ctx, train, h)
    net = ctx.mlp(seed=7)
    losses = net.train(X, t, epochs=25, batch=2048, lr=2e-3, seed=1)
    assert losses[-1] < 0.05 * losses[0]
    g = synth.chung_lu(6000, 6.0, 2.5, seed=1)
    gr = ctx.graph(g)
    exact, _, st_e = ctx.core(gr, h)
    c, _, st = ctx.core_gated(gr, h, net, 0.2)
    gr.close()
    net.close()
    e, c = _u32(exact), _u32(c)
    acc = learned.accuracy(e, c)
    print(f"h={h}: exact {st_e['h_recomputes']} recomputes; gated {st['h_recomputes']} recomputes, "
          f"{st['gate_deferrals']} deferrals, {acc}", flush=True)
    assert (c >= e).all()
    assert st["gate_deferrals"] > 0
    assert st["h_recomputes"] < st_e["h_recomputes"]
    assert acc["exact_fraction"] >= 0.8
