"""GPU learned mode: MLP forward and backward against the reference
(bf16 contract), training, features against the CPU oracle, and the gain of
the trained network over the bound-only estimator."""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
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


def _rand_params(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, scale, size=omlp.N_PARAMS)
    return p.astype(np.float32)


@pytest.mark.parametrize("n", [16, 1000, 4099])
def test_forward_matches_reference(ctx, n):
    import torch
    net = ctx.mlp(seed=1)
    p = _rand_params(n)
    net.set(p)
    X = np.random.default_rng(n + 1).uniform(0.0, 1.6, size=(n, 8)).astype(np.float32)
    y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    ref, _ = omlp.forward(p, X, exact=False)
    err = np.abs(y - ref)
    print(f"forward n={n}: max err {err.max():.3e} mean {err.mean():.3e}", flush=True)
    assert err.max() <= 2e-2 * (1.0 + np.abs(ref).max())
    assert err.mean() <= 2e-3 * (1.0 + np.abs(ref).mean())
    net.close()


def test_backward_matches_reference(ctx):
    """Element-wise against the bf16 contract (itself pinned on a hand-built
    chain and, in float64, to finite differences).  Both sides round the
    same values to bf16; they differ only in how float32 (GPU, MFMA) and
    float64 (oracle) sum the products, at most a few units of 2^-24 of the
    sum of |terms| per element, well inside 1e-5 of the largest entry."""
    import torch
    net = ctx.mlp(seed=2)
    p = _rand_params(7)
    net.set(p)
    rng = np.random.default_rng(8)
    n = 777
    X = rng.uniform(0.0, 1.6, size=(n, 8)).astype(np.float32)
    t = rng.uniform(0.0, 1.5, size=n).astype(np.float32)
    loss = net.gradient(torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda())
    _, g = net.get()
    g_ref = omlp.backward(p, X, t, exact=False)
    l_ref = float(np.mean((omlp.forward(p, X, exact=False)[0] - t) ** 2))
    err = np.abs(g.astype(np.float64) - g_ref)
    scale = np.abs(g_ref).max()
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"backward: loss {loss:.8f} vs {l_ref:.8f}, norm error {rel:.3e}, "
          f"max element error {err.max() / scale:.3e} of the largest entry", flush=True)
    assert abs(loss - l_ref) <= 1e-5 * max(l_ref, 1e-6)
    assert (err <= 1e-5 * scale + 1e-4 * np.abs(g_ref)).all(), np.argsort(-err)[:8]
    # the bf16 contract stays close to the exact float64 gradient, which is
    # itself pinned to finite differences on the CPU
    g64 = omlp.backward(p, X, t, exact=True)
    assert np.linalg.norm(g - g64) / np.linalg.norm(g64) < 8e-2
    net.close()


def test_adam_steps_match_reference(ctx):
    """Two khc_mlp_train steps (one full-batch minibatch per epoch) against
    the float64 Adam of Kingma and Ba, element by element: moments and
    parameters.  The gradient of each step is read with khc_mlp_gradient at
    the same parameters (the training pass sums the same rows in another
    order, a float32 difference far below the tolerances)."""
    import torch
    rng = np.random.default_rng(31)
    n, lr = 3000, 1e-2
    X = torch.from_numpy(rng.uniform(0.0, 1.6, size=(n, 8)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.uniform(0.0, 1.5, size=n).astype(np.float32)).cuda()
    net = ctx.mlp(seed=4)
    p0 = _rand_params(32)
    net.set(p0)
    m_prev = np.zeros(omlp.N_PARAMS)
    v_prev = np.zeros(omlp.N_PARAMS)
    p_prev = p0.astype(np.float64)
    for step in (1, 2):
        net.gradient(X, t)
        _, g = net.get()
        g = g.astype(np.float64)
        net.train(X, t, epochs=1, batch=n, lr=lr, seed=step)
        p, _ = net.get()
        m, v, k = net.moments()
        assert k == step
        p_ref, m_ref, v_ref = omlp.adam_step(p_prev, g, m_prev, v_prev, step, lr)
        gs = np.abs(g).max()
        assert np.allclose(m, m_ref, rtol=1e-4, atol=1e-6 * gs)
        assert np.allclose(v, v_ref, rtol=1e-4, atol=1e-6 * gs * gs)
        # where |g| is far above eps the update is insensitive to the summation order
        big = np.abs(g) > 1e-3 * gs
        assert big.sum() > 1000
        assert np.allclose(p[big], p_ref[big], rtol=1e-6, atol=1e-5 * lr)
        # Adam moves a parameter by at most lr * |m^| / sqrt(v^), which is 1 at
        # the first step and at most 1.0014 at the second (Cauchy-Schwarz)
        assert (np.abs(p - p_prev) <= lr * 1.0015 + 1e-6).all()
        print(f"adam step {step}: max |dp - dp_ref| {np.abs(p[big] - p_ref[big]).max():.3e}", flush=True)
        p_prev, m_prev, v_prev = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    net.close()


def test_training_reduces_loss(ctx):
    import torch
    teacher = _rand_params(11, 0.3)
    rng = np.random.default_rng(12)
    X = rng.uniform(0.0, 1.6, size=(20000, 8)).astype(np.float32)
    t, _ = omlp.forward(teacher, X, exact=True)
    net = ctx.mlp(seed=3)
    losses = net.train(torch.from_numpy(X).cuda(), torch.from_numpy(t.astype(np.float32)).cuda(),
                       epochs=12, batch=1024, lr=3e-3, seed=5)
    print("epoch losses", losses, flush=True)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.2 * losses[0]
    net.close()


@pytest.mark.parametrize("h", [2, 3, 4])
def test_features_match_oracle(ctx, h):
    import torch
    g = synth.chung_lu(1500, 8.0, 2.5, seed=4)
    alive = synth.random_alive(g.n, 0.8, 9)
    gr = ctx.graph(g)
    X, lb, ub = ctx.features(gr, h, torch.from_numpy(alive).cuda())
    X = X.cpu().numpy()
    lb = lb.cpu().numpy().view(np.uint32)
    ub = ub.cpu().numpy().view(np.uint32)
    gr.close()
    a, b = max(1, h - 3), max(1, h - 2)
    dj = {j: oracle.hdeg(g, j, alive).astype(np.float64) for j in sorted({a, b, h - 1})}
    live = alive.astype(bool)
    n_live = int(live.sum())
    for v in range(g.n):
        if not live[v]:
            assert not X[v].any() and lb[v] == 0 and ub[v] == 0
            continue
        nb = [w for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if live[w]]
        c = dj[h - 1][nb] if nb else np.zeros(0)
        f = [dj[a][v], dj[b][v], dj[h - 1][v]]
        if nb:
            f += [c.min(), c.mean(), c.max(), dj[a][nb].mean(), dj[b][nb].mean()]
        else:
            f += [0.0] * 5
        ref = np.log1p(np.array(f)) / 8.0
        assert np.allclose(X[v], ref, rtol=1e-5, atol=1e-6), (v, X[v], ref)
        assert lb[v] == int(max(dj[h - 1][v], c.max() if nb else 0))
        assert ub[v] == max(int(lb[v]), int(min(n_live - 1, c.sum())))


@pytest.mark.parametrize("kind", [0, 1])
def test_mlp_samples_match_host(ctx, kind):
    """khc_mlp_samples: the features of the live vertices in vertex order
    (rows of khc_features / khc_gate_features) and log1p of the oracle's
    h-degree over 8; khc_alive_after against numpy."""
    import torch
    g = synth.chung_lu(2500, 8.0, 2.5, seed=14)
    h = 3
    alive = synth.random_alive(g.n, 0.7, 5)
    a = torch.from_numpy(alive).cuda()
    gr = ctx.graph(g)
    X, t = ctx.mlp_samples(gr, h, a, kind=kind)
    if kind == 0:
        Xall, _, _ = ctx.features(gr, h, a)
    else:
        dm = oracle.hdeg(g, h - 1, alive).astype(np.uint32)
        Xall = ctx.gate_features(gr, h, torch.from_numpy(dm.view(np.int32)).cuda(), a)
    rnd = np.random.default_rng(3).integers(0, 50, size=g.n).astype(np.uint32)
    got = ctx.alive_after(torch.from_numpy(rnd.view(np.int32)).cuda(), 17).cpu().numpy()
    gr.close()
    live = np.flatnonzero(alive)
    assert X.shape == (live.size, 8) and t.shape == (live.size,)
    assert np.array_equal(X.cpu().numpy(), Xall.cpu().numpy()[live])
    d = oracle.hdeg(g, h, alive).astype(np.float64)[live]
    assert np.allclose(t.cpu().numpy(), (np.log1p(d) / 8.0).astype(np.float32), rtol=2e-7, atol=0)
    assert np.array_equal(got, (rnd >= 17).astype(np.uint8))


def test_bounds_bracket_exact_degree(ctx):
    import torch
    g = synth.rmat(11, 8, seed=6)
    for h in (2, 3, 4):
        gr = ctx.graph(g)
        _, lb, ub = ctx.features(gr, h)
        d = ctx.hdeg(gr, h)
        gr.close()
        lb, ub, d = (t.cpu().numpy().view(np.uint32) for t in (lb, ub, d))
        assert (lb <= d).all() and (d <= ub).all()


@pytest.mark.parametrize("h", [2, 4])
def test_learned_mode_beats_bounds_only(ctx, h):
    """Train on exact h-degrees of peeling states of small Chung-Lu graphs,
    then peel an unseen graph of the same family: the network must give
    more exact core numbers and a smaller error than the estimator that uses
    the exact lower bound alone (the method without the network)."""
    from paper_2006_03372_amd import learned
    train_graphs = [synth.chung_lu(3000, 6.0, 2.5, 200 + i) for i in range(6)]
    X, t = learned.training_set(ctx, train_graphs, h)
    net = ctx.mlp(seed=7)
    losses = net.train(X, t, epochs=25, batch=2048, lr=2e-3, seed=1)
    print("training samples", X.shape[0], "losses", losses[[0, -1]], flush=True)
    # pooled over three unseen graphs of the same family
    e, cl, cb = [], [], []
    for seed in (1, 2, 3):
        gr = ctx.graph(synth.chung_lu(3000, 6.0, 2.5, seed))
        exact, _, _ = ctx.core(gr, h)
        learned_core, _, st = ctx.core_approx(gr, h, net)
        bound_core, _, _ = ctx.core_approx(gr, h, None)
        gr.close()
        e.append(exact.cpu().numpy().view(np.uint32))
        cl.append(learned_core.cpu().numpy().view(np.uint32))
        cb.append(bound_core.cpu().numpy().view(np.uint32))
    e, cl, cb = np.concatenate(e), np.concatenate(cl), np.concatenate(cb)
    acc_l = learned.accuracy(e, cl)
    acc_b = learned.accuracy(e, cb)
    print("learned", acc_l, "bounds only", acc_b, flush=True)
    assert losses[-1] < 0.05 * losses[0]
    assert acc_l["exact_fraction"] >= acc_b["exact_fraction"]
    # The gain depends on how loose the exact bounds are.  At h = 2 they are
    # loose and the network cuts the bound-only MAE to about an eighth
    # (measured 0.67 against 5.4); at h = 4 four hops reach most of these
    # graphs, the lower bound is nearly tight and the network's gain is
    # small (measured 8.88 against 11.11, a ratio of 0.80).  Each margin
    # keeps headroom above its measured ratio.
    assert acc_l["mae"] < {2: 0.3, 4: 0.9}[h] * acc_b["mae"]
    assert acc_l["precision"] > acc_b["precision"]
    net.close()


def test_network_on_rmat_h4(ctx):
    """On the R-MAT family at h = 4 the exact lower bound is nearly tight, so
    the approximate mode's clamped estimate mostly equals it and the network
    cannot gain there.  The network itself is still not degenerate: trained
    on small R-MAT graphs, its raw estimates on an unseen one differ from the
    lower bound on most vertices and track the exact 4-hop degree."""
    import torch
    from paper_2006_03372_amd import learned
    train = [synth.rmat(11, 8, seed=400 + i) for i in range(6)]
    X, t = learned.training_set(ctx, train, 4)
    net = ctx.mlp(seed=7)
    net.train(X, t, epochs=25, batch=2048, lr=2e-3, seed=1)
    g = synth.rmat(11, 8, seed=1)
    gr = ctx.graph(g)
    Xt, lb, ub = ctx.features(gr, 4)
    d = ctx.hdeg(gr, 4)
    y = net.forward(Xt)
    gr.close()
    net.close()
    est = np.expm1(8.0 * y.cpu().numpy().astype(np.float64))
    lb, ub, d = (a.cpu().numpy().view(np.uint32).astype(np.float64) for a in (lb, ub, d))
    live = d > 0
    rel_net = np.abs(est[live] - d[live]) / d[live]
    rel_lb = (d[live] - lb[live]) / d[live]
    clamped_at_lb = np.mean(np.clip(np.rint(est[live]), lb[live], ub[live]) == lb[live])
    print(f"median relative error: network {np.median(rel_net):.4f}, lower bound {np.median(rel_lb):.4f}; "
          f"clamped estimate at the lower bound on {clamped_at_lb:.3f} of vertices", flush=True)
    assert np.mean(np.rint(est[live]) != lb[live]) > 0.5
    assert np.median(rel_net) < 0.1


def test_training_is_reproducible(ctx):
    """Gradients are summed in a fixed order, so two runs from the same seeds
    end with the same parameters bit for bit."""
    import torch
    rng = np.random.default_rng(21)
    X = torch.from_numpy(rng.uniform(0.0, 1.6, size=(30000, 8)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.uniform(0.0, 1.5, size=30000).astype(np.float32)).cuda()
    out = []
    for _ in range(2):
        net = ctx.mlp(seed=9)
        losses = net.train(X, t, epochs=3, batch=4096, lr=1e-3, seed=4)
        p, _ = net.get()
        out.append((losses, p))
        net.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1].view(np.uint32), out[1][1].view(np.uint32))


def test_approx_without_network_is_valid(ctx):
    """With the bound-only estimator every vertex still gets a core number no
    larger than its initial bound and the removal levels never decrease."""
    g = synth.rmat(11, 8, seed=3)
    gr = ctx.graph(g)
    core, est, st = ctx.core_approx(gr, 3, None, with_estimate=True)
    _, lb, ub = ctx.features(gr, 3)
    gr.close()
    c = core.cpu().numpy().view(np.uint32)
    assert (c <= ub.cpu().numpy().view(np.uint32)).all()
    assert st["rounds"] >= 1


def test_save_and_load(ctx, tmp_path):
    import torch
    from paper_2006_03372_amd import khcore
    a = ctx.mlp(seed=5)
    a.set(_rand_params(3))
    path = str(tmp_path / "net.bin")
    a.save(path)
    b = ctx.mlp(seed=6)
    b.load(path)
    pa, _ = a.get()
    pb, _ = b.get()
    assert np.array_equal(pa.view(np.uint32), pb.view(np.uint32))
    X = torch.from_numpy(np.random.default_rng(2).uniform(0, 1.6, size=(300, 8)).astype(np.float32)).cuda()
    assert torch.equal(a.forward(X), b.forward(X))
    # a truncated file is refused and leaves the network as it was
    with open(path, "rb") as f:
        blob = f.read()
    with open(path, "wb") as f:
        f.write(blob[:-4])
    with pytest.raises(khcore.KhcError):
        b.load(path)
    pb2, _ = b.get()
    assert np.array_equal(pb.view(np.uint32), pb2.view(np.uint32))
    a.close()
    b.close()
