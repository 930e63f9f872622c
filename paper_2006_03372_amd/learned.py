"""Learned approximate mode: training data, training and evaluation.

Training samples come from the method itself: for each training graph the
exact GPU peeling gives, for every vertex, the round it is removed in; the
graph induced by the vertices still present after round r (khc_alive_after)
is a state the approximate driver will meet.  For several such states the
library computes, on the device, the eight features of every live vertex
and the regression target log1p(d^h) / 8 from its exact h-degree
(khc_mlp_samples).  Training runs on the GPU (khc_mlp_train).  Accuracy is judged against exact core numbers: the
fraction of vertices with the exact core, the mean absolute error, and the
precision of the paper's Section V (Exp-4), 1 - mean over v of
|c(v) - c^(v)| / c(v), taken over vertices whose exact core is not 0.

The learned recompute gate (khcore_decompose_gated) trains the same network
on other inputs: the gate features (khc_gate_features) built from the exact
(h-1)-degrees of each state, with the same targets.  Its evaluation runs the
exact bounded schedule and the gated one at several margins and reports the
time, the recomputes the gate saved and the accuracy.
"""
from __future__ import annotations

import numpy as np

FEATURE_SCALE = 8.0


def _torch():
    import torch
    return torch


def states_of(ctx, gr, h, fractions=(0.0, 0.2, 0.4, 0.6, 0.8)):
    """Alive masks (device uint8) after the given fractions of the exact
    peeling rounds, plus the exact decomposition (core, round)."""
    core, rnd, st = ctx.core(gr, h, with_round=True)
    rounds = int(st["rounds"])
    masks = [ctx.alive_after(rnd, int(f * rounds)) for f in fractions]
    return masks, core, rnd


def samples(ctx, gr, h, masks):
    """Features and targets of the live vertices of every state (built by
    khc_mlp_samples on the device)."""
    torch = _torch()
    xs, ts = zip(*(ctx.mlp_samples(gr, h, m, kind=0) for m in masks))
    return torch.cat(xs), torch.cat(ts)


def gate_samples(ctx, gr, h, masks):
    """Gate features and targets of the live vertices of every state (built
    by khc_mlp_samples on the device)."""
    torch = _torch()
    xs, ts = zip(*(ctx.mlp_samples(gr, h, m, kind=1) for m in masks))
    return torch.cat(xs), torch.cat(ts)


def gate_training_set(ctx, graphs, h, fractions=(0.0, 0.2, 0.4, 0.6, 0.8)):
    torch = _torch()
    xs, ts = [], []
    for g in graphs:
        gr = ctx.graph(g)
        masks, _, _ = states_of(ctx, gr, h, fractions)
        X, t = gate_samples(ctx, gr, h, masks)
        xs.append(X)
        ts.append(t)
        gr.close()
    return torch.cat(xs).contiguous(), torch.cat(ts).contiguous()


def training_set(ctx, graphs, h, fractions=(0.0, 0.2, 0.4, 0.6, 0.8)):
    torch = _torch()
    xs, ts = [], []
    for g in graphs:
        gr = ctx.graph(g)
        masks, _, _ = states_of(ctx, gr, h, fractions)
        X, t = samples(ctx, gr, h, masks)
        xs.append(X)
        ts.append(t)
        gr.close()
    return torch.cat(xs).contiguous(), torch.cat(ts).contiguous()


def accuracy(core_exact, core_approx):
    """Fraction exact, mean absolute error, paper precision (core 0 left out)."""
    c = np.asarray(core_exact, dtype=np.int64)
    a = np.asarray(core_approx, dtype=np.int64)
    err = np.abs(c - a)
    nz = c > 0
    prec = 1.0 - float(np.mean(err[nz] / c[nz])) if nz.any() else 1.0
    return {"exact_fraction": float(np.mean(err == 0)), "mae": float(np.mean(err)), "precision": prec}


def evaluate(h=4, train_scale=16, train_edge_factor=8, train_count=32, train_seed=101, test_scale=18,
             test_edge_factor=8, epochs=10, batch=4096, lr=2e-3, log=print, family="rmat", train_n=20000,
             test_n=200000, mean_degree=8.0, sampling_rates=(0.05, 0.1, 0.2)):
    """Train the network on small graphs of one family and peel a larger one
    exactly, with the network, with the lower bound alone, with an
    untrained network and with the sampling mode at each rate; returns
    times and accuracies.  family "rmat": R-MAT
    graphs of train_scale / test_scale; "chung-lu": Chung-Lu graphs (beta
    2.5, mean_degree) of train_n / test_n vertices."""
    import time
    from . import khcore, synth
    torch = _torch()
    ctx = khcore.Context(0)
    ctx.set_option(khcore.OPT_MAX_WIDTH, 32)
    ctx.set_option(khcore.OPT_WAVES_PER_CU, 8)
    t0 = time.time()
    if family == "rmat":
        graphs = (synth.rmat(train_scale, train_edge_factor, seed=train_seed + i) for i in range(train_count))
        train_desc = f"R-MAT scale {train_scale} ef {train_edge_factor}"
    else:
        graphs = (synth.chung_lu(train_n, mean_degree, 2.5, train_seed + i) for i in range(train_count))
        train_desc = f"Chung-Lu n={train_n} mean {mean_degree} beta 2.5"
    xs, ts = [], []
    for i, g in enumerate(graphs):
        gr = ctx.graph(g)
        masks, _, _ = states_of(ctx, gr, h)
        X, t = samples(ctx, gr, h, masks)
        xs.append(X)
        ts.append(t)
        gr.close()
        log(f"training graph {i + 1}/{train_count}: {X.shape[0]} samples ({time.time() - t0:.0f} s)")
    X, t = torch.cat(xs).contiguous(), torch.cat(ts).contiguous()
    del xs, ts
    net = ctx.mlp(seed=7)
    t1 = time.time()
    losses = net.train(X, t, epochs=epochs, batch=batch, lr=lr, seed=1)
    torch.cuda.synchronize()
    out = {"h": h, "train": {"graphs": f"{train_desc}, seeds {train_seed}..{train_seed + train_count - 1}",
                             "samples": int(X.shape[0]), "epochs": epochs, "seconds": round(time.time() - t1, 2),
                             "loss_first": float(losses[0]), "loss_last": float(losses[-1])}}
    del X, t
    if family == "rmat":
        g = synth.rmat(test_scale, test_edge_factor, seed=1)
        test_desc = f"R-MAT scale {test_scale} ef {test_edge_factor}, seed 1"
    else:
        g = synth.chung_lu(test_n, mean_degree, 2.5, 1)
        test_desc = f"Chung-Lu n={test_n} mean {mean_degree} beta 2.5, seed 1"
    gr = ctx.graph(g)
    out["test"] = {"graph": test_desc, "n": g.n, "edges": g.num_edges}

    def run(name, fn):
        t2 = time.time()
        ctx.set_progress(lambda r, removed, level: log(f"  {name}: {time.time() - t2:.0f} s, round {r}, "
                                                        f"{removed} removed"), 20000)
        core, st = fn()
        torch.cuda.synchronize()
        ctx.set_progress(None)
        return core.cpu().numpy().view(np.uint32), st, time.time() - t2

    exact, st, te = run("exact", lambda: ctx.core(gr, h)[::2])
    out["exact"] = {"seconds": round(te, 2), "rounds": st["rounds"], "h_recomputes": st["h_recomputes"]}
    untrained = ctx.mlp(seed=7)
    for name, m in (("learned", net), ("lower_bound_only", None), ("untrained", untrained)):
        core, st, ta = run(name, lambda: ctx.core_approx(gr, h, m)[::2])
        out[name] = {"seconds": round(ta, 2), "rounds": st["rounds"], "speedup_vs_exact": round(te / ta, 3),
                     **accuracy(exact, core)}
        log(f"{name}: {out[name]}")
    # the paper's own approximate variant beside it: the sampling mode at
    # several rates, each on a vertex sample drawn here from a fixed seed
    for rate in sampling_rates:
        mask = torch.from_numpy((np.random.default_rng(12345).random(g.n) < rate).astype(np.uint8)).cuda()
        core, st, ta = run(f"sampling r={rate}", lambda: ctx.core_sampled(gr, h, mask)[::2])
        out[f"sampling_r{rate}"] = {"seconds": round(ta, 2), "rounds": st["rounds"],
                                    "speedup_vs_exact": round(te / ta, 3), **accuracy(exact, core)}
        log(f"sampling r={rate}: {out[f'sampling_r{rate}']}")
    gr.close()
    ctx.close()
    return out


def evaluate_gate(h=4, train_scale=16, train_edge_factor=8, train_count=32, train_seed=101, test_scale=18,
                  test_edge_factor=8, epochs=10, batch=4096, lr=2e-3, log=print, family="rmat", train_n=20000,
                  test_n=200000, mean_degree=8.0, margins=(0.0, 0.1, 0.2, 0.3)):
    """Train the gate network on small graphs of one family, then decompose a
    larger one exactly (bounded schedule), gated with the trained network at
    each margin, gated with an untrained network, and gated without a
    network (which must equal the exact run)."""
    import time
    from . import khcore, synth
    torch = _torch()
    ctx = khcore.Context(0)
    t0 = time.time()
    if family == "rmat":
        graphs = (synth.rmat(train_scale, train_edge_factor, seed=train_seed + i) for i in range(train_count))
        train_desc = f"R-MAT scale {train_scale} ef {train_edge_factor}"
    else:
        graphs = (synth.chung_lu(train_n, mean_degree, 2.5, train_seed + i) for i in range(train_count))
        train_desc = f"Chung-Lu n={train_n} mean {mean_degree} beta 2.5"
    xs, ts = [], []
    for i, g in enumerate(graphs):
        gr = ctx.graph(g)
        masks, _, _ = states_of(ctx, gr, h)
        X, t = gate_samples(ctx, gr, h, masks)
        xs.append(X)
        ts.append(t)
        gr.close()
        log(f"training graph {i + 1}/{train_count}: {X.shape[0]} samples ({time.time() - t0:.0f} s)")
    X, t = torch.cat(xs).contiguous(), torch.cat(ts).contiguous()
    del xs, ts
    net = ctx.mlp(seed=7)
    t1 = time.time()
    losses = net.train(X, t, epochs=epochs, batch=batch, lr=lr, seed=1)
    torch.cuda.synchronize()
    out = {"h": h, "mode": "gate",
           "train": {"graphs": f"{train_desc}, seeds {train_seed}..{train_seed + train_count - 1}",
                     "samples": int(X.shape[0]), "epochs": epochs, "seconds": round(time.time() - t1, 2),
                     "loss_first": float(losses[0]), "loss_last": float(losses[-1])}}
    del X, t
    if family == "rmat":
        g = synth.rmat(test_scale, test_edge_factor, seed=1)
        test_desc = f"R-MAT scale {test_scale} ef {test_edge_factor}, seed 1"
    else:
        g = synth.chung_lu(test_n, mean_degree, 2.5, 1)
        test_desc = f"Chung-Lu n={test_n} mean {mean_degree} beta 2.5, seed 1"
    gr = ctx.graph(g)
    out["test"] = {"graph": test_desc, "n": g.n, "edges": g.num_edges}

    def run(name, fn):
        torch.cuda.synchronize()
        t2 = time.time()
        ctx.set_progress(lambda r, removed, level: log(f"  {name}: {time.time() - t2:.0f} s, round {r}, "
                                                        f"{removed} removed"), 20000)
        core, st = fn()
        torch.cuda.synchronize()
        ctx.set_progress(None)
        return core.cpu().numpy().view(np.uint32), st, time.time() - t2

    exact, st, te = run("exact", lambda: ctx.core(gr, h)[::2])
    out["exact"] = {"seconds": round(te, 2), "rounds": st["rounds"], "h_recomputes": st["h_recomputes"]}
    log(f"exact: {out['exact']}")
    untrained = ctx.mlp(seed=7)
    cases = [(f"gated_m{m}", net, m) for m in margins] + [("gated_untrained_m0.2", untrained, 0.2),
                                                          ("gated_no_network", None, 0.0)]
    for name, m, margin in cases:
        core, st, ta = run(name, lambda: ctx.core_gated(gr, h, m, margin)[::2])
        out[name] = {"seconds": round(ta, 2), "rounds": st["rounds"], "speedup_vs_exact": round(te / ta, 3),
                     "h_recomputes": st["h_recomputes"], "deferrals": st["gate_deferrals"],
                     "never_below_exact": bool((core >= exact).all()), **accuracy(exact, core)}
        log(f"{name}: {out[name]}")
    gr.close()
    ctx.close()
    return out


def main():
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="train the learned-mode network and evaluate it against "
                                             "exact peeling")
    ap.add_argument("--h", type=int, default=4)
    ap.add_argument("--train-scale", type=int, default=16)
    ap.add_argument("--train-count", type=int, default=32)
    ap.add_argument("--test-scale", type=int, default=18)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--family", choices=("rmat", "chung-lu"), default="rmat")
    ap.add_argument("--train-n", type=int, default=20000)
    ap.add_argument("--test-n", type=int, default=200000)
    ap.add_argument("--mean-degree", type=float, default=8.0)
    ap.add_argument("--sampling-rates", default="0.05,0.1,0.2", help="rates of the sampling-mode runs ('' for none)")
    ap.add_argument("--gate", action="store_true", help="train and evaluate the learned recompute gate instead")
    ap.add_argument("--margins", default="0,0.1,0.2,0.3", help="gate margins to evaluate")
    a = ap.parse_args()
    if a.gate:
        out = evaluate_gate(h=a.h, train_scale=a.train_scale, train_count=a.train_count, test_scale=a.test_scale,
                            test_edge_factor=16 if a.test_scale >= 20 else 8, epochs=a.epochs,
                            log=lambda m: print(m, file=sys.stderr, flush=True), family=a.family,
                            train_n=a.train_n, test_n=a.test_n, mean_degree=a.mean_degree,
                            margins=tuple(float(x) for x in a.margins.split(",") if x))
        print(json.dumps(out), flush=True)
        return
    out = evaluate(h=a.h, train_scale=a.train_scale, train_count=a.train_count, test_scale=a.test_scale,
                   test_edge_factor=16 if a.test_scale >= 20 else 8, epochs=a.epochs,
                   log=lambda m: print(m, file=sys.stderr, flush=True), family=a.family, train_n=a.train_n,
                   test_n=a.test_n, mean_degree=a.mean_degree,
                   sampling_rates=tuple(float(x) for x in a.sampling_rates.split(",") if x))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
