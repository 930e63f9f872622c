"""Learned approximate mode: training data, training and evaluation.

Training samples come from the method itself: for each training graph the
exact GPU peeling gives, for every vertex, the round it is removed in; the
graph induced by the vertices still present after round r is a state the
approximate driver will meet.  For several such states the library computes
the eight features (khc_features) and the exact h-degrees (khdeg_compute),
which are the regression targets log1p(d^h) / 8.  Training runs on the GPU
(khc_mlp_train).  Accuracy is judged against exact core numbers: the
fraction of vertices with the exact core, the mean absolute error, and the
precision of the paper's Section V (Exp-4), 1 - mean over v of
|c(v) - c^(v)| / c(v), taken over vertices whose exact core is not 0.
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
    torch = _torch()
    core, rnd, st = ctx.core(gr, h, with_round=True)
    rounds = int(st["rounds"])
    r = rnd.view(torch.int32)
    masks = []
    for f in fractions:
        r0 = int(f * rounds)
        masks.append((r >= r0).to(torch.uint8))
    return masks, core, rnd


def samples(ctx, gr, h, masks):
    """Features and targets of the live vertices of every state."""
    torch = _torch()
    xs, ts = [], []
    for m in masks:
        X, _, _ = ctx.features(gr, h, m)
        d = ctx.hdeg(gr, h, m)
        live = m.bool()
        xs.append(X[live])
        ts.append(torch.log1p(d[live].double()).float() / FEATURE_SCALE)
    return torch.cat(xs), torch.cat(ts)


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
