"""Reference forward and backward pass of the learned-mode MLP.

TEST INFRASTRUCTURE ONLY (shares no code with the GPU library).

Network: 8 inputs -> 64 -> 64 (ReLU) -> 1, layer l computing W_l x + b_l,
parameters packed as W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3
(4801 values).  The target is a mean squared error over the rows.

Two variants:
  * exact=True: plain float64 arithmetic (used to pin the analytic backward
    against finite differences);
  * exact=False: the library's precision contract -- inputs, weights and
    hidden activations rounded to bfloat16 (round to nearest even) before
    each matrix product, products summed in float64 here (float32 on the
    GPU), biases kept in float32, the ReLU derivative read from the rounded
    activation, the hidden-layer gradients rounded to bfloat16 before their
    matrix products.

The optimiser reference is Adam (Kingma and Ba, "Adam: A Method for
Stochastic Optimization", Algorithm 1) with bias-corrected moments, in
float64: adam_step().
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 8, 64
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = p[off:off + size].reshape(shape)
        off += size
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    nan = np.isnan(a)
    r = r.astype(np.uint32)
    if nan.any():
        r[nan] = (a.view(np.uint32)[nan] | 0x400000) & 0xFFFF0000
    return r.view(np.float32).astype(np.float64)


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def forward(params, X, exact=False):
    """Returns (y, cache) for rows X (n x 8)."""
    P = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    if exact:
        rd = lambda v: v  # noqa: E731
        W1, W2, W3 = P["W1"], P["W2"], P["W3"]
        b1, b2, b3 = P["b1"], P["b2"], P["b3"][0]
    else:
        rd = bf16
        W1, W2, W3 = bf16(P["W1"]), bf16(P["W2"]), bf16(P["W3"])
        b1, b2, b3 = _f32(P["b1"]), _f32(P["b2"]), _f32(P["b3"])[0]
    x = rd(X)
    z1 = x @ W1.T + b1
    h1 = rd(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + b2
    h2 = rd(np.maximum(z2, 0.0))
    y = h2 @ W3 + b3
    return y, {"x": x, "h1": h1, "h2": h2, "rd": rd, "P": P}


def loss(params, X, t, exact=True):
    y, _ = forward(params, X, exact)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(params, X, t, exact=False):
    """Gradient of mean((y - t)^2) with respect to the packed parameters."""
    y, c = forward(params, X, exact)
    P, rd, x, h1, h2 = c["P"], c["rd"], c["x"], c["h1"], c["h2"]
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n
    W3 = P["W3"] if exact else _f32(P["W3"])
    W2 = P["W2"] if exact else bf16(P["W2"])
    g = {}
    g["W3"] = dy @ h2
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, W3) * (h2 > 0)
    g["b2"] = dz2.sum(axis=0)
    dz2r = rd(dz2)
    g["W2"] = dz2r.T @ h1
    dz1 = rd((dz2r @ W2) * (h1 > 0))
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = dz1.T @ x[:, :N_IN]
    return pack(g)


def finite_difference(params, X, t, eps=1e-6, idx=None):
    """Central differences of the float64 loss at the given parameter indices."""
    p = np.asarray(params, dtype=np.float64).copy()
    idx = range(p.size) if idx is None else idx
    out = []
    for i in idx:
        old = p[i]
        p[i] = old + eps
        lp = loss(p, X, t, exact=True)
        p[i] = old - eps
        lm = loss(p, X, t, exact=True)
        p[i] = old
        out.append((lp - lm) / (2 * eps))
    return np.array(out)


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1), float64.

    step is the 1-based index t of this update.  Returns (params', m', v'):
      m' = beta1 m + (1 - beta1) g
      v' = beta2 v + (1 - beta2) g^2
      params' = params - lr * (m' / (1 - beta1^t)) / (sqrt(v' / (1 - beta2^t)) + eps)
    """
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m1 = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v1 = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m1 / (1.0 - beta1 ** step)
    vhat = v1 / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m1, v1
