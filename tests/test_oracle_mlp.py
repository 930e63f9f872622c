"""Pins for the MLP reference (CPU): bf16 rounding values, closed-form
networks, and the analytic backward against finite differences."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_values():
    # exactly representable values are kept
    for v in (0.0, 1.0, -2.5, 0.15625, 2.0 ** 100, -(2.0 ** -100)):
        assert mlp.bf16(v) == np.float32(v)
    # ties go to the even mantissa: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    # above halfway rounds up, below rounds down
    assert mlp.bf16(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    assert mlp.bf16(1.0 + 2 ** -9) == 1.0
    assert np.isnan(mlp.bf16(np.nan))


def _params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=mlp.N_PARAMS)


def test_zero_weights_give_output_bias():
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["b3"][0] = 0.75
    X = np.random.default_rng(1).normal(size=(5, 8))
    y, _ = mlp.forward(mlp.pack(p), X, exact=True)
    assert np.allclose(y, 0.75)


def test_constructed_network_computes_a_feature():
    # y = relu(x0) - relu(-x0) = x0 through the two hidden layers
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["W1"][0, 0], p["W1"][1, 0] = 1.0, -1.0
    p["W2"][0, 0], p["W2"][1, 1] = 1.0, 1.0
    p["W3"][0], p["W3"][1] = 1.0, -1.0
    X = np.random.default_rng(2).normal(size=(7, 8))
    y, _ = mlp.forward(mlp.pack(p), X, exact=True)
    assert np.allclose(y, X[:, 0])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = _params(3)
    X = rng.normal(size=(12, 8))
    t = rng.normal(size=12)
    g = mlp.backward(p, X, t, exact=True)
    idx = list(rng.choice(mlp.N_PARAMS, size=120, replace=False)) + [4800, 512, 4736]
    fd = mlp.finite_difference(p, X, t, idx=idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-7)


def test_rounded_variant_close_to_exact():
    rng = np.random.default_rng(4)
    p = _params(4, 0.2)
    X = rng.normal(size=(50, 8))
    y64, _ = mlp.forward(p, X, exact=True)
    y16, _ = mlp.forward(p, X, exact=False)
    assert np.max(np.abs(y64 - y16)) < 0.05 * (1 + np.max(np.abs(y64)))


# ---------------------------------------------------------------------------
# bf16 contract of the backward pass, pinned on a hand-built case.
#
# One input row x = (x0, 0, ..., 0), target 0, and a chain of single units:
# W1[0][0] = a, W2[0][0] = c, W3[0] = e, every other parameter 0.  Then only
# unit 0 of each hidden layer is active and the loss is (y - 0)^2 with
#   y = bf16(h2) * bf16(e),  h2 = bf16(relu(h1 * bf16(c))),
#   h1 = bf16(relu(bf16(x0) * bf16(a))).
# The values below are chosen so that every rounding point of the contract
# moves the result; each rounding is written out by hand (bf16 keeps 7
# fraction bits, so near 1 its grid is 1 + k/128).
from fractions import Fraction as Fr

X0 = 1 + 2 ** -8 + 2 ** -10       # bf16 -> 1 + 2^-7   (above the midpoint 1 + 2^-8)
A = 1 + 2 ** -7 + 2 ** -10        # bf16 -> 1 + 2^-7   (below the midpoint 1 + 3*2^-8)
C = 1 + 2 ** -7 + 2 ** -9         # bf16 -> 1 + 2^-7
E = 1 + 2 ** -8 + 2 ** -11        # bf16 -> 1 + 2^-7   (above the midpoint 1 + 2^-8)


def _chain_params():
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["W1"][0, 0], p["W2"][0, 0], p["W3"][0] = A, C, E
    return mlp.pack(p)


def _hand_gradient():
    """The contract's gradient of the chain, by hand in exact arithmetic."""
    q = Fr(1, 128)
    xr = 1 + q                       # bf16(X0)
    ar = 1 + q                       # bf16(A)
    z1 = xr * ar                     # 1 + 2^-6 + 2^-14
    h1 = 1 + 2 * q                   # bf16(z1): the 2^-14 is dropped
    cr = 1 + q                       # bf16(C)
    z2 = h1 * cr                     # 1 + 3/128 + 2^-13
    h2 = 1 + 3 * q                   # bf16(z2)
    er = 1 + q                       # bf16(E) (forward only)
    y = h2 * er                      # 1 + 2^-5 + 3 * 2^-14, exact in fp32
    dy = 2 * y                       # d/dy of (y - 0)^2 over one row
    g = {"W3": dy * h2, "b3": dy}
    dz2 = dy * Fr(E)                 # the backward reads the fp32 master W3
    g["b2"] = dz2
    # bf16(dz2): dz2 = 2.07192..., grid step 2^-6 in [2, 4)
    dz2r = Fr(133, 64)               # 2 + 5/64 = 2.078125 is nearest (2.0625 + 2^-6 = 2.078125)
    assert abs(dz2 - dz2r) < Fr(1, 128)
    g["W2"] = dz2r * h1
    dz1_raw = dz2r * cr              # 2.0943603515625
    dz1 = Fr(67, 32)                 # bf16: 2 + 3/32 = 2.09375
    assert abs(dz1_raw - dz1) < Fr(1, 128)
    g["b1"] = dz1
    g["W1"] = dz1 * xr
    return {k: float(v) for k, v in g.items()}, float(y)


def test_bf16_backward_on_hand_built_chain():
    p = _chain_params()
    X = np.zeros((1, 8))
    X[0, 0] = X0
    want, y_want = _hand_gradient()
    y, _ = mlp.forward(p, X, exact=False)
    assert y[0] == y_want
    g = mlp.unpack(mlp.backward(p, X, np.zeros(1), exact=False))
    assert g["W3"][0] == want["W3"]
    assert g["b3"][0] == want["b3"]
    assert g["b2"][0] == want["b2"]
    assert g["W2"][0, 0] == want["W2"]
    assert g["b1"][0] == want["b1"]
    assert g["W1"][0, 0] == want["W1"]
    # every other entry is zero (inactive units)
    flat = mlp.backward(p, X, np.zeros(1), exact=False)
    assert np.count_nonzero(flat) == 6


def test_hand_built_chain_discriminates_every_rounding_point():
    """Dropping any one rounding of the contract changes the hand values,
    so the pin above fails for a contract with a rounding point missing."""
    q = Fr(1, 128)
    want, y_want = _hand_gradient()
    # no rounding of x0, a, h1, c or h2 in the forward pass: y moves
    exact_y = Fr(X0) * Fr(A)
    for alt in (Fr(X0) * (1 + q), (1 + q) * Fr(A)):
        assert float(alt) != float((1 + q) * (1 + q))
    assert float(exact_y * Fr(C)) != float((1 + 2 * q) * (1 + q))
    assert float((1 + 3 * q) * Fr(E)) != y_want                       # W3 not rounded forward
    assert float((1 + 2 * q) * (1 + q) * (1 + q)) != y_want           # h2 not rounded
    # backward: bf16 W3 instead of the fp32 master, unrounded dz2, unrounded dz1
    dy = 2 * Fr(y_want)
    assert float(dy * (1 + q)) != want["b2"]
    assert float(dy * Fr(E) * (1 + 2 * q)) != want["W2"]
    assert float(Fr(133, 64) * (1 + q)) != want["b1"]
    assert float(Fr(133, 64) * (1 + q) * (1 + q)) != want["W1"]


# ---------------------------------------------------------------------------
# Adam (Kingma and Ba, Algorithm 1) pins.

def test_adam_first_step_moves_by_lr_times_sign():
    """With bias correction the first update is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0, -7.0])
    p = np.array([1.0, 2.0, -1.0, 0.5, 0.0])
    p1, m1, v1 = mlp.adam_step(p, g, np.zeros(5), np.zeros(5), 1, 0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    assert p1[3] == p[3]  # zero gradient, zero moments: no move


def test_adam_constant_gradient_keeps_the_step():
    """A constant gradient gives bias-corrected moments g and g^2 at every
    step, so every update is lr * g / (|g| + eps)."""
    g = np.array([0.25, -4.0])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 6):
        p_new, m, v = mlp.adam_step(p, g, m, v, t, 0.1)
        assert np.allclose(p_new - p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        p = p_new


def test_adam_two_steps_by_hand():
    """g1 = +1 then g2 = -1: m2 = 0.9*0.1 - 0.1 = -0.01, corrected by
    1 - 0.9^2 = 0.19; v2 = 0.999*0.001 + 0.001 = 0.001999, corrected by
    1 - 0.999^2 = 0.001999 to exactly 1.  Second move: +lr * 0.01/0.19."""
    p1, m1, v1 = mlp.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, 1.0)
    p2, m2, v2 = mlp.adam_step(p1, -np.ones(1), m1, v1, 2, 1.0)
    assert np.isclose(m2[0], -0.01, rtol=1e-12)
    assert np.isclose(v2[0], 0.001999, rtol=1e-12)
    assert np.isclose(p2[0] - p1[0], (0.01 / 0.19) / (1.0 + 1e-8), rtol=1e-9)
