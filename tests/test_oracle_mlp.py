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
