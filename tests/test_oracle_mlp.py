"""Pins of the surrogate MLP oracle (4 -> 64 -> 64 -> 1, SiLU, mean squared error).

* backpropagation equals central finite differences of the loss (FP64);
* bfloat16 rounding is round-to-nearest-even on the float32 bit pattern;
* the feature map (square-root stretch of d, |u|, |v|) sends the training box
  onto [-1, 1]^4, its centre in square-root coordinates onto 0.
"""
import numpy as np
import pytest


def _params(rng, scale=0.5):
    return rng.normal(0.0, scale, 4545)


def test_backprop_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(7)
    p = _params(rng)
    x = rng.uniform(-1, 1, (9, 4))
    t = rng.uniform(0, 1, 9)
    loss, g = oracle_lib.mlp_loss_grad(p, x, t)
    # every bias and first/last-layer weight, plus a sample of W2
    picks = list(range(0, 320)) + list(rng.choice(np.arange(320, 4416), 200, replace=False)) \
        + list(range(4416, 4545))
    h = 1e-6
    for k in picks:
        pp = p.copy(); pp[k] += h
        pm = p.copy(); pm[k] -= h
        lp, _ = oracle_lib.mlp_loss_grad(pp, x, t)
        lm, _ = oracle_lib.mlp_loss_grad(pm, x, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, k


def test_forward_consistent_with_loss(oracle_lib):
    rng = np.random.default_rng(8)
    p = _params(rng)
    x = rng.uniform(-1, 1, (33, 4))
    t = rng.uniform(0, 1, 33)
    y = oracle_lib.mlp_forward(p, x)
    loss, _ = oracle_lib.mlp_loss_grad(p, x, t)
    assert loss == pytest.approx(np.mean((y - t) ** 2), rel=1e-14)
    # a network with only output bias is a constant
    q = np.zeros(4545); q[-1] = 0.37
    np.testing.assert_array_equal(oracle_lib.mlp_forward(q, x), np.full(33, 0.37))


def test_bf16_rounding_is_nearest_even(oracle_lib):
    r = oracle_lib.bf16_round
    assert r(1.0) == 1.0
    assert r(1.0 + 2 ** -8) == 1.0                  # tie -> even (mantissa ...0)
    assert r(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6    # tie -> even (rounds up to ...10)
    assert r(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    assert r(-3.0) == -3.0
    # against numpy's view of float32 bits
    rng = np.random.default_rng(9)
    v = rng.normal(0, 10, 1000).astype(np.float32)
    u = v.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    ref = u.view(np.float32).astype(np.float64)
    got = np.array([r(float(x)) for x in v])
    np.testing.assert_array_equal(got, ref)


def test_bf16_mode_differs_only_by_rounding(oracle_lib):
    rng = np.random.default_rng(10)
    p = _params(rng, 0.3)
    x = rng.uniform(-1, 1, (64, 4))
    y64 = oracle_lib.mlp_forward(p, x)
    y16 = oracle_lib.mlp_forward(p, x, bf16=True)
    assert 0 < np.max(np.abs(y16 - y64)) < 0.05 * np.max(np.abs(y64))


def test_feature_map_box(oracle_lib):
    raw = np.array([[0.0, 0.0, 0.0, 0.25], [30.0, -3.0, 3.0, 1.0], [7.5, 0.75, -0.75, 0.625]])
    f = oracle_lib.surrogate_features(raw)
    np.testing.assert_allclose(f, [[-1, -1, -1, -1], [1, 1, 1, 1], [0, 0, 0, 0]], atol=1e-15)
