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


# --- forward value pinned by closed forms ----------------------------------------
# The logistic function at ln k is k / (k + 1), so SiLU(z) = z / (1 + e^-z) takes
# the closed values SiLU(ln k) = ln k * k / (k + 1) and SiLU(-ln k) = -ln k / (k + 1).
# The networks below route inputs through single hidden units so that every
# pre-activation is +-ln k; the outputs are then sums of logarithms.  A different
# activation (GELU, tanh, sigmoid), a transposed W1 or W2 (W[o][i] read as W[i][o])
# or a misplaced bias/output weight changes the value.
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 256, 320, 4416, 4480, 4544


def _w1(p, o, i, v):
    p[OFF_W1 + 4 * o + i] = v


def _w2(p, o, i, v):
    p[OFF_W2 + 64 * o + i] = v


def test_forward_closed_form_one_path(oracle_lib):
    """x1 -> hidden-1 unit 0 -> hidden-2 unit 5 -> output, with W2[5][0] = 4 ln2 / ln3."""
    ln2, ln3 = np.log(2.0), np.log(3.0)
    p = np.zeros(4545)
    _w1(p, 0, 1, 1.0)                          # z1[0] = x1
    _w2(p, 5, 0, 4.0 * ln2 / ln3)              # z2[5] = W2[5][0] h1[0]; W2[0][5] stays 0
    p[OFF_W3 + 5] = 1.5
    p[OFF_B3] = 0.1
    x = np.array([[0.37, ln3, -0.55, 0.81],    # z1 = ln3: h1 = 3/4 ln3, z2 = ln8: h2 = 8/9 ln8
                  [-0.9, -ln3, 0.2, -0.4]])    # z1 = -ln3: h1 = -1/4 ln3, z2 = -ln2: h2 = -1/3 ln2
    y = oracle_lib.mlp_forward(p, x)
    np.testing.assert_allclose(y, [0.1 + 4.0 * ln2, 0.1 - 0.5 * ln2], rtol=0, atol=1e-14)


def test_forward_closed_form_all_inputs(oracle_lib):
    """Every input, both bias vectors and two output weights in use."""
    ln2, ln3 = np.log(2.0), np.log(3.0)
    p = np.zeros(4545)
    _w1(p, 7, 0, 1.0)                          # z1[7] = x0 + ln2 = ln4 : h1 = 4/5 ln4
    p[OFF_B1 + 7] = ln2
    _w1(p, 8, 2, -2.0)                         # z1[8] = -2 x2 = ln3     : h1 = 3/4 ln3
    _w1(p, 9, 3, 2.0)                          # z1[9] = 2 x3 = -ln3     : h1 = -1/4 ln3
    _w1(p, 10, 1, 0.5)                         # z1[10] = x1 / 2 = ln2   : h1 = 2/3 ln2
    for i in (7, 8, 9, 10):
        _w2(p, 20, i, 1.0)
    # z2[20] = 8/5 ln2 + 3/4 ln3 - 1/4 ln3 + 2/3 ln2 + b2 = ln2 with this bias: h2 = 2/3 ln2
    p[OFF_B2 + 20] = ln2 - (1.6 * ln2 + 0.5 * ln3 + 2.0 / 3.0 * ln2)
    _w2(p, 21, 9, 4.0)                         # z2[21] = -ln3 : h2 = -1/4 ln3
    p[OFF_W3 + 20] = 3.0                       # + 2 ln2
    p[OFF_W3 + 21] = -4.0                      # + ln3
    p[OFF_B3] = -1.0
    x = np.array([[ln2, 2.0 * ln2, -0.5 * ln3, -0.5 * ln3]])
    y = oracle_lib.mlp_forward(p, x)
    np.testing.assert_allclose(y, [np.log(12.0) - 1.0], rtol=0, atol=1e-14)
