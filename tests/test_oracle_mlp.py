"""Pins the oracle's MLP proposal: forward/backward by central finite
differences (FP64, rounding off), the closed-form softmax-KL gradient, a
hand-computed Adam step, GELU values, bfloat16 rounding."""
import math

import numpy as np

from oracle import mlp


def test_bf16_rounding_ties_to_even():
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even (1)
    assert mlp.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even (1 + 2^-6)
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6
    assert mlp.bf16_round(np.float32(1.0 + 2 ** -8 + 2 ** -20)) == 1.0 + 2 ** -7
    assert mlp.bf16_round(np.float32(-3.0)) == -3.0


def test_gelu_values():
    assert mlp.gelu(0.0) == 0.0
    # tanh form at x = 1: 0.5 (1 + tanh(sqrt(2/pi) * 1.044715))
    expect = 0.5 * (1 + math.tanh(math.sqrt(2 / math.pi) * 1.044715))
    assert abs(mlp.gelu(1.0) - expect) < 1e-15
    assert abs(mlp.gelu(-20.0)) < 1e-12 and abs(mlp.gelu(20.0) - 20.0) < 1e-12
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = {k: v.astype(np.float64) for k, v in mlp.init_params(3).items()}
    F = rng.normal(0, 1, (7, mlp.N_IN))
    dy = rng.normal(0, 1, 7)
    y, c = mlp.forward(p, F, rounding=False)
    g = mlp.backward(c, dy)
    h = 1e-6
    for k in mlp.PARAM_ORDER:
        flat = p[k].ravel()
        for idx in rng.choice(flat.shape[0], min(6, flat.shape[0]), replace=False):
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pm = {kk: vv.copy() for kk, vv in p.items()}
            pp[k].ravel()[idx] += h
            pm[k].ravel()[idx] -= h
            fd = (np.dot(dy, mlp.forward(pp, F, rounding=False)[0]) - np.dot(dy, mlp.forward(pm, F, rounding=False)[0])) / (2 * h)
            assert abs(g[k].ravel()[idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_softmax_kl_gradient_closed_form():
    rng = np.random.default_rng(1)
    y = rng.normal(0, 1, 10)
    ps = rng.uniform(0, 1, 10)
    groups = [np.arange(0, 4), np.arange(4, 10)]
    for idx in groups:
        ps[idx] /= ps[idx].sum()
    loss, dy = mlp.softmax_kl(y, ps, groups)
    h = 1e-6
    for k in range(10):
        yp, ym = y.copy(), y.copy()
        yp[k] += h
        ym[k] -= h
        fd = (mlp.softmax_kl(yp, ps, groups)[0] - mlp.softmax_kl(ym, ps, groups)[0]) / (2 * h)
        assert abs(dy[k] - fd) < 1e-7
    # KL of identical distributions is zero
    l0, d0 = mlp.softmax_kl(np.log(ps), ps, groups)
    assert abs(l0) < 1e-12 and np.abs(d0).max() < 1e-12


def test_adam_step_by_hand():
    p = {k: np.zeros(1) for k in mlp.PARAM_ORDER}
    p["b3"] = np.array([1.0])
    g = {k: np.zeros(1) for k in mlp.PARAM_ORDER}
    g["b3"] = np.array([0.5])
    z = {k: np.zeros(1) for k in mlp.PARAM_ORDER}
    out, m, v = mlp.adam_step(p, g, z, z, 1, lr=0.1)
    # t = 1: m_hat = g, v_hat = g^2 -> step = lr * g / (|g| + eps)
    assert abs(out["b3"][0] - (1.0 - 0.1 * 0.5 / (0.5 + 1e-8))) < 1e-15
    assert abs(m["b3"][0] - 0.05) < 1e-15 and abs(v["b3"][0] - 0.00025) < 1e-15


def test_weights_from_logits():
    w = mlp.weights_from_logits(np.array([0.0, -np.log(2.0), -100.0], np.float32))
    assert w[0] == 1 << 24 and abs(int(w[1]) - (1 << 23)) <= 1 and w[2] == 1


def test_targets_follow_column_std():
    t = np.array([[0.0, 1.0, 5.0], [0.0, 3.0, 5.0]])
    p = mlp.targets(t, 3)
    # sigma = (0, 1, 0), mean sigma = 1/3, mix 3 mean sigma = 1: weights (1, 2, 1)
    expect = np.array([1.0, 2.0, 1.0])
    np.testing.assert_allclose(p, expect / expect.sum(), rtol=1e-14)
