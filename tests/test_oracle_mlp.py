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


GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    for ln in open(__import__("os").path.join(GOLDEN, name)):
        ln = ln.strip()
        if ln and not ln.startswith("#"):
            rows.append(ln.split())
    return rows


def test_features_of_a_hand_worked_slice():
    """tests/golden/features_toy.txt: every feature of two columns, derived by
    hand from the definitions (count normalisation, cosine signs, logs)."""
    stats = dict(count=np.array([2, 1]), sum=np.array([6.0, 0.0]), sumsq=np.array([20.0, 0.0]),
                 min=np.array([2.0, 0.0]), max=np.array([4.0, 0.0]), zeros=np.array([0.0, 1.0]))
    geo = dict(centroid=np.array([1.0, 0.0, 0.0]), diag=2.0, mean_normal=np.array([0.0, 0.0, 1.0]))
    clusters = dict(pos=np.array([[1.0, 0.0, 3.0], [1.0, 4.0, 0.0]]),
                    nrm=np.array([[0.0, 0.0, -1.0], [0.0, -1.0, 0.0]]),
                    intensity=np.array([6.0, 2.0]), bbox_diag=np.array([0.5, 0.0]), members=np.array([4, 1]))
    F = mlp.features(stats, geo, clusters, np.array([0, 1]), 3)
    want = np.array([[float(v) for v in r[1:]] for r in _golden_rows("features_toy.txt")])
    assert want.shape == (2, 12)
    # the +1e-6 / +1e-12 guards of the definitions move the values by < 1e-6
    np.testing.assert_allclose(F, want, rtol=0, atol=2e-6)


def _one_unit_net(F0, W1, b1, W2, b2, W3, b3):
    p = {k: np.zeros(v.shape, np.float32) for k, v in mlp.init_params(0).items()}
    p["W1"][0, 0], p["b1"][0], p["W2"][0, 0], p["b2"][0], p["W3"][0, 0], p["b3"][0] = W1, b1, W2, b2, W3, b3
    F = np.zeros((1, mlp.N_IN), np.float32)
    F[0, 0] = F0
    return p, F


def test_every_bf16_rounding_point_of_the_forward_pass():
    """tests/golden/mlp_bf16_rounding_cases.txt: for each rounding point (W1,
    W2, W3, h1, h2) a network whose output moves by more than 5% of |y| if that point
    alone were dropped; the oracle must give the hand-worked rounded value."""
    rows = _golden_rows("mlp_bf16_rounding_cases.txt")
    assert {r[0] for r in rows} == {"W1", "W2", "W3", "h1", "h2"}
    for r in rows:
        vals = [float(v) for v in r[1:]]
        p, F = _one_unit_net(*vals[:7])
        y, _ = mlp.forward(p, F, rounding=True)
        assert y[0] == vals[7], (r[0], y[0])
        assert abs(vals[7] - vals[8]) > 0.05 * abs(vals[7]), r[0]
