"""Pins of the float64 MLP reference (CPU only)."""
import numpy as np

from oracle import mlp

F, H = 8, 16


def _data(seed, n=40):
    g = np.random.default_rng(seed)
    theta = g.standard_normal(F * H + 2 * H + 1) * 0.5
    X = g.standard_normal((n, F))
    y = (g.random(n) < 0.4).astype(np.float64)
    return theta, X, y


def test_backprop_matches_central_differences():
    for seed in range(3):
        theta, X, y = _data(seed)
        ga = mlp.grad(theta, X, y, F, H)
        gn = mlp.finite_difference(theta, X, y, F, H)
        assert np.allclose(ga, gn, rtol=1e-5, atol=1e-8)


def test_forward_closed_form_cases():
    theta = np.zeros(F * H + 2 * H + 1)
    X = np.ones((3, F))
    assert np.allclose(mlp.forward(theta, X, F, H), 0.0)
    # loss of a zero network is log 2 whatever the labels
    assert np.isclose(mlp.loss(theta, X, [0, 1, 1], F, H), np.log(2.0))
    # one active hidden unit: s = w2[0] * relu(sum_f W1[f,0] * x_f + b1[0]) + b2
    W1, b1, w2, b2 = mlp.unpack(theta, F, H)
    theta2 = theta.copy()
    theta2[0:F * H].reshape(F, H)[:, 0] = 1.0
    theta2[F * H + H + 0] = 2.0
    theta2[-1] = -1.0
    Xv = np.array([[1, 2, 3, 0, 0, 0, 0, -1.0], [-5, 0, 0, 0, 0, 0, 0, 0.0]])
    assert np.allclose(mlp.forward(theta2, Xv, F, H), [2.0 * 5.0 - 1.0, -1.0])


def test_adam_decreases_loss():
    theta, X, y = _data(7, n=200)
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, y, F, H)
    for t in range(1, 101):
        theta, m, v = mlp.adam_step(theta, mlp.grad(theta, X, y, F, H), m, v, t, 1e-2)
    assert mlp.loss(theta, X, y, F, H) < l0


def test_bf16_round_known_values():
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even) -> 1 + 2^-6
    # 1 + 2^-8 + 2^-20 is just above halfway -> 1 + 2^-7
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, -2.5, 3.0e-3], np.float32)
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2.0 ** -6 and r[3] == 1 + 2.0 ** -7
    assert r[4] == -2.5
    # relative error bound of round-to-nearest with an 8-bit significand
    assert abs(r[5] - 3.0e-3) <= 2.0 ** -8 * 3.0e-3
