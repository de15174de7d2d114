"""Pins of the MLP oracle: finite-difference gradient, a hand-computed tiny
network, ADAM's first step, feature standardisation, warm/cold-start maps."""
import math

import numpy as np

from oracle import mlp, occupations
from paper_2512_13550_amd import inputs


def test_gradient_against_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) + 0.01 * rng.standard_normal(mlp.NPARAMS)
    X = rng.standard_normal((7, 5))
    t = rng.uniform(0, math.pi / 2, 7)
    _, g = mlp.loss_and_grad(p, X, t)
    idx = np.concatenate([rng.choice(mlp.NPARAMS, 60, replace=False), [mlp.NPARAMS - 1, 0, 645]])
    eps = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAMS); e[i] = eps
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1e-3, abs(g[i])) + 1e-11


def test_hand_computed_network():
    # only w3 and b3 non-zero: H2 = tanh(0) = 0, so z = b3 and theta = pi/2 sigmoid(b3)
    p = np.zeros(mlp.NPARAMS)
    p[-1] = 0.3
    theta, _ = mlp.forward(p, np.ones((3, 5)))
    assert np.allclose(theta, 0.5 * math.pi / (1 + math.exp(-0.3)))
    # a single path: W1[0][0] = a, W2[0][0] = b, w3[0] = c
    a, b, c = 0.7, -1.1, 0.9
    q = mlp.unpack(p)
    q["W1"][0, 0] = a; q["W2"][0, 0] = b; q["w3"][0] = c
    x = np.array([[0.5, 0, 0, 0, 0]])
    z = c * math.tanh(b * math.tanh(a * 0.5)) + 0.3
    assert abs(mlp.forward(p, x)[0][0] - 0.5 * math.pi / (1 + math.exp(-z))) < 1e-15


def test_adam_first_step():
    g = np.array([0.5, -2.0, 0.0])
    p1, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=1e-30)
    assert np.allclose(p1, [-0.1, 0.1, 0.0])


def test_features_standardised():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((12, 12)); J = A @ A.T
    K = np.abs(rng.standard_normal((12, 12))); K = K + K.T; K[np.diag_indices(12)] = np.diag(J)
    F = mlp.features(rng.standard_normal(12), J, K)
    assert np.allclose(F.mean(axis=0), 0, atol=1e-14)
    assert np.allclose(F.std(axis=0), 1)
    assert np.allclose(F[:, 0], F[:, 1])           # J_pp == K_pp


def test_warm_and_cold_start_maps():
    members = np.array(inputs.pairing(16, 4, 3))
    for mapping in ("trig", "softmax"):
        g0 = mlp.cold_gamma(members, mapping)
        n0 = occupations.occupations(g0, members, 16, mapping)
        for row in members:
            assert abs(n0[row[0]] - 0.98) < 1e-12
            assert np.allclose(n0[row[1:]], 0.02 / 3)
        rng = np.random.default_rng(1)
        theta = rng.uniform(0, math.pi / 2, 16)
        gw = mlp.warm_gamma(theta, members, mapping)
        nw = occupations.occupations(gw, members, 16, mapping)
        for row in members:
            assert abs(nw[row].sum() - 1) < 1e-12
        # a feasible target is reproduced exactly
        n_t = occupations.occupations(rng.uniform(0.1, 1.2, (4, 3)), members, 16, mapping)
        back = occupations.occupations(mlp.warm_gamma(mlp.target_angles(n_t), members, mapping),
                                       members, 16, mapping)
        assert np.allclose(back, n_t, atol=1e-10)
