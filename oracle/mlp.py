"""Learned warm start for the occupation optimiser (not in the paper; the
occupations it predicts are always refined by the ON optimiser).

Per orbital p the features are (J_pp, K_pp, h_pp, mean_q J_pq, mean_q K_pq),
each standardised over the orbitals of its instance (z-score; J_pp = K_pp, so
two features coincide).  A 5 -> 128 -> 128 -> 1 perceptron with tanh hidden
units and a scaled sigmoid output predicts the angle theta_p in [0, pi/2] with
n_p = cos^2 theta_p.  Loss: mean squared error on theta.  Parameters are one
flat vector: W1 [5][128], b1 [128], W2 [128][128], b2 [128], w3 [128], b3.
"""
from __future__ import annotations

import math

import numpy as np

D_IN, D_H = 5, 128
SHAPES = [("W1", (D_IN, D_H)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
          ("w3", (D_H,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = p[o:o + k].reshape(shp)
        o += k
    return out


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng([seed, 0x3A])
    parts = []
    for name, shp in SHAPES:
        if name.startswith("b"):
            parts.append(np.zeros(int(np.prod(shp))))
        else:
            fan_in = shp[0]
            fan_out = shp[1] if len(shp) > 1 else 1
            a = math.sqrt(6.0 / (fan_in + fan_out))
            parts.append(rng.uniform(-a, a, int(np.prod(shp))))
    return np.concatenate(parts)


def features(hdiag, J, K):
    """[norb][5] standardised features of one instance."""
    F = np.stack([np.diag(J), np.diag(K), hdiag, J.mean(axis=1), K.mean(axis=1)], axis=1)
    mu = F.mean(axis=0)
    sd = F.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return (F - mu) / sd


def forward(p, X):
    q = unpack(p)
    A1 = X @ q["W1"] + q["b1"]
    H1 = np.tanh(A1)
    A2 = H1 @ q["W2"] + q["b2"]
    H2 = np.tanh(A2)
    z = H2 @ q["w3"] + q["b3"][0]
    s = 1.0 / (1.0 + np.exp(-z))
    theta = 0.5 * math.pi * s
    return theta, (X, H1, H2, s)


def loss_and_grad(p, X, target):
    """MSE loss and its gradient with respect to the flat parameter vector."""
    q = unpack(p)
    theta, (X, H1, H2, s) = forward(p, X)
    r = theta - target
    m = X.shape[0]
    loss = float(np.mean(r * r))
    dtheta = 2.0 * r / m
    dz = dtheta * 0.5 * math.pi * s * (1.0 - s)
    g = {}
    g["w3"] = H2.T @ dz
    g["b3"] = np.array([dz.sum()])
    dA2 = np.outer(dz, q["w3"]) * (1.0 - H2 * H2)
    g["W2"] = H1.T @ dA2
    g["b2"] = dA2.sum(axis=0)
    dA1 = (dA2 @ q["W2"].T) * (1.0 - H1 * H1)
    g["W1"] = X.T @ dA1
    g["b1"] = dA1.sum(axis=0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def adam(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def target_angles(n):
    """theta = arccos(sqrt(n)), the angle whose cos^2 is the occupation."""
    return np.arccos(np.sqrt(np.clip(n, 0.0, 1.0)))


def warm_gamma(theta, members, mapping, nfloor=1e-12):
    """Occupations cos^2(theta) projected onto each subspace's sum rule (each
    share at least nfloor), then mapped back to the optimiser's variables
    (softmax: gamma_i = log(n_pi/n_g); trigonometric: the inverse
    trigonometric map with n_g >= 1/2)."""
    from oracle.occupations import inverse_trig
    n = np.cos(theta) ** 2
    ns, ng1 = members.shape
    ng = ng1 - 1
    nn = n.copy()
    for row in members:
        tot = n[row].sum()
        vals = n[row] / tot if tot > 0 else np.full(ng1, 1.0 / ng1)
        vals = np.clip(vals, nfloor, None)
        if mapping == "trig" and vals[0] < 0.5:
            rest = vals[1:].sum()
            vals[1:] *= 0.5 / rest
            vals[0] = 0.5
        nn[row] = vals / vals.sum()
    if mapping == "trig":
        return inverse_trig(nn, members, ng)
    gamma = np.zeros((ns, ng))
    for g, row in enumerate(members):
        gamma[g] = np.log(nn[row[1:]] / nn[row[0]])
    return gamma


def cold_gamma(members, mapping, nstrong=0.98):
    """Cold start: n_g = 0.98, the hole shared equally by the weak orbitals."""
    ns, ng1 = members.shape
    ng = ng1 - 1
    if mapping == "softmax":
        return np.full((ns, ng), math.log((1.0 - nstrong) / ng / nstrong))
    from oracle.occupations import inverse_trig
    norb = int(members.max()) + 1
    n = np.zeros(norb)
    for row in members:
        n[row[0]] = nstrong
        n[row[1:]] = (1.0 - nstrong) / ng
    return inverse_trig(n, members, ng)
