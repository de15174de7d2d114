"""Pins of the rotation oracle: closed forms and exact properties."""
import numpy as np
import pytest

from oracle import rotation


def test_two_by_two_closed_form():
    th = 0.7
    y = np.array([[0.0, th], [-th, 0.0]])
    U = rotation.expm_antisym(y)
    ref = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]])
    assert np.max(np.abs(U - ref)) < 1e-15


def test_block_diagonal_rotations_and_orthogonality():
    rng = np.random.default_rng(0)
    ths = rng.uniform(-3, 3, 5)
    y = np.zeros((10, 10))
    for i, th in enumerate(ths):
        y[2 * i, 2 * i + 1] = th
        y[2 * i + 1, 2 * i] = -th
    P = np.linalg.qr(rng.standard_normal((10, 10)))[0]
    U = rotation.expm_antisym(P @ y @ P.T)
    D = np.zeros((10, 10))
    for i, th in enumerate(ths):
        D[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]]
    assert np.max(np.abs(U - P @ D @ P.T)) < 1e-13
    assert np.max(np.abs(U.T @ U - np.eye(10))) < 1e-14


def test_rotate_columns_convention():
    # C' = C U: column p of C' is sum_q U_qp (column q of C)
    rng = np.random.default_rng(1)
    C = rng.standard_normal((6, 4))
    y = rng.standard_normal((4, 4)) * 0.3
    y = y - y.T
    U = rotation.expm_antisym(y)
    Cp = rotation.rotate(C, y)
    for p in range(4):
        assert np.allclose(Cp[:, p], sum(U[q, p] * C[:, q] for q in range(4)), atol=1e-14)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(2)
    g = rng.standard_normal((5, 5))
    g = g - g.T
    y, m, v = rotation.adam_step(g, np.zeros_like(g), np.zeros_like(g), 1, lr=0.01, eps=1e-30)
    off = ~np.eye(5, dtype=bool)
    assert np.allclose(y[off], -0.01 * np.sign(g[off]), atol=1e-15)
    assert np.all(y.diagonal() == 0)
    assert np.array_equal(y, -y.T)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
