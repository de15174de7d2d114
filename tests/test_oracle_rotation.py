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


def spd(rng, n):
    A = rng.standard_normal((n, n))
    return A @ A.T / n + np.eye(n)


def test_orthonormality_error_brute_force():
    # E_pq = sum_mu,nu C_mu,p S_mu,nu C_nu,q - delta_pq, written out on a tiny case
    rng = np.random.default_rng(3)
    C = rng.standard_normal((5, 3))
    S = spd(rng, 5)
    E = rotation.orthonormality_error(C, S)
    for p in range(3):
        for q in range(3):
            ref = sum(C[mu, p] * S[mu, nu] * C[nu, q] for mu in range(5) for nu in range(5))
            assert abs(E[p, q] - (ref - (p == q))) < 1e-13
    assert np.array_equal(rotation.orthonormality_error(C), C.T @ C - np.eye(3))


@pytest.mark.parametrize("with_S", [False, True])
def test_newton_schulz_step_leaves_the_closed_form_error(with_S):
    # C^T S C = I + E0 (E0 symmetric): after C (I - E0/2) the error is
    # (I - E0/2)(I + E0)(I - E0/2) - I = -3/4 E0^2 + 1/4 E0^3
    rng = np.random.default_rng(4)
    nbf, norb = 9, 6
    S = spd(rng, nbf) if with_S else None
    L = np.linalg.cholesky(S) if with_S else np.eye(nbf)
    Q = np.linalg.solve(L.T, np.linalg.qr(rng.standard_normal((nbf, norb)))[0])   # Q^T S Q = I
    A = rng.standard_normal((norb, norb)) * 1e-3
    C = Q @ (np.eye(norb) + A)
    E0 = rotation.orthonormality_error(C, S)
    C1, err = rotation.orthonormalize(C, S, tol=0.0)
    assert err == float(np.max(np.abs(E0))) and err > 1e-4
    E1 = rotation.orthonormality_error(C1, S)
    assert np.max(np.abs(E1 - (-0.75 * E0 @ E0 + 0.25 * E0 @ E0 @ E0))) < 1e-14
    assert np.max(np.abs(E1)) < 2 * err ** 2


def test_orthonormalize_within_tolerance_returns_the_input():
    rng = np.random.default_rng(5)
    C = np.linalg.qr(rng.standard_normal((8, 5)))[0]
    C2, err = rotation.orthonormalize(C, tol=1e-12)
    assert err < 1e-15 and np.array_equal(C2, C)
