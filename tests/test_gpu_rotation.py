"""Parity of the FP64 rotation step (exp of an antisymmetric generator, C U,
ADAM) against the oracle.  Bar: 1e-13 normwise (FP64 throughout)."""
import numpy as np
import pytest
import torch

from oracle import rotation
from paper_2512_13550_amd import inputs
from gpu_util import dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu


# Norb below ~1000 runs the products on 64-wide tiles with a few K splits,
# 1024 (64 tiles of 128) on 128-wide tiles with more splits: both plans here
@pytest.mark.parametrize("norb,scale", [(48, 1e-2), (260, 0.3), (131, 30.0), (3, 2.0), (500, 1e-2),
                                        (1024, 0.05)])
def test_expm_and_rotate(norb, scale):
    nof = need_gpu()
    print(f"case expm norb={norb} scale={scale}", flush=True)
    y = inputs.make_antisym(5, 0, norb, scale=scale)
    U = nof.expm_antisym(dev(y))
    Uref = rotation.expm_antisym(y)
    assert normwise(host(U), Uref) <= 1e-13
    C = inputs.make_C(3, norb + 17, norb)
    Cn = nof.rotate_orbitals(dev(C), U)
    assert normwise(host(Cn), C @ Uref) <= 1e-13


def test_zero_generator_gives_identity():
    nof = need_gpu()
    U = host(nof.expm_antisym(dev(np.zeros((70, 70)))))
    assert np.array_equal(U, np.eye(70))


def test_adam_steps():
    nof = need_gpu()
    norb = 97
    rng = np.random.default_rng(0)
    m = np.zeros((norb, norb)); v = np.zeros((norb, norb))
    md, vd = dev(m), dev(v)
    for t in range(1, 4):
        g = rng.standard_normal((norb, norb)); g = g - g.T
        y, m, v = rotation.adam_step(g, m, v, t, lr=0.02)
        yd = nof.adam_step(dev(g), md, vd, t, lr=0.02)
        assert normwise(host(yd), y) <= 1e-14
        assert normwise(host(md), m) <= 1e-15
        assert np.array_equal(host(yd), -host(yd).T)


def spd(rng, n):
    A = rng.standard_normal((n, n))
    return A @ A.T / n + np.eye(n)


@pytest.mark.parametrize("nbf,norb,with_S", [(40, 30, False), (130, 97, True), (520, 500, False),
                                              (1041, 1024, True)])
def test_orthonormalize(nbf, norb, with_S):
    """max|C^T S C - I| and the Newton-Schulz repair against the oracle: C
    untouched (bit for bit) within the tolerance, repaired past it."""
    nof = need_gpu()
    print(f"case orthonormalize nbf={nbf} norb={norb} S={with_S}", flush=True)
    rng = np.random.default_rng(nbf)
    S = spd(rng, nbf) if with_S else None
    L = np.linalg.cholesky(S) if with_S else np.eye(nbf)
    Q = np.linalg.solve(L.T, np.linalg.qr(rng.standard_normal((nbf, norb)))[0])   # Q^T S Q = I
    C = Q @ (np.eye(norb) + 1e-4 * rng.standard_normal((norb, norb)))
    Sd = dev(S) if with_S else None
    C1_ref, err_ref = rotation.orthonormalize(C, S, tol=0.0)
    Cd = dev(C)
    err = float(nof.orthonormalize(Cd, Sd, tol=1.0))
    assert abs(err - err_ref) <= 1e-13 and torch.equal(Cd, dev(C))
    err = float(nof.orthonormalize(Cd, Sd, tol=0.0))
    assert abs(err - err_ref) <= 1e-13
    C1 = host(Cd)
    assert normwise(C1, C1_ref) <= 1e-13
    # the error left is the closed form of one step, -3/4 E0^2 + 1/4 E0^3
    E0 = rotation.orthonormality_error(C, S)
    E1 = rotation.orthonormality_error(C1, S)
    print("err", err, "after", float(np.max(np.abs(E1))), flush=True)
    assert np.max(np.abs(E1 - (-0.75 * E0 @ E0 + 0.25 * E0 @ E0 @ E0))) <= 1e-13
