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
