"""Learned warm start on the GPU: features, forward, loss gradient, ADAM and
the warm-start map against the oracle (FP32 kernels against FP64 oracle),
then a small end-to-end run: the network is trained on converged occupations
from the plain optimiser and reduces the optimiser's iterations on held-out
larger instances without changing the converged energy."""
import math

import numpy as np
import pytest
import torch

from oracle import dfjk, mlp, occupations
from paper_2512_13550_amd import inputs
from gpu_util import dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu


def small_jk(norb, seed):
    B = inputs.make_B(seed, norb, 3 * norb, 8.0)
    C = inputs.make_C(seed, norb, norb)
    H = inputs.make_H(seed, norb)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    return np.diag(dfjk.one_electron(H, C)).copy(), J, K


@pytest.mark.parametrize("norb", [40, 257])
def test_features(norb):
    nof = need_gpu()
    hd, J, K = small_jk(norb, 1)
    X = host(nof.mlp_features(dev(hd), dev(J), dev(K)))
    assert normwise(X, mlp.features(hd, J, K)) <= 1e-6


def test_forward_loss_grad_adam():
    nof = need_gpu()
    rng = np.random.default_rng(0)
    p = mlp.init_params(3) + 0.05 * rng.standard_normal(mlp.NPARAMS)
    p32 = p.astype(np.float32)
    X = rng.standard_normal((301, 5)).astype(np.float32)
    t = rng.uniform(0, math.pi / 2, 301).astype(np.float32)
    p64, X64, t64 = p32.astype(np.float64), X.astype(np.float64), t.astype(np.float64)
    th = host(nof.mlp_forward(dev(X, torch.float32), dev(p32, torch.float32)))
    assert normwise(th, mlp.forward(p64, X64)[0]) <= 2e-6
    loss, g = nof.mlp_loss_grad(dev(X, torch.float32), dev(t, torch.float32), dev(p32, torch.float32))
    lref, gref = mlp.loss_and_grad(p64, X64, t64)
    assert abs(float(loss) - lref) <= 1e-5 * lref
    assert normwise(host(g), gref) <= 1e-4
    m = torch.zeros(mlp.NPARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    pd = dev(p32, torch.float32)
    nof.mlp_adam(pd, g, m, v, 1, lr=1e-3)
    pref, _, _ = mlp.adam(p64, host(g), np.zeros(mlp.NPARAMS), np.zeros(mlp.NPARAMS), 1, lr=1e-3)
    assert np.max(np.abs(host(pd) - pref)) <= 1e-6


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
def test_warm_gamma_map(mapping):
    nof = need_gpu()
    ns, ng = 6, 3
    norb = ns * (ng + 1) + 2
    members = np.array(inputs.pairing(norb, ns, ng))
    theta = np.random.default_rng(2).uniform(0.02, 1.5, norb).astype(np.float32)
    m = nof.MAP_TRIG if mapping == "trig" else nof.MAP_SOFTMAX
    g = host(nof.mlp_warm_gamma(dev(theta, torch.float32), dev(members.astype(np.int32), torch.int32), m,
                                norb, 1e-3))
    ref = mlp.warm_gamma(theta.astype(np.float64), members, mapping, 1e-3)
    assert normwise(g, ref) <= 1e-10
    n_g = occupations.occupations(g, members, norb, mapping)
    for row in members:
        assert abs(n_g[row].sum() - 1.0) < 1e-13


def test_trained_network_against_cold_start():
    """Trains on converged ONs of small instances and reports, on held-out
    larger instances, the optimiser's iterations from the cold start, from the
    network's warm start and from the converged point itself (the ideal warm
    start).  Checks that training reduces the loss, that every start converges
    to the same energy, and that the warm start needs fewer iterations than
    the cold start on average (the runs are bitwise repeatable: fixed-order
    reductions everywhere)."""
    nof = need_gpu()
    from paper_2512_13550_amd import warmstart
    fac = warmstart.InstanceFactory(nof, gap=0.5)
    rng = np.random.default_rng(7)
    X, T, it_train = warmstart.build_dataset(nof, fac, range(5000, 5060), (60, 90), (8, 20), rng)
    params, hist = warmstart.train(nof, X, T, epochs=60, batch=1024, lr=3e-3, seed=1)
    print("train rows", X.shape[0], "loss", hist[0], "->", hist[-1], flush=True)
    assert hist[-1] < 0.5 * hist[0]
    rows = warmstart.evaluate(nof, fac, params, range(9000, 9006), 150, 30)
    cold = np.array([r["iters_cold"] for r in rows])
    warm = np.array([r["iters_warm"] for r in rows])
    ideal = np.array([r["iters_restart"] for r in rows])
    dE = np.array([abs(r["E_warm"] - r["E_cold"]) for r in rows])
    print("held-out iters cold", cold, "warm", warm, "restart", ideal, "max |dE|", dE.max(), flush=True)
    assert all(r["converged"] for r in rows)
    assert dE.max() <= 1e-7
    assert ideal.max() <= 5
    assert warm.mean() < cold.mean()


@pytest.mark.parametrize("mapping", [0, 1])
def test_cold_start_through_device_map(mapping):
    """The cold start (n_g = 0.98, the hole shared equally) built by the
    device-side map inversion equals the closed form of either map (to the
    FP32 rounding of the angles handed over)."""
    nof = need_gpu()
    from paper_2512_13550_amd import warmstart
    fac = warmstart.InstanceFactory(nof, gap=0.5)
    inst = fac.make(77, 60, 12, mapping=mapping)
    g = host(warmstart.cold_gamma(inst))
    ng = inst["ng"]
    n = occupations.occupations(g, inst["members"], inst["norb"], "trig" if mapping == 0 else "softmax")
    for row in inst["members"]:
        assert abs(n[row[0]] - 0.98) < 1e-6
        assert np.all(np.abs(n[row[1:]] - 0.02 / ng) < 1e-6)
