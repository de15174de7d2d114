"""Parity of the FP64 occupation update (mappings, functional energy and
gradient, PNOF5 and PNOF7 coefficients, L-BFGS) against the oracle.

Bars: E relative 1e-12, dE/dgamma and n normwise 1e-10 (FP64, different
summation order); a few L-BFGS iterations reproduce the oracle's iterates to
1e-8; at convergence E agrees to 1e-9 relative."""
import numpy as np
import pytest
import torch

from oracle import dfjk, functionals, occupations
from paper_2512_13550_amd import inputs
from gpu_util import dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu


def on_instance(ns, ng, seed, gap=1.0, extra=0):
    norb = ns * (ng + 1) + extra
    B = inputs.make_B(seed, norb, 3 * norb, 8.0)
    C = inputs.make_C(seed, norb, norb)
    H = inputs.make_H(seed, norb)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    hd = np.diag(dfjk.one_electron(H, C)).copy()
    members = occupations.aufbau_members(hd, ns, ng)
    hd[members[:, 0]] -= gap
    return norb, members, hd, J, K


def gpu_occ(nof, norb, members, mapping, functional):
    m = {"trig": nof.MAP_TRIG, "softmax": nof.MAP_SOFTMAX}[mapping]
    f = {"hf": nof.FUNC_HF, "pnof5": nof.FUNC_PNOF5, "pnof7": nof.FUNC_PNOF7}[functional]
    return nof.Occupations(norb, torch.from_numpy(members.astype(np.int32)).cuda(), m, f)


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
@pytest.mark.parametrize("functional", ["hf", "pnof5", "pnof7"])
@pytest.mark.parametrize("ns,ng,extra", [(4, 3, 0), (125, 3, 0), (9, 1, 5)])
def test_energy_grad(mapping, functional, ns, ng, extra):
    nof = need_gpu()
    norb, members, hd, J, K = on_instance(ns, ng, 3, extra=extra)
    rng = np.random.default_rng(1)
    gamma = rng.uniform(0.1, 1.4, (ns, ng)) if mapping == "trig" else rng.uniform(-4, 0, (ns, ng))
    E, g, n = occupations.energy_and_grad(gamma, members, norb, mapping, hd, J, K, functional)
    occ = gpu_occ(nof, norb, members, mapping, functional)
    Eg, gg, ngpu = occ.energy_grad(dev(gamma), dev(hd), dev(J), dev(K))
    torch.cuda.synchronize()
    assert int(occ.info[2]) == 0
    assert abs(float(Eg) - E) <= 1e-12 * abs(E)
    assert normwise(host(gg), g) <= 1e-10
    assert normwise(host(ngpu), n) <= 1e-14


@pytest.mark.parametrize("functional", ["hf", "pnof5", "pnof7"])
def test_functional_coefficients(functional):
    nof = need_gpu()
    norb, members, hd, J, K = on_instance(12, 3, 4, extra=3)
    n = occupations.occupations(np.full((12, 3), 0.4), members, norb, "trig")
    cJ, cK = functionals.coefficients(n, members, functional)
    occ = gpu_occ(nof, norb, members, "trig", functional)
    gJ, gK = occ.coefficients(dev(n))
    assert normwise(host(gJ), cJ) <= 1e-15
    assert normwise(host(gK), cK) <= 1e-15


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
def test_lbfgs_first_iterates_match(mapping):
    nof = need_gpu()
    norb, members, hd, J, K = on_instance(10, 3, 5)
    x0 = np.full((10, 3), 0.3 if mapping == "trig" else -3.0)
    for its in (1, 3, 6):
        x, n, E, it, ok = occupations.optimize_lbfgs(x0, members, norb, mapping, hd, J, K, "pnof5",
                                                     maxit=its, tol=0.0)
        occ = gpu_occ(nof, norb, members, mapping, "pnof5")
        g = dev(x0)
        Eg, ng_, info = occ.optimize(g, dev(hd), dev(J), dev(K), maxit=its, tol=0.0)
        torch.cuda.synchronize()
        assert int(info[0]) == it
        assert normwise(host(g), x) <= 1e-8, its
        assert abs(float(Eg) - E) <= 1e-11 * abs(E)


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
@pytest.mark.parametrize("ns,ng,functional", [(10, 3, "pnof5"), (125, 3, "pnof5"), (10, 3, "pnof7"),
                                              (125, 3, "pnof7")])
def test_lbfgs_converges_to_oracle_minimum(mapping, ns, ng, functional):
    nof = need_gpu()
    norb, members, hd, J, K = on_instance(ns, ng, 6)
    x0 = np.full((ns, ng), 0.3 if mapping == "trig" else -3.0)
    x, n, E, it, ok = occupations.optimize_lbfgs(x0, members, norb, mapping, hd, J, K, functional,
                                                 maxit=3000, tol=1e-8)
    assert ok
    occ = gpu_occ(nof, norb, members, mapping, functional)
    g = dev(x0)
    Eg, ng_, info = occ.optimize(g, dev(hd), dev(J), dev(K), maxit=3000, tol=1e-8)
    torch.cuda.synchronize()
    print(mapping, ns, "oracle iters", it, "gpu iters", int(info[0]), "E", E, float(Eg), flush=True)
    assert int(info[1]) == 1 and int(info[2]) == 0
    assert abs(float(Eg) - E) <= 1e-9 * abs(E)
    for row in members:
        assert abs(host(ng_)[row].sum() - 1.0) < 1e-13


def test_out_of_range_members_are_reported():
    nof = need_gpu()
    norb, members, hd, J, K = on_instance(4, 3, 7)
    bad = members.copy()
    bad[2, 1] = norb + 5
    occ = gpu_occ(nof, norb, bad, "trig", "pnof5")
    g = dev(np.full((4, 3), 0.3))
    occ.optimize(g, dev(hd), dev(J), dev(K), maxit=10)
    torch.cuda.synchronize()
    assert int(occ.info[2]) == nof.E_ARG
