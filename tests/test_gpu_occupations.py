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


@pytest.mark.parametrize("functional", ["hf", "pnof5"])
def test_softmax_large_arguments(functional):
    """Softmax variables beyond exp's range (gamma >= 710): the map stays
    finite and on the sum rule, and E, dE/dgamma and n equal the oracle's."""
    nof = need_gpu()
    norb, members, hd, J, K = on_instance(6, 3, 8)
    gamma = np.array([[710.0, 0.0, -5.0], [800.0, 800.0, 1000.0], [1000.0, 1000.0, -1000.0],
                      [-1000.0, -800.0, -750.0], [709.0, 709.5, 0.5], [-2.0, -3.0, -1.0]])
    E, g, n = occupations.energy_and_grad(gamma, members, norb, "softmax", hd, J, K, functional)
    assert np.isfinite(E) and np.all(np.isfinite(g))
    occ = gpu_occ(nof, norb, members, "softmax", functional)
    Eg, gg, ngpu = occ.energy_grad(dev(gamma), dev(hd), dev(J), dev(K))
    torch.cuda.synchronize()
    nh = host(ngpu)
    assert np.all(np.isfinite(nh)) and np.isfinite(float(Eg))
    for row in members:
        assert abs(nh[row].sum() - 1.0) < 1e-15
    assert abs(float(Eg) - E) <= 1e-12 * abs(E)
    assert normwise(nh, n) <= 1e-15
    assert normwise(host(gg), g) <= 1e-10


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
def test_lbfgs_vectors_in_lds_or_workspace_agree(mapping, monkeypatch):
    """The L-BFGS iteration vectors in LDS (every problem up to 144 KB of
    them) or in the workspace give bit-identical iterates."""
    nof = need_gpu()
    norb, members, hd, J, K = on_instance(20, 3, 9)
    x0 = np.full((20, 3), 0.3 if mapping == "trig" else -3.0)
    out = []
    for force in ("0", "1"):
        monkeypatch.setenv("NOF_OCC_VECTORS_IN_WORKSPACE", force)
        occ = gpu_occ(nof, norb, members, mapping, "pnof5")
        g = dev(x0)
        Eg, ng_, info = occ.optimize(g, dev(hd), dev(J), dev(K), maxit=400, tol=1e-9)
        torch.cuda.synchronize()
        out.append((host(g), float(Eg), host(info).tolist()))
    assert out[0][2] == out[1][2] and out[0][2][1] == 1
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_lbfgs_beyond_lds_matches_oracle_minimum():
    """Norb = 1000 with 250 subspaces of 3 weak orbitals needs ~174 KB of
    iteration vectors, more than the LDS holds: the workspace placement runs
    and reaches the oracle's minimum."""
    nof = need_gpu()
    ns, ng, norb, seed = 250, 3, 1000, 10
    B = inputs.make_B(seed, norb, 40, 25.0, threads=16)
    C = inputs.make_C(seed, norb, norb)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    hd = np.diag(dfjk.one_electron(inputs.make_H(seed, norb), C)).copy()
    members = occupations.aufbau_members(hd, ns, ng)
    hd[members[:, 0]] -= 1.0
    x0 = np.full((ns, ng), -3.0)
    x, n, E, it, ok = occupations.optimize_lbfgs(x0, members, norb, "softmax", hd, J, K, "pnof5",
                                                 maxit=3000, tol=1e-8)
    assert ok
    occ = gpu_occ(nof, norb, members, "softmax", "pnof5")
    g = dev(x0)
    Eg, ng_, info = occ.optimize(g, dev(hd), dev(J), dev(K), maxit=3000, tol=1e-8)
    torch.cuda.synchronize()
    print("oracle iters", it, "gpu iters", int(info[0]), flush=True)
    assert int(info[1]) == 1 and int(info[2]) == 0
    assert abs(float(Eg) - E) <= 1e-9 * abs(E)


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_lbfgs_kink_minima_match_oracle(seed):
    """Roles the one-electron energies contradict: weak occupations go to
    zero at kinks of E in the trigonometric angles.  The projected L-BFGS on
    the box converges on the GPU as in the oracle, to the same energy, with
    every variable inside the box."""
    nof = need_gpu()
    ns, ng = 6, 3
    norb = ns * (ng + 1)
    members = np.array(inputs.pairing(norb, ns, ng))
    B = inputs.make_B(seed, norb, 3 * norb, 4.0)
    C = inputs.make_C(seed, norb, norb)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    hd = np.diag(dfjk.one_electron(inputs.make_H(seed, norb), C)).copy()
    x0 = np.full((ns, ng), 0.6)
    x, n, E, it, ok = occupations.optimize_lbfgs(x0, members, norb, "trig", hd, J, K, "pnof5",
                                                 maxit=5000, tol=1e-9)
    assert ok
    occ = gpu_occ(nof, norb, members, "trig", "pnof5")
    g = dev(x0)
    Eg, ng_, info = occ.optimize(g, dev(hd), dev(J), dev(K), maxit=5000, tol=1e-9)
    torch.cuda.synchronize()
    lo, hi = occupations.variable_bounds("trig", (ns, ng))
    gh = host(g)
    assert int(info[1]) == 1 and int(info[2]) == 0
    assert np.all(gh >= lo) and np.all(gh <= hi)
    assert abs(float(Eg) - E) <= 1e-10 * abs(E)
