"""Pins of the occupation mappings, the functional's dE/dn and the ON optimiser."""
import numpy as np
import pytest

from oracle import dfjk, functionals, occupations
from paper_2512_13550_amd import inputs


def members_of(ns, ng, norb=None):
    norb = ns * (ng + 1) if norb is None else norb
    return np.array(inputs.pairing(norb, ns, ng)), norb


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
@pytest.mark.parametrize("ng", [1, 2, 3, 5])
def test_sum_rule_and_bounds(mapping, ng):
    ns = 7
    members, norb = members_of(ns, ng)
    rng = np.random.default_rng(ng)
    for _ in range(20):
        gamma = rng.uniform(-4, 4, (ns, ng))
        n = occupations.occupations(gamma, members, norb, mapping)
        for row in members:
            assert abs(n[row].sum() - 1.0) < 1e-14
        assert np.all(n >= 0) and np.all(n <= 1)
        if mapping == "trig":
            assert np.all(n[members[:, 0]] >= 0.5 - 1e-15)
        else:
            assert np.all(n > 0)


def test_trig_inverse_roundtrip():
    ns, ng = 6, 3
    members, norb = members_of(ns, ng)
    rng = np.random.default_rng(3)
    gamma = rng.uniform(0.05, 1.5, (ns, ng))
    n = occupations.occupations(gamma, members, norb, "trig")
    g2 = occupations.inverse_trig(n, members, ng)
    assert np.allclose(occupations.occupations(g2, members, norb, "trig"), n, atol=1e-14)


def _jk(norb, seed):
    B = inputs.make_B(seed, norb, 3 * norb, 4.0, threads=1)
    C = inputs.make_C(seed, norb, norb)
    H = inputs.make_H(seed, norb)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    return np.diag(dfjk.one_electron(H, C)).copy(), J, K


@pytest.mark.parametrize("functional", ["hf", "pnof5", "pnof7"])
def test_dEdn_against_finite_differences(functional):
    ns, ng = 3, 2
    members, norb = members_of(ns, ng)
    hd, J, K = _jk(norb, 1)
    rng = np.random.default_rng(0)
    n = rng.uniform(0.05, 0.9, norb)
    g = functionals.denergy_dn(n, hd, J, K, members, functional)
    eps = 1e-6
    for r in range(norb):
        e = np.zeros(norb); e[r] = eps
        fd = (functionals.energy_of_n(n + e, hd, J, K, members, functional)
              - functionals.energy_of_n(n - e, hd, J, K, members, functional)) / (2 * eps)
        assert abs(fd - g[r]) < 1e-7 * max(1.0, abs(g[r]))


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
@pytest.mark.parametrize("functional", ["hf", "pnof5", "pnof7"])
def test_dEdgamma_against_finite_differences(mapping, functional):
    ns, ng = 3, 3
    members, norb = members_of(ns, ng)
    hd, J, K = _jk(norb, 2)
    rng = np.random.default_rng(1)
    gamma = rng.uniform(0.2, 1.3, (ns, ng))
    _, grad, _ = occupations.energy_and_grad(gamma, members, norb, mapping, hd, J, K, functional)
    eps = 1e-6
    for g in range(ns):
        for i in range(ng):
            d = np.zeros_like(gamma); d[g, i] = eps
            Ep = occupations.energy_and_grad(gamma + d, members, norb, mapping, hd, J, K, functional)[0]
            Em = occupations.energy_and_grad(gamma - d, members, norb, mapping, hd, J, K, functional)[0]
            assert abs((Ep - Em) / (2 * eps) - grad[g, i]) < 1e-7 * max(1.0, abs(grad[g, i]))


def test_two_electron_two_orbital_exact_minimum():
    """One electron pair in two orbitals: the PNOF5 energy at its minimum over
    the trigonometric variable is the lower eigenvalue of the 2x2 problem
    [[a, -K], [-K, b]] with a = 2h_gg + J_gg, b = 2h_pp + J_pp (all PNOFs are
    exact for two electrons)."""
    members = np.array([[0, 1]])
    for seed in range(5):
        hd, J, K = _jk(2, 10 + seed)
        a, b = 2 * hd[0] + J[0, 0], 2 * hd[1] + J[1, 1]
        if a > b:      # the strong orbital must be the lower one for n_g >= 1/2
            hd = hd[::-1].copy(); J = J[::-1, ::-1].copy(); K = K[::-1, ::-1].copy()
            a, b = b, a
        exact = 0.5 * (a + b) - np.sqrt(0.25 * (a - b) ** 2 + K[0, 1] ** 2)
        x, n, E, it, ok = occupations.optimize_lbfgs(np.array([[0.3]]), members, 2, "trig", hd, J, K,
                                                  "pnof5", tol=1e-10, maxit=2000)
        assert ok
        assert abs(E - exact) < 1e-12 * max(1.0, abs(exact))


@pytest.mark.parametrize("mapping", ["trig", "softmax"])
def test_optimizer_reaches_a_stationary_minimum(mapping):
    from scipy.optimize import minimize
    ns, ng = 4, 3
    norb = ns * (ng + 1)
    hd, J, K = _jk(norb, 5)
    members = occupations.aufbau_members(hd, ns, ng)
    hd[members[:, 0]] -= 1.0          # occupied/virtual gap of the synthetic ON instance
    x0 = np.full((ns, ng), 0.3 if mapping == "trig" else -3.0)
    x, n, E, it, ok = occupations.optimize_lbfgs(x0, members, norb, mapping, hd, J, K, "pnof5",
                                              tol=1e-8, maxit=5000)
    assert ok, it
    f = lambda v: occupations.energy_and_grad(v.reshape(ns, ng), members, norb, mapping, hd, J, K, "pnof5")[0]
    jac = lambda v: occupations.energy_and_grad(v.reshape(ns, ng), members, norb, mapping, hd, J, K, "pnof5")[1].ravel()
    res = minimize(f, x0.ravel(), jac=jac, method="L-BFGS-B", options=dict(gtol=1e-11, ftol=1e-15, maxiter=10000))
    # an independent library optimiser from the same start finds no lower energy,
    # and the gradient vanishes at the returned point
    assert E <= res.fun + 1e-9 * max(1.0, abs(E))
    assert np.max(np.abs(jac(x.ravel()))) < 1e-6


def _grid_jk(norb, seed):
    """h_pp, J, K on the kernel-on-grid tensor (K >= 0 there)."""
    B = inputs.make_B_grid(norb, 4 * norb, seed=seed)
    C = inputs.make_C(seed, norb, norb)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    return np.diag(dfjk.one_electron(inputs.make_H(seed, norb), C)).copy(), J, K


def test_pnof7_reduces_to_pnof5():
    """One subspace: no interpair term.  Occupations 0 or 1: Phi = 0, so the
    interpair term vanishes for any number of subspaces."""
    members = np.array([[0, 1, 2]])
    hd, J, K = _jk(3, 4)
    n = np.array([0.9, 0.07, 0.03])
    for f in (functionals.coefficients, ):
        c5, c7 = f(n, members, "pnof5"), f(n, members, "pnof7")
        assert np.array_equal(c5[0], c7[0]) and np.array_equal(c5[1], c7[1])
    ns, ng = 3, 2
    members, norb = members_of(ns, ng)
    hd, J, K = _jk(norb, 5)
    n = np.zeros(norb)
    n[members[:, 0]] = 1.0
    assert functionals.energy_of_n(n, hd, J, K, members, "pnof7") == \
        functionals.energy_of_n(n, hd, J, K, members, "pnof5")


def test_pnof7_interpair_term_lowers_the_energy():
    """With K >= 0 (kernel-on-grid tensor) the interpair term -Phi_p Phi_q K_pq
    only lowers E, by exactly sum over ordered pairs of different subspaces;
    a sign or factor slip in Pi fails this."""
    ns, ng = 3, 2
    members, norb = members_of(ns, ng)
    hd, J, K = _grid_jk(norb, 6)
    assert np.all(K >= 0)
    rng = np.random.default_rng(6)
    n = occupations.occupations(rng.uniform(0.3, 1.2, (ns, ng)), members, norb, "trig")
    E5 = functionals.energy_of_n(n, hd, J, K, members, "pnof5")
    E7 = functionals.energy_of_n(n, hd, J, K, members, "pnof7")
    phi = np.sqrt(n * (1 - n))
    grp, _ = functionals.group_of(norb, members)
    inter = sum(phi[p] * phi[q] * K[p, q] for p in range(norb) for q in range(norb)
                if grp[p] != grp[q])
    assert inter > 0
    assert abs((E5 - E7) - inter) <= 1e-12 * max(1.0, abs(E7))


def test_pnof7_two_electron_exact():
    """One pair: PNOF7 has no interpair term and keeps PNOF5's exact
    two-electron two-orbital minimum."""
    members = np.array([[0, 1]])
    hd, J, K = _jk(2, 12)
    a, b = 2 * hd[0] + J[0, 0], 2 * hd[1] + J[1, 1]
    if a > b:
        hd = hd[::-1].copy(); J = J[::-1, ::-1].copy(); K = K[::-1, ::-1].copy()
        a, b = b, a
    exact = 0.5 * (a + b) - np.sqrt(0.25 * (a - b) ** 2 + K[0, 1] ** 2)
    x, n, E, it, ok = occupations.optimize_lbfgs(np.array([[0.3]]), members, 2, "trig", hd, J, K,
                                                 "pnof7", tol=1e-10, maxit=2000)
    assert ok and abs(E - exact) < 1e-12 * max(1.0, abs(exact))


def test_pnof7_cumulant_against_spin_orbital_2rdm():
    """The PNOF7 (Delta, Pi) through Eq. (PNOF)'s coefficients gives the energy
    of the spin-orbital 2RDM built from the same cumulant."""
    import _bruteforce as bf
    ns, ng = 2, 1
    members, norb = members_of(ns, ng)
    B = inputs.make_B(8, norb, 3 * norb, 4.0, threads=1)
    C = inputs.make_C(8, norb, norb)
    H = inputs.make_H(8, norb)
    n = occupations.occupations(np.array([[0.4], [0.7]]), members, norb, "trig")
    Delta, Pi = functionals.delta_pi(n, members, "pnof7")
    assert np.any(Pi[members[0][:, None], members[1][None, :]] != 0)
    b, _ = dfjk.mo_transform(B, C)
    h = dfjk.one_electron(H, C)
    J, K = dfjk.jk(b)
    cJ, cK = dfjk.coeffs_from_cumulant(n, Delta, Pi)
    E = dfjk.energy(n, h, J, K, cJ, cK)
    Ebf = bf.spin_orbital_energy(n, h, bf.mo_eri(B, C), Delta, Pi)
    assert abs(E - Ebf) <= 1e-12 * max(1.0, abs(Ebf))


# ---- closed-form values of the two ON maps (Occupation Number Optimization) ----
# Hand-evaluated from the printed equations at angles / exponentials whose
# squares are exact rationals; a sin^2 <-> cos^2 swap, a shifted index or a
# wrong subspace assignment changes at least one value.

def _member_orders():
    # natural order and a scrambled assignment of the four orbitals
    return [np.array([[0, 1, 2, 3]]), np.array([[2, 0, 3, 1]])]


def test_trig_map_hand_values():
    """Eq. trigo-n_sdono_gamma and the weak-orbital chain, N_g = 3:
    gamma_g = pi/3 (cos^2 = 1/4): n_g = (1 + 1/4)/2 = 5/8, h_g = 3/8;
    gamma_p1 = pi/6 (sin^2 = 1/4): n_p1 = 3/8 * 1/4 = 3/32;
    gamma_p2 = pi/3 (sin^2 = 3/4, cos^2 = 1/4): n_p2 = 3/8 * 3/4 * 3/4 = 27/128,
    n_p3 = 3/8 * 3/4 * 1/4 = 9/128."""
    gamma = np.array([[np.pi / 3, np.pi / 6, np.pi / 3]])
    expect = [5 / 8, 3 / 32, 27 / 128, 9 / 128]
    for members in _member_orders():
        n = occupations.occupations(gamma, members, 4, "trig")
        for k, p in enumerate(members[0]):
            assert abs(n[p] - expect[k]) < 4e-16, (members, k)


@pytest.mark.parametrize("g,ng_expect", [(0.0, 1.0), (np.pi / 4, 0.75), (np.pi / 2, 0.5),
                                          (2 * np.pi / 3, 0.625)])
def test_trig_map_strong_orbital_hand_values(g, ng_expect):
    """N_g = 1: n_g = (1 + cos^2 gamma)/2 and the single weak orbital takes the hole."""
    n = occupations.occupations(np.array([[g]]), np.array([[1, 0]]), 2, "trig")
    assert abs(n[1] - ng_expect) < 4e-16 and abs(n[0] - (1 - ng_expect)) < 4e-16


def test_softmax_map_hand_values():
    """Eqs. softmax-n_sdono_gamma and n_wdono_gamma1: exp(gamma) = (1, 2, 3)
    gives n_g = 1/7 and n_p = (1/7, 2/7, 3/7); exp(gamma) = (1/2, 1/4) gives
    n_g = 4/7, n_p = (2/7, 1/7)."""
    for members in _member_orders():
        n = occupations.occupations(np.log([[1.0, 2.0, 3.0]]), members, 4, "softmax")
        for k, p in enumerate(members[0]):
            assert abs(n[p] - [1 / 7, 1 / 7, 2 / 7, 3 / 7][k]) < 4e-16
    n = occupations.occupations(np.log([[0.5, 0.25]]), np.array([[2, 0, 1]]), 3, "softmax")
    assert np.allclose(n, [2 / 7, 1 / 7, 4 / 7], rtol=0, atol=4e-16)


@pytest.mark.parametrize("gamma", [[710.0, 0.0, -5.0], [800.0, 800.0, 1000.0], [1000.0, 1000.0, -1000.0],
                                   [-1000.0, -800.0, -750.0], [709.0, 709.5, 0.5]])
def test_softmax_map_large_arguments(gamma):
    """The softmax map is defined for every gamma: occupations stay finite,
    non-negative and on the sum rule where exp(gamma) alone overflows, and
    equal the map evaluated in 60-digit decimal arithmetic."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    members = np.array([[0, 1, 2, 3]])
    with np.errstate(over="raise", invalid="raise"):
        n = occupations.occupations(np.array([gamma]), members, 4, "softmax")
        gr = occupations.chain_rule(np.array([gamma]), members, 4, "softmax", np.array([1.0, -2.0, 0.5, 3.0]))
    assert np.all(np.isfinite(n)) and np.all(n >= 0) and abs(n.sum() - 1.0) < 1e-15
    assert np.all(np.isfinite(gr))
    e = [Decimal(x).exp() for x in gamma]
    den = 1 + sum(e)
    ref = [float(1 / den)] + [float(x / den) for x in e]
    assert np.allclose(n, ref, rtol=1e-14, atol=1e-300)


def test_pnof5_equals_geminal_product_expectation():
    """PNOF5 is the energy of an antisymmetrized product of strongly
    orthogonal geminals, each in natural-orbital form with coefficient
    +sqrt(n_g) on its strong orbital and -sqrt(n_p) on every weak one (the
    sign choice behind Pi = -sqrt(n n) with the strong orbital and
    +sqrt(n n) between weak orbitals; Pernal, Comput. Theor. Chem. 1003 (2013)
    127).  <Psi|H|Psi> is evaluated here by brute force in Fock space from h and
    the four-index integrals, with no cumulant or coefficient matrix: a wrong
    weak-weak sign, a missing interpair exchange term or a factor slip fails."""
    import _bruteforce as bf
    for ns, ng, seed in ((1, 2, 21), (1, 3, 22), (2, 2, 23), (3, 1, 24)):
        members, norb = members_of(ns, ng)
        B = inputs.make_B(seed, norb, 3 * norb, 4.0, threads=1)
        C = inputs.make_C(seed, norb, norb)
        h = dfjk.one_electron(inputs.make_H(seed, norb), C)
        eri = bf.mo_eri(B, C)
        b, _ = dfjk.mo_transform(B, C)
        J, K = dfjk.jk(b)
        rng = np.random.default_rng(seed)
        n = occupations.occupations(rng.uniform(0.2, 1.3, (ns, ng)), members, norb, "trig")
        c = -np.sqrt(n)
        c[members[:, 0]] = np.sqrt(n[members[:, 0]])
        psi = bf.geminal_product_state([list(r) for r in members], c)
        Ebf, norm = bf.expectation_energy(psi, h, eri)
        assert abs(norm - 1.0) < 1e-14
        E5 = functionals.energy_of_n(n, np.diag(h).copy(), J, K, members, "pnof5")
        assert abs(E5 - Ebf) < 1e-12 * max(1.0, abs(Ebf)), (ns, ng, E5, Ebf)
        # the opposite weak-weak sign is a different (non-geminal) energy
        if ng >= 2:
            c2 = c.copy()
            c2[members[:, 1]] *= -1.0
            Ebad, _ = bf.expectation_energy(bf.geminal_product_state([list(r) for r in members], c2), h, eri)
            assert abs(E5 - Ebad) > 1e-8


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_box_optimizer_reaches_kink_minima(seed):
    """Roles that the one-electron energies contradict (the first orbitals
    strong, no gap) push weak occupations to zero, where PNOF5's
    sqrt(n_p n_q) terms make E a kink in the angles: no gradient vanishes
    there.  The optimiser on the box of the trigonometric variables stops with
    a vanishing projected gradient, and the point is a local minimum checked
    without the gradient code: E rises (central one-sided differences of E)
    when any variable held at a face moves inwards, and the free components
    are stationary.  (A variable can also be flat there: once an earlier
    factor cos^2 theta_l is zero, the later angles move no occupation.)"""
    ns, ng = 6, 3
    members, norb = members_of(ns, ng)
    hd, J, K = _jk(norb, seed)
    x0 = np.full((ns, ng), 0.6)
    x, n, E, it, ok = occupations.optimize_lbfgs(x0, members, norb, "trig", hd, J, K, "pnof5",
                                                 maxit=5000, tol=1e-9)
    assert ok, it
    lo, hi = occupations.variable_bounds("trig", (ns, ng))
    assert np.all(x >= lo) and np.all(x <= hi)
    f = lambda v: occupations.energy_and_grad(v, members, norb, "trig", hd, J, K, "pnof5")[0]
    at_face = (x <= lo) | (x >= hi)
    assert at_face.any()            # the instance does have kink minima
    for idx in zip(*np.nonzero(at_face)):
        for step in (1e-6, 1e-4):
            v = x.copy()
            v[idx] += step if x[idx] <= lo[idx] else -step
            assert f(v) >= E - 1e-13 * abs(E), (idx, step)
    for idx in zip(*np.nonzero(~at_face)):
        v1 = x.copy(); v1[idx] += 1e-6
        v2 = x.copy(); v2[idx] -= 1e-6
        assert abs(f(v1) - f(v2)) / 2e-6 < 1e-6
