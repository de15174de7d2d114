"""Pins of the alternating NO + ON optimisation (oracle/solver.py).

1. Closed-shell HF: with the HF-like coefficients and occupations frozen at
   1 (ns orbitals) / 0, the NO optimisation must reach the minimum of the
   closed-shell Hartree-Fock energy, which a textbook Roothaan SCF with DIIS
   (Pulay, Chem. Phys. Lett. 73 (1980)) finds independently by
   diagonalising the Fock matrix F = H + J[D] - K[D] of the AO density
   D = C_occ C_occ^T (orthonormal AO basis, B = the fitted three-index tensor).
2. PNOF5 on a kernel-on-grid tensor: at convergence lambda is symmetric,
   re-optimising the occupations gains nothing, and no small rotation of the
   orbitals or change of the occupation variables lowers the energy.  (With
   the trigonometric map this instance alternates without settling within
   200 outer iterations at the default learning rate; the softmax map, the
   numerically more stable one, converges.)
"""
import numpy as np
import pytest

from oracle import dfjk, functionals, mlp, occupations, rotation, solver
from paper_2512_13550_amd import inputs
from _scf import scf_energy


def test_hf_minimum_equals_roothaan_scf():
    nbf, naux, nocc = 24, 96, 6
    B = inputs.make_B_grid(nbf, naux, seed=3)
    H = inputs.make_H(3, nbf)
    C0 = inputs.make_C(3, nbf, nbf)
    members = np.array(inputs.pairing(nbf, nocc, 1), dtype=np.int64)
    gamma = np.zeros((nocc, 1))                       # trig: n = 1 strong, 0 weak
    n = occupations.occupations(gamma, members, nbf, "trig")
    assert np.allclose(np.sort(n)[::-1][:nocc], 1.0) and np.isclose(n.sum(), nocc)
    r = solver.solve(B, C0, H, members, "trig", "hf", gamma, max_outer=3, no_steps=4000,
                     tol_lambda=1e-9, on_maxit=0)
    assert r["converged"]
    E_scf = scf_energy(B, H, nocc)
    assert abs(r["E"] - E_scf) <= 1e-10 * abs(E_scf), (r["E"], E_scf)


@pytest.mark.parametrize("mapping", ["softmax"])
def test_pnof5_converged_point_is_stationary(mapping):
    nbf, naux, ns, ng = 24, 96, 6, 2
    B = inputs.make_B_grid(nbf, naux, seed=5)
    H = inputs.make_H(5, nbf)
    C0 = inputs.make_C(5, nbf, nbf)
    members = np.array(inputs.pairing(nbf, ns, ng), dtype=np.int64)
    gamma0 = mlp.cold_gamma(members, mapping)
    hist = []
    r = solver.solve(B, C0, H, members, mapping, "pnof5", gamma0, max_outer=200, tol_lambda=1e-6,
                     tol_energy=1e-10, history=hist)
    assert r["converged"], (r["outer"], r["asym"])
    C, gamma, E = r["C"], r["gamma"], r["E"]
    # the energy of the returned point
    b, _ = dfjk.mo_transform(B, C)
    h = dfjk.one_electron(H, C)
    J, K = dfjk.jk(b)
    n = occupations.occupations(gamma, members, nbf, mapping)
    cJ, cK = functionals.coefficients(n, members, "pnof5")
    assert abs(dfjk.energy(n, h, J, K, cJ, cK) - E) <= 1e-12 * abs(E)
    assert E < hist[0][0]
    # the orbitals stayed orthonormal to rounding over the whole run (the
    # checks after each sweep saw no drift worth a repair)
    assert r["orth"] <= 1e-13
    assert np.max(np.abs(C.T @ C - np.eye(nbf))) <= 1e-13
    # re-optimising the occupations at the final orbitals gains nothing (the
    # last NO sweep follows the ON step, so the ON gradient is not exactly 0)
    _, _, E_on, _, _ = occupations.optimize_lbfgs(gamma, members, nbf, mapping, np.diag(h), J, K, "pnof5")
    assert E_on >= E - 1e-9
    # no small rotation or occupation change lowers E
    rng = np.random.default_rng(0)
    for _ in range(4):
        Y = rng.standard_normal((nbf, nbf))
        y = 1e-3 * (Y - Y.T)
        b2, _ = dfjk.mo_transform(B, rotation.rotate(C, y))
        h2 = dfjk.one_electron(H, rotation.rotate(C, y))
        J2, K2 = dfjk.jk(b2)
        assert dfjk.energy(n, h2, J2, K2, cJ, cK) >= E - 1e-9
        gp = gamma + 1e-3 * rng.standard_normal(gamma.shape)
        Ep, _, _ = occupations.energy_and_grad(gp, members, nbf, mapping, np.diag(h), J, K, "pnof5")
        assert Ep >= E - 1e-10


# ---- iterative diagonalization of the generalized pseudo-Fockian (orbopt = 1) ----

def test_pseudo_fock_diagonal_at_symmetric_lambda():
    """A symmetric lambda (the minimum) gives a diagonal pseudo-Fockian, whose
    eigenvectors are the current orbitals: the step leaves C unchanged."""
    from oracle import diagonalization
    rng = np.random.default_rng(1)
    A = rng.standard_normal((9, 9))
    lam = A + A.T
    F = diagonalization.pseudo_fock(lam, np.diag(lam), 1.0)
    assert np.array_equal(F, np.diag(np.diag(lam)))
    C = inputs.make_C(1, 12, 9)
    C2, e, V = diagonalization.step(C, lam, None, 1.0)
    assert np.array_equal(V, np.eye(9)) and np.array_equal(C2, C)


def test_pseudo_fock_step_descends_to_first_order():
    """Small asymmetry: the diagonalization rotates the orbitals by
    y_pq = -g_pq / (4 |d_q - d_p|) to first order (a descent step for every
    pair, whatever the index order of the diagonal), so the energy change
    predicted by the gradient, sum_{p<q} g_pq y_pq, is negative."""
    from oracle import diagonalization
    rng = np.random.default_rng(2)
    m = 8
    d = rng.permutation(np.linspace(-3.0, 2.0, m))          # diagonal not sorted by index
    S = rng.standard_normal((m, m)); S = S + S.T
    Aa = rng.standard_normal((m, m)); Aa = Aa - Aa.T
    eps = 1e-6
    lam = np.diag(d) + 0.1 * (S - np.diag(np.diag(S))) + eps * Aa
    g = 4.0 * (lam - lam.T)
    _, _, V = diagonalization.step(np.eye(m), lam, d, 1.0)
    y = (V - V.T) / 2.0                                     # first-order generator
    for p in range(m):
        for q in range(p + 1, m):
            expect = -g[p, q] / (4.0 * abs(d[q] - d[p]))
            assert abs(y[p, q] - expect) <= 1e-3 * abs(expect) + 1e-12
    dE = sum(g[p, q] * y[p, q] for p in range(m) for q in range(p + 1, m))
    assert dE < 0.0


def test_iterative_diagonalization_hf_equals_roothaan_scf():
    """0/1 occupations, HF-like coefficients: the iterative diagonalization
    converges to the minimum that the textbook Roothaan SCF with DIIS finds
    independently, with lambda symmetric."""
    nbf, naux, nocc = 24, 96, 6
    B = inputs.make_B_grid(nbf, naux, seed=3)
    H = inputs.make_H(3, nbf)
    C0 = inputs.make_C(3, nbf, nbf)
    members = np.array(inputs.pairing(nbf, nocc, 1), dtype=np.int64)
    gamma = np.zeros((nocc, 1))
    r = solver.solve(B, C0, H, members, "trig", "hf", gamma, max_outer=3, no_steps=2000,
                     tol_lambda=1e-8, on_maxit=0, orbopt=1, maxoff=1.0)
    assert r["converged"], (r["asym"], r["no_steps"])
    E_scf = scf_energy(B, H, nocc)
    assert abs(r["E"] - E_scf) <= 1e-10 * abs(E_scf), (r["E"], E_scf)


def test_greedy_overlap_match_hand_cases():
    """The greedy overlap matching on hand-made overlap matrices: a
    permutation matrix is read back; a case where the optimal sum assignment
    and the greedy rule differ takes the single largest overlap first."""
    from oracle import diagonalization
    P = np.eye(4)[[2, 0, 3, 1]]           # eigenvector k lives on orbital P[:, k].argmax()
    assert list(diagonalization.greedy_overlap_match(P)) == [1, 3, 0, 2]
    U = np.array([[0.9, 0.8], [0.8, 0.0]])
    # greedy: (r0, k0) = 0.9 first, then (r1, k1) = 0.0;  the sum-optimal would pick 0.8 + 0.8
    assert list(diagonalization.greedy_overlap_match(U)) == [0, 1]
    T = np.array([[0.5, 0.5], [0.5, 0.5]])  # ties: smaller r, then smaller k
    assert list(diagonalization.greedy_overlap_match(T)) == [0, 1]
