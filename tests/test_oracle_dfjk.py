"""Pins of the CPU oracle's DF-JK / generalized-Fock functions (no GPU).

Each test checks the oracle against something other than itself: four-index
integrals, the spin-orbital 2RDM energy, finite differences, the textbook
closed-shell Fock matrix, exact invariants, and a kernel-on-grid tensor with
physical positivity.
"""
import numpy as np
import pytest

from oracle import dfjk
from paper_2512_13550_amd import inputs
import _bruteforce as bf


def small_instance(seed, nbf=10, naux=24, norb=None, decay=4.0):
    norb = nbf if norb is None else norb
    B = inputs.make_B(seed, nbf, naux, decay, threads=1)
    C = inputs.make_C(seed, nbf, norb)
    H = inputs.make_H(seed, nbf)
    return B, C, H


def rand_sym(rng, m, scale=1.0):
    A = rng.standard_normal((m, m)) * scale
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_jk_against_four_index(seed):
    # tiny workload shape: Nbf=48, Naux=192, Norb=48
    w = inputs.WORKLOADS["tiny"]
    B = inputs.make_B(w.seed + seed, w.nbf, w.naux, w.decay, threads=1)
    C = inputs.make_C(w.seed + seed, w.nbf, w.norb)
    b, D = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    g = bf.mo_eri(B, C)
    idx = np.arange(w.norb)
    J4 = g[idx[:, None], idx[:, None], idx[None, :], idx[None, :]]   # (pp|qq)
    K4 = g[idx[:, None], idx[None, :], idx[None, :], idx[:, None]]   # (pq|qp)
    assert np.max(np.abs(J - J4)) <= 1e-12 * np.max(np.abs(J4))
    assert np.max(np.abs(K - K4)) <= 1e-12 * np.max(np.abs(K4))
    # b itself: (pq|rs) = sum_P b_pq b_rs
    bf_ = b.reshape(w.naux, -1)
    g2 = (bf_.T @ bf_).reshape(g.shape)
    assert np.max(np.abs(g2 - g)) <= 1e-12 * np.max(np.abs(g))
    assert np.array_equal(D, np.diagonal(b, axis1=1, axis2=2))


def test_transform_rectangular_against_four_index():
    # Norb < Nbf: transpose mistakes change the shape or the values
    B, C, _ = small_instance(3, nbf=12, naux=30, norb=7)
    b, D = dfjk.mo_transform(B, C)
    assert b.shape == (30, 7, 7) and D.shape == (30, 7)
    g = bf.mo_eri(B, C)
    bf_ = b.reshape(30, -1)
    assert np.allclose((bf_.T @ bf_).reshape(g.shape), g, rtol=0, atol=1e-13 * np.abs(g).max())
    # explicit element: b^P_pq = sum_mu,nu C_mu p B^P_mu nu C_nu q
    P, p, q = 5, 2, 6
    ref = sum(C[m, p] * B[P, m, n_] * C[n_, q] for m in range(12) for n_ in range(12))
    assert abs(b[P, p, q] - ref) < 1e-14


def test_invariants_any_B():
    w = inputs.WORKLOADS["tiny"]
    B = inputs.make_B(7, w.nbf, w.naux, w.decay, threads=1)
    C = inputs.make_C(7, w.nbf, w.nbf)             # square orthogonal C
    b, D = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    s = np.max(np.abs(J))
    assert np.max(np.abs(J - J.T)) <= 1e-14 * s
    assert np.max(np.abs(K - K.T)) <= 1e-14 * s
    assert np.max(np.abs(np.diag(J) - np.diag(K))) <= 1e-14 * s
    assert np.all(K >= 0)
    assert np.all(J ** 2 <= np.outer(np.diag(J), np.diag(J)) * (1 + 1e-12))
    # orthogonal invariance with Norb = Nbf
    assert np.isclose(K.sum(), np.sum(B * B), rtol=1e-12)
    assert np.isclose(J.sum(), np.sum(np.trace(B, axis1=1, axis2=2) ** 2), rtol=1e-12)


def test_physical_positivity_on_grid_tensor():
    # With a positive, positive-definite kernel, J_pq >= K_pq >= 0.
    B = inputs.make_B_grid(14, 60, seed=1)
    C = inputs.make_C(11, 14, 14)
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    tol = 1e-12 * np.abs(J).max()
    assert np.all(K >= -tol)
    assert np.all(J - K >= -tol)
    assert np.all(np.abs(np.diag(J) - np.diag(K)) <= tol)


@pytest.mark.parametrize("seed", [0, 1])
def test_energy_against_spin_orbital_2rdm(seed):
    rng = np.random.default_rng(100 + seed)
    m = 5
    B, C, H = small_instance(seed, nbf=m, naux=11)
    n = rng.uniform(0.05, 0.95, m)
    Delta = rand_sym(rng, m, 0.3)
    Pi = rand_sym(rng, m, 0.3)
    b, _ = dfjk.mo_transform(B, C)
    h = dfjk.one_electron(H, C)
    J, K = dfjk.jk(b)
    cJ, cK = dfjk.coeffs_from_cumulant(n, Delta, Pi)
    E = dfjk.energy(n, h, J, K, cJ, cK)
    Ebf = bf.spin_orbital_energy(n, h, bf.mo_eri(B, C), Delta, Pi)
    assert abs(E - Ebf) <= 1e-12 * max(1.0, abs(Ebf))


def test_closed_shell_hf_energy_and_fock():
    w = inputs.WORKLOADS["tiny"]
    B = inputs.make_B(w.seed, w.nbf, w.naux, w.decay, threads=1)
    C = inputs.make_C(w.seed, w.nbf, w.norb)
    H = inputs.make_H(w.seed, w.nbf)
    nocc = w.nstrong
    n = np.zeros(w.norb)
    n[:nocc] = 1.0
    Z = np.zeros((w.norb, w.norb))
    cJ, cK = dfjk.coeffs_from_cumulant(n, Z, Z)
    out = dfjk.iteration(B, C, H, n, cJ, cK)
    h, J, K = out["h"], out["J"], out["K"]
    occ = slice(0, nocc)
    E_hf = 2 * np.trace(h[occ, occ]) + np.sum(2 * J[occ, occ] - K[occ, occ])
    assert abs(out["E"] - E_hf) <= 1e-12 * abs(E_hf)
    F = C.T @ bf.ao_closed_shell_fock(H, B, C[:, :nocc]) @ C
    lam_ref = F * n[None, :]
    assert np.max(np.abs(out["lam"] - lam_ref)) <= 1e-12 * np.abs(F).max()
    g_ref = 4 * F * (n[None, :] - n[:, None])
    assert np.max(np.abs(out["g"] - g_ref)) <= 1e-12 * np.abs(F).max()


def _energy_of_C(B, C, H, n, cJ, cK):
    b, _ = dfjk.mo_transform(B, C)
    J, K = dfjk.jk(b)
    return dfjk.energy(n, dfjk.one_electron(H, C), J, K, cJ, cK)


@pytest.mark.parametrize("norb", [9, 6])
def test_lambda_against_unconstrained_finite_differences(norb):
    # 4 lambda = C^T dE/dC for arbitrary symmetric cJ, cK: pins every element.
    rng = np.random.default_rng(5)
    nbf = 9
    B, C, H = small_instance(4, nbf=nbf, naux=17, norb=norb)
    n = rng.uniform(0, 1, norb)
    cJ = rand_sym(rng, norb)
    cK = rand_sym(rng, norb)
    b, _ = dfjk.mo_transform(B, C)
    lam, g, _, _ = dfjk.gen_fock(b, n, dfjk.one_electron(H, C), cJ, cK)
    eps = 1e-5
    G = np.zeros_like(C)
    for mu in range(nbf):
        for s in range(norb):
            Cp = C.copy(); Cp[mu, s] += eps
            Cm = C.copy(); Cm[mu, s] -= eps
            G[mu, s] = (_energy_of_C(B, Cp, H, n, cJ, cK) - _energy_of_C(B, Cm, H, n, cJ, cK)) / (2 * eps)
    lam_fd = 0.25 * C.T @ G
    assert np.max(np.abs(lam - lam_fd)) <= 1e-7 * np.abs(lam).max()


def test_gradient_against_rotation_finite_differences():
    # g_pq = dE/dy_pq for C' = C exp(y), y antisymmetric (orbitals as columns)
    from scipy.linalg import expm
    rng = np.random.default_rng(9)
    B, C, H = small_instance(8, nbf=8, naux=20)
    m = 8
    n = rng.uniform(0, 1, m)
    Delta, Pi = rand_sym(rng, m, 0.2), rand_sym(rng, m, 0.2)
    cJ, cK = dfjk.coeffs_from_cumulant(n, Delta, Pi)
    b, _ = dfjk.mo_transform(B, C)
    _, g, _, _ = dfjk.gen_fock(b, n, dfjk.one_electron(H, C), cJ, cK)
    eps = 1e-5
    for (p, q) in [(0, 1), (2, 7), (5, 3), (6, 4)]:
        y = np.zeros((m, m)); y[p, q] = eps; y[q, p] = -eps
        Ep = _energy_of_C(B, C @ expm(y), H, n, cJ, cK)
        Em = _energy_of_C(B, C @ expm(-y), H, n, cJ, cK)
        fd = (Ep - Em) / (2 * eps)
        assert abs(fd - g[p, q]) <= 1e-7 * max(1.0, np.abs(g).max())


def test_linearity_in_coefficients():
    rng = np.random.default_rng(3)
    B, C, H = small_instance(2, nbf=10, naux=20)
    m = 10
    n = rng.uniform(0, 1, m)
    b, _ = dfjk.mo_transform(B, C)
    h = dfjk.one_electron(H, C)
    J, K = dfjk.jk(b)
    c1 = (rand_sym(rng, m), rand_sym(rng, m))
    c2 = (rand_sym(rng, m), rand_sym(rng, m))
    a, s = 0.7, -1.3
    c3 = (a * c1[0] + s * c2[0], a * c1[1] + s * c2[1])
    E0 = dfjk.energy(n, h, J, K, 0 * J, 0 * K)
    E1, E2, E3 = (dfjk.energy(n, h, J, K, *c) - E0 for c in (c1, c2, c3))
    assert abs(E3 - (a * E1 + s * E2)) <= 1e-12 * (abs(E1) + abs(E2))
    L0 = dfjk.gen_fock(b, n, h, 0 * J, 0 * K)[0]
    L1, L2, L3 = (dfjk.gen_fock(b, n, h, *c)[0] - L0 for c in (c1, c2, c3))
    assert np.max(np.abs(L3 - (a * L1 + s * L2))) <= 1e-12 * np.abs(L1).max()


def test_streamed_matches_in_memory():
    B, C, H = small_instance(6, nbf=11, naux=37)
    rng = np.random.default_rng(1)
    n = rng.uniform(0, 1, 11)
    cJ, cK = rand_sym(rng, 11), rand_sym(rng, 11)
    ref = dfjk.iteration(B, C, H, n, cJ, cK)
    st = dfjk.streamed_iteration(lambda lo, hi: B[lo:hi], 37, C, H, n, cJ, cK, pblock=5)
    for k in ("J", "K", "lam", "g"):
        assert np.allclose(st[k], ref[k], rtol=0, atol=1e-13 * np.abs(ref[k]).max())
    assert abs(st["E"] - ref["E"]) <= 1e-13 * abs(ref["E"])


def test_exchange_term_per_q_identity():
    """The identity behind the GPU route of the FP64 and INT8 exchange-type
    term: for symmetric b^P and symmetric cK,
        sum_P sum_q b^P_rq cK_sq b^P_qs = sum_q cK[q][s] G^q_rs,
        G^q_rs = sum_P b^P[q][r] b^P[q][s]   (each G^q symmetric),
    checked against the oracle's F2 by brute-force loops over the indices;
    with a non-symmetric cK the right side (which reads row q of cK) differs,
    so the route relies on the coefficient matrices' symmetry."""
    rng = np.random.default_rng(71)
    naux, norb = 5, 6
    b = rng.standard_normal((naux, norb, norb))
    b = 0.5 * (b + b.transpose(0, 2, 1))
    cK = rng.standard_normal((norb, norb))
    cK = cK + cK.T
    n = rng.uniform(0.0, 1.0, norb)
    _, _, _, F2 = dfjk.gen_fock(b, n, np.zeros((norb, norb)), np.zeros((norb, norb)), cK)
    G = np.zeros((norb, norb, norb))
    for q in range(norb):
        for r in range(norb):
            for s in range(norb):
                G[q, r, s] = sum(b[P, q, r] * b[P, q, s] for P in range(naux))
    assert np.array_equal(G, G.transpose(0, 2, 1))
    via = np.zeros((norb, norb))
    for r in range(norb):
        for s in range(norb):
            via[r, s] = sum(cK[q, s] * G[q, r, s] for q in range(norb))
    assert np.max(np.abs(via - F2)) <= 1e-12 * np.max(np.abs(F2))
    cA = cK + np.triu(rng.standard_normal((norb, norb)), 1)      # not symmetric
    _, _, _, F2a = dfjk.gen_fock(b, n, np.zeros((norb, norb)), np.zeros((norb, norb)), cA)
    via_a = np.einsum("qs,qrs->rs", cA, G)
    assert np.max(np.abs(via_a - F2a)) > 1e-3 * np.max(np.abs(F2a))
