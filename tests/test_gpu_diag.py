"""Iterative diagonalization of the generalized pseudo-Fockian on the GPU
(nof_pseudo_fock_diag, and nof_solve with orbopt = 1) against the oracle
(oracle/diagonalization.py: the same pseudo-Fockian, numpy's symmetric
eigensolver, the same greedy overlap matching).

Bars: eigenvalues normwise 1e-12; V normwise within 50 eps ||F|| / (smallest
eigenvalue gap) (the first-order bound on eigenvectors that two correct
eigensolvers may differ by), at most 1e-9; the HF case reaches the
independent Roothaan SCF minimum to 1e-10; with the occupations fixed, a
PNOF5 run of diagonalization steps follows the oracle's to 1e-9 (with ON
steps in between, a softmax weak occupation driven toward zero lands at
n ~ 1e-13 on one side and 0 on the other -- a flat exponential tail where the
L-BFGS step scales with the inverse curvature -- which moves E by about
sqrt(n) K; the ON steps are compared with the oracle in their own tests)."""
import numpy as np
import pytest
import torch

from oracle import diagonalization, mlp, solver
from paper_2512_13550_amd import inputs
from gpu_util import dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu


def lam_case(m, seed, asym=0.05):
    """A Lagrangian with a spread diagonal, a symmetric part and a smaller
    antisymmetric part (the shape lambda has away from the minimum)."""
    rng = np.random.default_rng(seed)
    d = rng.permutation(np.linspace(-4.0, 1.0, m))
    S = rng.standard_normal((m, m))
    A = rng.standard_normal((m, m))
    return np.diag(d) + 0.05 * (S + S.T) + asym * (A - A.T)


@pytest.mark.parametrize("m,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (301, 4), (500, 5)])
@pytest.mark.parametrize("given_diag", [False, True])
def test_pseudo_fock_diag_matches_oracle(m, seed, given_diag):
    nof = need_gpu()
    print(f"case m={m} seed={seed} diag={given_diag}", flush=True)
    lam = lam_case(m, seed)
    diag = np.diag(lam) + 0.01 * np.random.default_rng(seed + 100).standard_normal(m) if given_diag else None
    F = diagonalization.pseudo_fock(lam, np.diag(lam) if diag is None else diag, 0.3)
    e_ref, V_ref = diagonalization.diagonalize(F)
    V, e, info = nof.pseudo_fock_diag(dev(lam), dev(diag) if given_diag else None, 0.3)
    torch.cuda.synchronize()
    inf = host(info)
    assert inf[0] >= 0 and inf[1] >= 1
    print("sweeps", inf[0], "matching rounds", inf[1], flush=True)
    gap = np.min(np.diff(np.sort(e_ref))) if m > 1 else 1.0
    tolV = min(1e-9, max(1e-12, 50 * 2.2e-16 * np.max(np.abs(e_ref)) / gap))
    print("V normwise", normwise(host(V), V_ref), "bound", tolV, flush=True)
    assert normwise(host(V), V_ref) <= tolV
    assert normwise(host(e), e_ref) <= 1e-12
    Vh = host(V)
    # accumulated rotations keep V orthogonal to a few m eps
    assert np.max(np.abs(Vh.T @ Vh - np.eye(m))) <= 4 * m * 2.2e-16 + 1e-15


def test_symmetric_lambda_is_a_fixed_point():
    nof = need_gpu()
    lam = lam_case(40, 9, asym=0.0)
    V, e, info = nof.pseudo_fock_diag(dev(lam), None, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(host(V), np.eye(40)) and np.array_equal(host(e), np.diag(lam))


def test_solve_iterative_diagonalization_hf_equals_roothaan_scf():
    """0/1 occupations: the GPU loop with orbopt = 1 reaches the minimum that
    the Roothaan SCF with DIIS finds independently."""
    nof = need_gpu()
    from _scf import scf_energy
    nbf, naux, nocc = 24, 96, 6
    B = inputs.make_B_grid(nbf, naux, seed=3)
    H = inputs.make_H(3, nbf)
    C = dev(inputs.make_C(3, nbf, nbf))
    members = np.array(inputs.pairing(nbf, nocc, 1), dtype=np.int32)
    g = dev(np.zeros((nocc, 1)))
    r = nof.solve(dev(B), C, dev(H), torch.from_numpy(members).cuda(), nof.MAP_TRIG, nof.FUNC_HF, g,
                  max_outer=3, no_steps=2000, tol_lambda=1e-8, on_maxit=0, orbopt=1, maxoff=1.0)
    E_scf = scf_energy(B, H, nocc)
    print("orbopt=1 HF", r["E"], "SCF", E_scf, "steps", r["no_steps"], flush=True)
    assert r["converged"] and r["status"] == 0
    assert abs(r["E"] - E_scf) <= 1e-10 * abs(E_scf)


def test_solve_iterative_diagonalization_trajectory_matches_oracle():
    """PNOF5, softmax map, occupations fixed at the cold start: two sweeps of
    eight diagonalization steps (the diagonal carried over between them)
    give the oracle's energies and orbitals."""
    nof = need_gpu()
    nbf, naux, ns, ng = 24, 96, 6, 2
    B = inputs.make_B_grid(nbf, naux, seed=5)
    H = inputs.make_H(5, nbf)
    C0 = inputs.make_C(5, nbf, nbf)
    members = np.array(inputs.pairing(nbf, ns, ng), dtype=np.int32)
    g0 = mlp.cold_gamma(members, "softmax")
    kw = dict(max_outer=2, no_steps=8, tol_lambda=0.0, tol_energy=0.0, orbopt=1, maxoff=1.0, on_maxit=0)
    ref = solver.solve(B, C0, H, members.astype(np.int64), "softmax", "pnof5", g0, **kw)
    C = dev(C0)
    g = dev(g0)
    r = nof.solve(dev(B), C, dev(H), torch.from_numpy(members).cuda(), nof.MAP_SOFTMAX, nof.FUNC_PNOF5, g, **kw)
    torch.cuda.synchronize()
    print("orbopt=1 PNOF5 E gpu", r["E"], "oracle", ref["E"], flush=True)
    assert abs(r["E"] - ref["E"]) <= 1e-9 * abs(ref["E"])
    assert normwise(host(C), ref["C"]) <= 1e-8
