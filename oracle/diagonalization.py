"""Iterative diagonalization of the generalized pseudo-Fockian (Natural
Orbital Optimization: the orbital-optimisation scheme selected by
IORBOPT = 1).

TEST INFRASTRUCTURE ONLY (see the package header).

At the minimum lambda is symmetric.  A symmetric matrix F whose off-diagonal
elements are the asymmetry of lambda is therefore diagonal there, and the
current orbitals are its eigenvectors; away from the minimum its
eigenvectors define the next orbitals.  The paper fixes the off-diagonal
elements only up to their orientation and leaves the diagonal open (no exact
expression exists).  Readings taken here:

* off-diagonal: F_pq = F_qp = s_pq (lambda_qp - lambda_pq) with
  s_pq = +1 when diag_p <= diag_q (p before q in the order of the diagonal),
  else -1.  To first order the eigenvectors then rotate the orbitals by
  y_pq = -g_pq / (4 |diag_q - diag_p|), g = 4 (lambda - lambda^T), a descent
  step for every pair whatever the orbitals' index order;
* every off-diagonal element is clamped to [-maxoff, maxoff] (damping of
  large early steps);
* diagonal: lambda_pp at the first step of a run, afterwards the
  eigenvalues of the previous step, each kept with its orbital;
* eigenvectors are matched to orbitals greedily by overlap: the largest
  |V_rk| among pairs whose orbital r and eigenvector k are both still free
  is taken first (ties to the smaller r, then the smaller k); each
  eigenvector gets a non-negative component on its orbital, so orbital roles
  survive the step;
* new orbitals C <- C V (orbitals as columns).

For 0/1 occupations with Delta = Pi = 0, lambda_rs = n_s F_rs with F the
closed-shell Fock matrix in the NO basis, so the occupied-virtual block of
this F is the Fock matrix's and the fixed point is the Roothaan SCF minimum.
"""
from __future__ import annotations

import numpy as np


def pseudo_fock(lam, diag, maxoff):
    """The generalized pseudo-Fockian of the readings above."""
    m = lam.shape[0]
    F = np.zeros((m, m))
    for p in range(m):
        F[p, p] = diag[p]
        for q in range(p + 1, m):
            s = 1.0 if diag[p] <= diag[q] else -1.0
            v = min(max(s * (lam[q, p] - lam[p, q]), -maxoff), maxoff)
            F[p, q] = v
            F[q, p] = v
    return F


def greedy_overlap_match(U):
    """orbital_of[k] for every eigenvector k (column of U): pairs (r, k) in
    decreasing |U_rk| (ties: smaller r, then smaller k), each taken when both
    r and k are still free."""
    m = U.shape[0]
    a = np.abs(U)
    order = sorted(((-a[r, k], r, k) for r in range(m) for k in range(m)))
    orbital_of = -np.ones(m, dtype=np.int64)
    row_used = np.zeros(m, dtype=bool)
    for _, r, k in order:
        if orbital_of[k] < 0 and not row_used[r]:
            orbital_of[k] = r
            row_used[r] = True
    return orbital_of


def diagonalize(F):
    """Eigenvalues and eigenvectors of the symmetric F, eigenvector k placed
    in column orbital_of[k] of the greedy overlap matching, signs fixed so
    that V_pp >= 0.  Returns (eigenvalues per orbital, V)."""
    w, U = np.linalg.eigh(F)
    orbital_of = greedy_overlap_match(U)
    V = np.empty_like(U)
    e = np.empty_like(w)
    V[:, orbital_of] = U
    e[orbital_of] = w
    sgn = np.where(np.diag(V) < 0.0, -1.0, 1.0)
    return e, V * sgn[None, :]


def step(C, lam, diag, maxoff):
    """One diagonalization step: returns (new C, new diagonal, V)."""
    if diag is None:
        diag = np.diag(lam).copy()
    e, V = diagonalize(pseudo_fock(lam, diag, maxoff))
    return C @ V, e, V
