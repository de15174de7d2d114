"""Density-fitted JK build and generalized-Fock contraction in the NO basis.

Notation (DoNOF 2.0, Theory): orbitals p,q,r,s; auxiliary index P;
b^P_pq = (C^T B^P C)_pq is the RI three-index tensor in the NO basis
(Single Point Energy Calculations, ERITYP='RI'); D[P][p] = b^P_pp.
J_pq = (pp|qq) and K_pq = (pq|qp) are the Coulomb and exchange integrals of
Eq. (PNOF); for real orbitals the time-inversion integral L equals K.

Every function is the plain definition written out in FP64.
"""
from __future__ import annotations

import numpy as np


def mo_transform(B: np.ndarray, C: np.ndarray):
    """b^P = C^T B^P C for every P, and D[P][p] = b^P_pp.

    The orbital transformation of the RI route (Single Point Energy
    Calculations, ERITYP='RI'): the AO three-index tensor B[P][mu][nu] is
    carried into the NO basis whose coefficients are the columns of C
    (phi_p = sum_mu C_mu,p chi_mu, NO Optimization).
    """
    B = np.asarray(B, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    T = np.matmul(B, C)                   # T^P = B^P C
    b = np.matmul(C.T, T)                 # b^P = C^T T^P
    D = np.ascontiguousarray(np.diagonal(b, axis1=1, axis2=2))
    return b, D


def one_electron(H: np.ndarray, C: np.ndarray) -> np.ndarray:
    """h = C^T H C: the one-electron integrals h_pq of Eq. (Energy) in the NO basis."""
    return C.T @ H @ C


def jk(b: np.ndarray):
    """J_pq = sum_P b^P_pp b^P_qq and K_pq = sum_P (b^P_pq)^2."""
    D = np.diagonal(b, axis1=1, axis2=2)
    J = D.T @ D
    K = np.einsum("Ppq,Ppq->pq", b, b)
    return J, K


def coeffs_from_cumulant(n: np.ndarray, Delta: np.ndarray, Pi: np.ndarray):
    """cJ = A and cK = B + C of Eq. (PNOF) from the cumulant matrices Delta, Pi.

    Inserting the cumulant expansion of the 2RDM (Theory: HF term plus the
    (2,2)-positivity cumulant with the sigma-sigma and alpha-beta blocks built
    from Delta and Pi) into Eq. (ENOF) gives
        E_ee = sum_pq [2(n_p n_q - Delta_pq) J_pq - (n_p n_q - Delta_pq) K_pq
                       + Pi_pq L_pq],
    so A = 2(nn^T - Delta), B = nn^T - Delta, C = -Pi, and with L = K the
    exchange-type coefficient is cK = nn^T - Delta - Pi.
    """
    nn = np.outer(n, n)
    cJ = 2.0 * (nn - Delta)
    cK = nn - Delta - Pi
    return cJ, cK


def energy(n, h, J, K, cJ, cK) -> float:
    """E = 2 sum_p n_p h_pp + sum_pq cJ_pq J_pq - sum_pq cK_pq K_pq   (Eq. PNOF)."""
    return float(2.0 * np.dot(n, np.diag(h)) + np.sum(cJ * J) - np.sum(cK * K))


def gen_fock(b, n, h, cJ, cK):
    """Lagrange multipliers lambda and orbital gradient g (NO Optimization).

    lambda is defined by the stationarity of the Lagrangian
    L = E - 2 sum_pq lambda_qp (<phi_p|phi_q> - delta_pq), i.e.
    4 lambda = C^T dE/dC.  Differentiating Eq. (PNOF) with J = D^T D and
    K = sum_P b^P o b^P (cJ, cK symmetric) gives
        lambda_rs = n_s h_rs + sum_P b^P_rs W[P][s]
                    - sum_P sum_q b^P_rq cK_sq b^P_qs,
        W = D cJ,
    and the gradient with respect to the antisymmetric rotation generator is
    g_pq = 4 (lambda_pq - lambda_qp).
    Returns (lambda, g, F1, F2) with F1 the Coulomb-type and F2 the
    exchange-type sum.
    """
    D = np.diagonal(b, axis1=1, axis2=2)
    W = D @ cJ                                            # W[P][s]
    F1 = np.einsum("Prs,Ps->rs", b, W)
    F2 = np.zeros_like(h)
    for P in range(b.shape[0]):
        F2 += b[P] @ (cK.T * b[P])                        # (cK_sq b_qs) indexed [q][s]
    lam = h * n[None, :] + F1 - F2
    g = 4.0 * (lam - lam.T)
    return lam, g, F1, F2


def iteration(B, C, H, n, cJ, cK):
    """One orbital-optimisation pass: transform, J/K, energy, lambda and g."""
    b, D = mo_transform(B, C)
    h = one_electron(H, C)
    J, K = jk(b)
    E = energy(n, h, J, K, cJ, cK)
    lam, g, F1, F2 = gen_fock(b, n, h, cJ, cK)
    return dict(b=b, D=D, h=h, J=J, K=K, E=E, lam=lam, g=g, F1=F1, F2=F2)


# ---------------------------------------------------------------------------
# Slab-streamed forms for inputs too large to hold b in host memory.  They
# compute exactly the definitions above, P slab by P slab.
# ---------------------------------------------------------------------------
def streamed_iteration(B_slab, naux, C, H, n, cJ, cK, want_fock=True, pblock=64):
    """Same results as ``iteration`` with B supplied one slab range at a time.

    ``B_slab(lo, hi)`` returns B[lo:hi] as float64.  Only b for one slab range
    is held at a time.  Returns J, K, E, lambda, g (no b).
    """
    norb = C.shape[1]
    h = one_electron(H, C)
    J = np.zeros((norb, norb))
    K = np.zeros((norb, norb))
    F1 = np.zeros((norb, norb))
    F2 = np.zeros((norb, norb))
    Dall = np.empty((naux, norb))
    for lo in range(0, naux, pblock):
        hi = min(naux, lo + pblock)
        b, D = mo_transform(B_slab(lo, hi), C)
        Dall[lo:hi] = D
        K += np.einsum("Ppq,Ppq->pq", b, b)
        if want_fock:
            W = D @ cJ
            F1 += np.einsum("Prs,Ps->rs", b, W)
            for P in range(hi - lo):
                F2 += b[P] @ (cK.T * b[P])
    J = Dall.T @ Dall
    E = energy(n, h, J, K, cJ, cK)
    out = dict(h=h, J=J, K=K, E=E, D=Dall)
    if want_fock:
        lam = h * n[None, :] + F1 - F2
        out.update(lam=lam, g=4.0 * (lam - lam.T), F1=F1, F2=F2)
    return out
