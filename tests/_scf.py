"""Closed-shell Roothaan SCF with DIIS (Pulay, Chem. Phys. Lett. 73 (1980)) in
an orthonormal AO basis with the fitted three-index tensor B: the textbook
reference for the HF minimum of the orbital optimisation."""
import numpy as np


def scf_energy(B, H, nocc, iters=300):
    e, V = np.linalg.eigh(H)
    Cocc = V[:, :nocc]
    Fs, errs = [], []
    E_old = None
    for _ in range(iters):
        D = Cocc @ Cocc.T
        Jm = np.einsum("Pmn,P->mn", B, 2.0 * np.einsum("Pab,ab->P", B, D))
        Km = np.einsum("Pma,ab,Pbn->mn", B, D, B)
        F = H + Jm - Km
        E = float(np.sum(D * (2.0 * H + Jm - Km)))
        err = F @ D - D @ F
        Fs, errs = (Fs + [F])[-8:], (errs + [err])[-8:]
        k = len(Fs)
        A = -np.ones((k + 1, k + 1))
        A[k, k] = 0.0
        for i in range(k):
            for j in range(k):
                A[i, j] = np.sum(errs[i] * errs[j])
        rhs = np.zeros(k + 1)
        rhs[k] = -1.0
        c = np.linalg.solve(A, rhs)[:k]
        _, V = np.linalg.eigh(sum(ci * Fi for ci, Fi in zip(c, Fs)))
        Cocc = V[:, :nocc]
        if E_old is not None and abs(E - E_old) < 1e-13 and np.max(np.abs(err)) < 1e-10:
            return E
        E_old = E
    raise AssertionError("SCF did not converge")


def scf_orbitals(B, H, nocc, iters=300):
    """All orbitals of the closed-shell SCF minimum (eigenvectors of the
    converged Fock matrix, ascending) and the 0/1 occupations."""
    e, V = np.linalg.eigh(H)
    Cocc = V[:, :nocc]
    for _ in range(iters):
        D = Cocc @ Cocc.T
        Jm = np.einsum("Pmn,P->mn", B, 2.0 * np.einsum("Pab,ab->P", B, D))
        Km = np.einsum("Pma,ab,Pbn->mn", B, D, B)
        F = H + Jm - Km
        e, V = np.linalg.eigh(F)
        new = V[:, :nocc]
        if np.max(np.abs(new @ new.T - D)) < 1e-13:
            break
        Cocc = new
    n = np.zeros(V.shape[1])
    n[:nocc] = 1.0
    return V, n
