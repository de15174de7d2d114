"""Independent brute-force routes used to pin the oracle (CPU only, tiny sizes).

None of these call the oracle.  They start from the paper's more primitive
definitions: four-index integrals (ERITYP='FULL' route), the spin-orbital
energy of Eq. (Energy) with the reconstructed 2RDM, and the textbook
closed-shell Fock operator in the AO basis.
"""
from __future__ import annotations

import numpy as np


def ao_eri(B):
    """(mu nu|lam sig) = sum_P B^P_mu,nu B^P_lam,sig (density-fitted four-index ERIs)."""
    nb = B.shape[1]
    Bf = B.reshape(B.shape[0], nb * nb)
    return (Bf.T @ Bf).reshape(nb, nb, nb, nb)


def mo_eri(B, C):
    """(pq|rs) by four quarter-transformations of the AO four-index tensor."""
    g = ao_eri(B)
    g = np.einsum("abcd,ap->pbcd", g, C)
    g = np.einsum("pbcd,bq->pqcd", g, C)
    g = np.einsum("pqcd,cr->pqrd", g, C)
    g = np.einsum("pqrd,ds->pqrs", g, C)
    return g


def spin_orbital_energy(n, h, eri, Delta, Pi):
    """E = sum_i n_i h_ii + sum_ijkl D_ijkl <kl|ij> over spin-orbitals.

    Spin-orbital i = (p, sigma), occupation n_p for either spin.  The 2RDM is
    the cumulant expansion D = (n_i n_j / 2)(d_ik d_jl - d_il d_jk) + lambda,
    with the sigma-sigma and alpha-beta cumulant blocks in terms of Delta and Pi;
    the beta-alpha block follows by exchanging the two particles.  <kl|ij> is
    (k i | l j) in chemists' notation, zero unless spin(k)=spin(i) and
    spin(l)=spin(j).  Spin-orbital index = 2*p + s (s=0 alpha, 1 beta).
    """
    m = len(n)
    M = 2 * m
    occ = np.repeat(n, 2)
    sp = np.tile([0, 1], m)
    orb = np.repeat(np.arange(m), 2)
    d = np.eye(M)
    Dm = np.zeros((M, M, M, M))
    # HF part
    Dm += 0.5 * np.einsum("i,j,ik,jl->ijkl", occ, occ, d, d)
    Dm -= 0.5 * np.einsum("i,j,il,jk->ijkl", occ, occ, d, d)
    # cumulant
    for i in range(M):
        for j in range(M):
            for k in range(M):
                for l in range(M):
                    si, sj, sk, sl = int(sp[i]), int(sp[j]), int(sp[k]), int(sp[l])
                    p, q, r, t = int(orb[i]), int(orb[j]), int(orb[k]), int(orb[l])
                    val = 0.0
                    if si == sj == sk == sl:
                        val = -0.5 * Delta[p, q] * (float(p == r and q == t) - float(p == t and q == r))
                    elif si == 0 and sj == 1 and sk == 0 and sl == 1:
                        val = -0.5 * Delta[p, q] * float(p == r and q == t) + 0.5 * Pi[p, r] * float(p == q and r == t)
                    elif si == 1 and sj == 0 and sk == 1 and sl == 0:
                        # beta-alpha: particles 1 and 2 exchanged in the alpha-beta block
                        val = -0.5 * Delta[q, p] * float(q == t and p == r) + 0.5 * Pi[q, t] * float(q == p and t == r)
                    Dm[i, j, k, l] += val
    # <kl|ij> = (k i|l j) with spin selection
    E1 = float(np.sum(occ * np.diag(h)[orb]))
    E2 = 0.0
    for i in range(M):
        for j in range(M):
            for k in range(M):
                if sp[k] != sp[i]:
                    continue
                for l in range(M):
                    if sp[l] != sp[j]:
                        continue
                    E2 += Dm[i, j, k, l] * eri[orb[k], orb[i], orb[l], orb[j]]
    return E1 + E2


def ao_closed_shell_fock(H, B, C_occ):
    """Textbook closed-shell Fock matrix in the AO basis, density-fitted:
    F = H + 2 J[P] - K[P],  P = C_occ C_occ^T,
    J[P] = sum_P B^P tr(B^P P),  K[P] = sum_P B^P P B^P."""
    Pd = C_occ @ C_occ.T
    F = H.copy()
    for BP in B:
        F += 2.0 * BP * np.sum(BP * Pd) - BP @ Pd @ BP
    return F


# ---- Fock-space brute force (occupation-number vectors, Jordan-Wigner signs) ----
# A state is a dict {bitmask: amplitude}; spin-orbital index 2*p + s (s = 0
# alpha, 1 beta).  Nothing here knows about cumulants or coefficient matrices.

def _annihilate(i, state):
    out = {}
    for det, a in state.items():
        if det >> i & 1:
            sign = -1.0 if bin(det & ((1 << i) - 1)).count("1") & 1 else 1.0
            d2 = det ^ (1 << i)
            out[d2] = out.get(d2, 0.0) + sign * a
    return out


def _create(i, state):
    out = {}
    for det, a in state.items():
        if not det >> i & 1:
            sign = -1.0 if bin(det & ((1 << i) - 1)).count("1") & 1 else 1.0
            d2 = det | (1 << i)
            out[d2] = out.get(d2, 0.0) + sign * a
    return out


def _inner(x, y):
    return sum(a * y.get(d, 0.0) for d, a in x.items())


def geminal_product_state(groups, coeffs):
    """Psi = prod_g (sum_{p in group g} c_p a+_{p alpha} a+_{p beta}) |0>:
    an antisymmetrized product of strongly orthogonal singlet geminals, each in
    its natural-orbital (Lowdin-Shull) form."""
    psi = {0: 1.0}
    for grp in groups:
        new = {}
        for p in grp:
            t = _create(2 * p, _create(2 * p + 1, psi))
            for d, a in t.items():
                new[d] = new.get(d, 0.0) + coeffs[p] * a
        psi = new
    return psi


def expectation_energy(psi, h, eri):
    """<Psi|H|Psi> with H = sum h_pq a+_p,s a_q,s + 1/2 sum (pq|rs) a+_p,s a+_r,t a_s,t a_q,s
    (chemists' notation (pq|rs)), by applying the operators to the state."""
    m = h.shape[0]
    M = 2 * m
    one = {i: _annihilate(i, psi) for i in range(M)}
    two = {(i, j): _annihilate(i, one[j]) for i in range(M) for j in range(M)}   # a_i a_j Psi
    E = 0.0
    for i in range(M):
        for j in range(M):
            if i % 2 == j % 2:
                E += h[i // 2, j // 2] * _inner(one[i], one[j])
    for p in range(M):
        for q in range(M):
            if p % 2 != q % 2:
                continue
            for r in range(M):
                for s in range(M):
                    if r % 2 != s % 2:
                        continue
                    v = eri[p // 2, q // 2, r // 2, s // 2]
                    if v != 0.0:
                        # <Psi| a+_p a+_r a_s a_q |Psi> = <a_r a_p Psi | a_s a_q Psi>
                        E += 0.5 * v * _inner(two[(r, p)], two[(s, q)])
    return E, _inner(psi, psi)
