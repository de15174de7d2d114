"""Occupation-dependent coefficients of Eq. (PNOF) for the functionals used here.

The paper cites the explicit functionals out (Table 1 lists PNOF5, PNOF7, GNOF,
GNOFm).  Two reconstructions are provided, both in the (Delta, Pi) form of the
(2,2)-positivity cumulant (Theory: sigma-sigma and alpha-beta blocks), which
``dfjk.coeffs_from_cumulant`` turns into cJ = 2(nn^T - Delta) and
cK = nn^T - Delta - Pi:

* "hf":    Delta = Pi = 0 (the HF-like term of the cumulant expansion alone);
* "pnof5": the independent-pair model on the orbital-pairing structure
  (subspaces Omega_g of one strong and N_g weak orbitals, Eq. OmegaG):
  Delta_pq = n_p n_q and Pi_pq = sign * sqrt(n_p n_q) inside one subspace
  (sign -1 when the strong orbital is involved, +1 between two weak orbitals,
  Pi_pp = n_p), zero between subspaces.  The formulas follow the cited
  literature (parity unpinned as a functional; its energy is pinned against
  the exact two-electron two-orbital result and the spin-orbital 2RDM).
* "pnof7": PNOF5 inside each subspace plus the interpair static term of the
  cited literature: between orbitals of different subspaces Delta_pq = 0 and
  Pi_pq = -Phi_p Phi_q with Phi_p = sqrt(n_p (1 - n_p)), so the pair adds
  -Phi_p Phi_q K_pq (L = K for real orbitals) to the HF-like n_p n_q (2J - K).
  Parity unpinned as a functional (formulas outside the paper); pinned: it
  reduces to PNOF5 for one subspace and for 0/1 occupations, the interpair
  term only lowers E where K >= 0, and its gradient matches finite
  differences.

``members`` is an (ns, ng+1) integer array: row g lists the strong orbital of
subspace g first, then its weak orbitals.
"""
from __future__ import annotations

import numpy as np


def group_of(norb, members):
    grp = -np.ones(norb, dtype=np.int64)
    strong = np.zeros(norb, dtype=bool)
    for g, row in enumerate(members):
        grp[row] = g
        strong[row[0]] = True
    return grp, strong


def delta_pi(n, members, functional):
    m = len(n)
    if functional == "hf":
        return np.zeros((m, m)), np.zeros((m, m))
    if functional not in ("pnof5", "pnof7"):
        raise ValueError(functional)
    grp, strong = group_of(m, members)
    Delta = np.zeros((m, m))
    Pi = np.zeros((m, m))
    for row in members:
        for p in row:
            for q in row:
                Delta[p, q] = n[p] * n[q]
                if p == q:
                    Pi[p, q] = n[p]
                else:
                    sgn = -1.0 if (strong[p] or strong[q]) else 1.0
                    Pi[p, q] = sgn * np.sqrt(n[p] * n[q])
    if functional == "pnof7":
        phi = np.sqrt(n * (1.0 - n))
        inter = interpair_mask(grp)
        Pi[inter] = -np.outer(phi, phi)[inter]
    return Delta, Pi


def interpair_mask(grp):
    """[p, q] True when p and q belong to different subspaces."""
    return (grp[:, None] >= 0) & (grp[None, :] >= 0) & (grp[:, None] != grp[None, :])


def coefficients(n, members, functional):
    """cJ, cK of Eq. (PNOF) for the chosen functional."""
    from oracle.dfjk import coeffs_from_cumulant
    Delta, Pi = delta_pi(n, members, functional)
    return coeffs_from_cumulant(n, Delta, Pi)


def energy_of_n(n, hdiag, J, K, members, functional):
    """Eq. (PNOF) at fixed h, J, K as a function of the occupations."""
    cJ, cK = coefficients(n, members, functional)
    return float(2.0 * np.dot(n, hdiag) + np.sum(cJ * J) - np.sum(cK * K))


def denergy_dn(n, hdiag, J, K, members, functional, nfloor=1e-300):
    """dE/dn_r, differentiated by hand from the coefficient definitions."""
    M = 2.0 * J - K
    g = 2.0 * hdiag + 2.0 * (M @ n)                     # HF-like part, all pairs
    if functional == "hf":
        return g
    grp, strong = group_of(len(n), members)
    for row in members:
        for r in row:
            # remove the intra-subspace (and diagonal) pairs from the HF-like part
            for q in row:
                g[r] -= 2.0 * n[q] * M[r, q]
            # diagonal: -cK_rr K_rr with cK_rr = -n_r  ->  + n_r J_rr
            g[r] += J[r, r]
            # intra-subspace exchange: -sum_{q != r} cK_rq K_rq, cK_rq = -Pi_rq
            for q in row:
                if q == r:
                    continue
                sgn = -1.0 if (strong[r] or strong[q]) else 1.0
                g[r] += sgn * 0.5 * np.sqrt(n[q] / max(n[r], nfloor)) * K[r, q] * 2.0
    if functional == "pnof7":
        # interpair: -sum over ordered pairs of different subspaces of
        # Phi_p Phi_q K_pq; d/dn_r = -2 Phi_r' sum_{q not in r's subspace} Phi_q K_rq,
        # Phi_r' = (1 - 2 n_r) / (2 Phi_r)
        phi = np.sqrt(n * (1.0 - n))
        S = np.where(interpair_mask(grp), K, 0.0) @ phi
        for r in range(len(n)):
            if grp[r] >= 0:
                g[r] -= 2.0 * (1.0 - 2.0 * n[r]) / (2.0 * max(phi[r], nfloor)) * S[r]
    return g
