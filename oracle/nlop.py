"""Static polarizability and hyperpolarizabilities from finite fields (NLOPs:
Polarizabilities and Hyperpolarizabilities).

TEST INFRASTRUCTURE ONLY (see the package header).

The field F along one axis enters the one-electron matrix as H(F) = H + F d,
with d the AO matrix of the field coupling (minus the dipole operator), so
the electronic dipole of the converged state is
    mu(F) = -2 sum_p n_p (C^T d C)_pp
(Hellmann-Feynman: mu = -dE/dF at the minimum).  The responses are
alpha = dmu/dF, beta = d^2mu/dF^2, gamma = d^3mu/dF^3 at F = 0, estimated by
the centred differences of the paper on the dyadic ladder h_k = step 2^(k-1),
then refined by the Romberg-Richardson triangle with p = 2 and the paper's
selection of the smallest vertical difference.
"""
from __future__ import annotations

import numpy as np


def dipole(C, n, d):
    """mu = -2 sum_p n_p (C^T d C)_pp."""
    return float(-2.0 * np.dot(n, np.diag(C.T @ d @ C)))


def estimates(prop, mu0, at_h, at_2h, h):
    """Centred finite-difference estimate of property prop (0 alpha, 1 beta,
    2 gamma) at step h from mu(0), at_h = (mu(+h), mu(-h)) and
    at_2h = (mu(+2h), mu(-2h))."""
    mp, mm = at_h
    m2p, m2m = at_2h
    if prop == 0:
        return (mp - mm) / (2.0 * h)
    if prop == 1:
        return (mp - 2.0 * mu0 + mm) / (h * h)
    return (m2p - 2.0 * mp + 2.0 * mm - m2m) / (2.0 * h ** 3)


def romberg(D):
    """Romberg triangle of the first column D[k] = D(h_k) (h_{k+1} = 2 h_k):
    R[k][j] = R[k][j-1] + (R[k][j-1] - R[k+1][j-1]) / (4^j - 1) (0-based j),
    defined for k + j < len(D); other entries are NaN."""
    m = len(D)
    R = np.full((m, m), np.nan)
    R[:, 0] = D
    for j in range(1, m):
        for k in range(m - j):
            R[k, j] = R[k, j - 1] + (R[k, j - 1] - R[k + 1, j - 1]) / (4.0 ** j - 1.0)
    return R


def select(R):
    """The paper's selection: over every vertical pair (k, k+1) of every column
    j that has a next column, the pair with the smallest |R[k+1][j] - R[k][j]|;
    the value is R[k][j+1] and that difference its uncertainty.  Equal
    differences: the candidate of smallest absolute value.
    Returns (value, uncertainty, k, j) with 0-based k, j of the pair."""
    m = R.shape[0]
    if m == 1:
        return R[0, 0], float("nan"), 0, 0
    best = None
    for j in range(m - 1):
        for k in range(m - j - 1):
            delta = abs(R[k + 1, j] - R[k, j])
            cand = R[k, j + 1]
            key = (delta, abs(cand))
            if best is None or key < best[0]:
                best = (key, cand, delta, k, j)
    return best[1], best[2], best[3], best[4]


def nlop(mu0, mu_p, mu_m, step, npoint):
    """alpha, beta, gamma from mu(0) and mu(+-h_k), h_k = step 2^(k-1),
    k = 1 .. npoint + 1 (mu_p[k-1] = mu(+h_k), mu_m[k-1] = mu(-h_k)); the
    ladder uses the npoint steps h_1 .. h_npoint (2 h_k = h_{k+1}).
    Returns a list of three dicts (table, value, uncertainty, k, j)."""
    out = []
    for prop in range(3):
        D = []
        for k in range(npoint):
            h = step * 2.0 ** k
            D.append(estimates(prop, mu0, (mu_p[k], mu_m[k]), (mu_p[k + 1], mu_m[k + 1]), h))
        R = romberg(np.array(D))
        v, dlt, kk, jj = select(R)
        out.append(dict(table=R, value=v, uncertainty=dlt, k=kk, j=jj))
    return out


def isotropic(axx, ayy, azz):
    """Isotropic polarizability and its anisotropy (Raman convention)."""
    mean = (axx + ayy + azz) / 3.0
    aniso = np.sqrt(((axx - ayy) ** 2 + (ayy - azz) ** 2 + (azz - axx) ** 2) / 2.0)
    return mean, aniso
