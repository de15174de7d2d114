"""Orbital-rotation step (NO Optimization section).

The NOs are updated by a unitary transformation U = exp(y) of an
antisymmetric generator y (y_pq = -y_qp); with orbitals as the columns of C,
phi'_p = sum_q U_qp phi_q gives C' = C U.  The generator comes from ADAM
(first and second moments of the orbital gradient only).  The NOs are
orthonormal (the constraint of the Lagrangian of the same section); products
of rotations keep that only up to rounding, hence a check with a repair.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm as _expm


def expm_antisym(y: np.ndarray) -> np.ndarray:
    """U = exp(y) (library matrix exponential, Pade with scaling and squaring)."""
    return _expm(np.asarray(y, dtype=np.float64))


def rotate(C: np.ndarray, y: np.ndarray) -> np.ndarray:
    """C' = C exp(y)."""
    return C @ expm_antisym(y)


def adam_step(g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One ADAM step (Kingma and Ba 2015) on the orbital gradient g.

    Returns (y, m, v): the moments are updated from g alone and the step is
    y = -lr * mhat / (sqrt(vhat) + eps) with bias-corrected moments.
    """
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    y = -lr * mh / (np.sqrt(vh) + eps)
    return y, m, v


def orthonormality_error(C: np.ndarray, S: np.ndarray | None = None) -> np.ndarray:
    """E = C^T S C - I, S the AO overlap (None: an orthonormal AO basis)."""
    C = np.asarray(C, dtype=np.float64)
    SC = C if S is None else np.asarray(S, dtype=np.float64) @ C
    return C.T @ SC - np.eye(C.shape[1])


def orthonormalize(C: np.ndarray, S: np.ndarray | None = None, tol: float = 0.0):
    """Check and repair: err = max|E|; when err > tol one Newton-Schulz step of
    the polar decomposition, C <- C (I - E/2), which leaves an error of order
    err^2.  Returns (C, err)."""
    C = np.asarray(C, dtype=np.float64)
    E = orthonormality_error(C, S)
    err = float(np.max(np.abs(E)))
    if err > tol:
        C = C @ (np.eye(C.shape[1]) - 0.5 * E)
    return C, err
