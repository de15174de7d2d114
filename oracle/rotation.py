"""Orbital-rotation step (NO Optimization section).

The NOs are updated by a unitary transformation U = exp(y) of an
antisymmetric generator y (y_pq = -y_qp); with orbitals as the columns of C,
phi'_p = sum_q U_qp phi_q gives C' = C U.  The generator comes from ADAM
(first and second moments of the orbital gradient only).
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
