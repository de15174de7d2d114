"""The alternating NO + ON optimisation to convergence (Theory: the energy is
minimised separately over occupations and orbitals; Occupation Number
Optimization; Natural Orbital Optimization).

TEST INFRASTRUCTURE ONLY (see the package header).

One outer iteration:
  1. ON step at fixed orbitals: b = C^T B C, h = C^T H C, J, K; the auxiliary
     variables gamma are optimised with the L-BFGS of ``occupations``; the
     coefficients cJ(n), cK(n) follow.
  2. NO sweep at fixed occupations: up to ``no_steps`` ADAM steps on the
     antisymmetric generator, each from the orbital gradient
     g = 4(lambda - lambda^T) of the current orbitals, U = exp(y), C <- C U.
     The sweep stops early once max|lambda - lambda^T| <= tol_lambda (the
     symmetry of the Lagrange multipliers at the minimum, monitored by
     NTHRESHL).
  3. Orthonormality check of the orbitals after the sweep: max|C^T C - I|,
     and one Newton-Schulz repair step when it exceeds tol_orth.
The loop ends when a sweep ends on the symmetry criterion and the energy
changed by at most tol_energy since the previous outer iteration (NTHRESHE),
or after ``max_outer`` iterations.

Readings (the ADAM details are cited out of the paper): the moments persist
over the whole run (one global step counter for the bias correction), the
learning rate is constant; the first NO step of a sweep reuses the integrals
of the ON step (the orbitals have not changed).

orbopt = 1 replaces the ADAM step by one step of the iterative
diagonalization of the generalized pseudo-Fockian (``diagonalization``);
its diagonal persists over the run like the ADAM moments.
"""
from __future__ import annotations

import numpy as np

from oracle import dfjk, diagonalization, functionals, occupations, rotation


def solve(B, C, H, members, mapping, functional, gamma, max_outer=100, no_steps=30, lr=0.01,
          beta1=0.9, beta2=0.999, eps=1e-8, tol_lambda=1e-5, tol_energy=1e-9, on_maxit=2000,
          on_tol=1e-8, tol_orth=1e-10, history=None, orbopt=2, maxoff=1.0):
    """Returns dict(C, gamma, n, E, asym, outer, no_steps, converged, orth,
    on_unconverged); orth is the largest max|C^T C - I| the checks found,
    on_unconverged the number of ON steps that stopped at on_maxit without
    meeting their test; converged needs the last ON step converged."""
    C = np.array(C, dtype=np.float64)
    gamma = np.array(gamma, dtype=np.float64)
    norb = C.shape[1]
    m = np.zeros((norb, norb))
    v = np.zeros((norb, norb))
    t_global = 0
    steps = 0
    E_prev = None
    converged = False
    E = asym = None
    orth = 0.0
    on_unconverged = 0
    diag = None
    n = occupations.occupations(gamma, members, norb, mapping)
    for outer in range(max_outer):
        b, _ = dfjk.mo_transform(B, C)
        h = dfjk.one_electron(H, C)
        J, K = dfjk.jk(b)
        on_ok = True
        if on_maxit > 0:
            gamma, n, _, _, on_ok = occupations.optimize_lbfgs(gamma, members, norb, mapping, np.diag(h),
                                                               J, K, functional, maxit=on_maxit, tol=on_tol)
            on_unconverged += 0 if on_ok else 1
        cJ, cK = functionals.coefficients(n, members, functional)
        for t in range(no_steps):
            if t > 0:
                b, _ = dfjk.mo_transform(B, C)
                h = dfjk.one_electron(H, C)
                J, K = dfjk.jk(b)
            E = dfjk.energy(n, h, J, K, cJ, cK)
            lam, g, _, _ = dfjk.gen_fock(b, n, h, cJ, cK)
            asym = float(np.max(np.abs(lam - lam.T)))
            if asym <= tol_lambda:
                break
            t_global += 1
            steps += 1
            if orbopt == 1:
                C, diag, _ = diagonalization.step(C, lam, diag, maxoff)
            else:
                y, m, v = rotation.adam_step(g, m, v, t_global, lr=lr, beta1=beta1, beta2=beta2, eps=eps)
                C = rotation.rotate(C, y)
        C, err = rotation.orthonormalize(C, tol=tol_orth)
        orth = max(orth, err)
        if history is not None:
            history.append((E, asym))
        if on_ok and asym <= tol_lambda and E_prev is not None and abs(E - E_prev) <= tol_energy:
            converged = True
            break
        E_prev = E
    return dict(C=C, gamma=gamma, n=n, E=E, asym=asym, outer=outer + 1, no_steps=steps,
                converged=converged, orth=orth, on_unconverged=on_unconverged)
