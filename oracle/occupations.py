"""Occupation-number (ON) mappings and optimisation (Occupation Number
Optimization section).

The ONs of each subspace Omega_g (one strong orbital g, N_g weak orbitals) are
expressed through N_g unconstrained variables so that the pairing sum rule of
Eq. (sum1), n_g + sum_i n_{p_i} = 1, and 0 <= n <= 1 hold automatically:

trigonometric:  n_g = (1 + cos^2 gamma_g) / 2, hole h_g = 1 - n_g,
                n_{p_i} = h_g cos^2 theta_1 ... cos^2 theta_{i-1} sin^2 theta_i (i < N_g),
                n_{p_Ng} = h_g cos^2 theta_1 ... cos^2 theta_{Ng-1};
                variables per subspace: (gamma_g, theta_1 .. theta_{Ng-1}).
softmax:        n_g = 1 / (1 + sum_k exp(gamma_k)), n_{p_i} = n_g exp(gamma_i);
                variables per subspace: (gamma_1 .. gamma_Ng).  Evaluated with
                numerator and denominator scaled by exp(-m), m = max(0, max_k
                gamma_k), so that no exponential overflows: the same values for
                every gamma, finite and summing to one also where exp(gamma_k)
                alone would overflow (gamma_k > 709).

gamma is stored (ns, ng).  The optimiser (parity reference for the GPU) is a
limited-memory BFGS with a backtracking Armijo line search.
"""
from __future__ import annotations

import numpy as np

from oracle import functionals


def occupations(gamma, members, norb, mapping):
    gamma = np.asarray(gamma, dtype=np.float64)
    ns, ng = gamma.shape
    n = np.zeros(norb)
    for g in range(ns):
        row = members[g]
        if mapping == "trig":
            ng_ = 0.5 * (1.0 + np.cos(gamma[g, 0]) ** 2)
            hole = 0.5 * np.sin(gamma[g, 0]) ** 2      # = 1 - n_g, without cancellation
            n[row[0]] = ng_
            P = 1.0
            for i in range(1, ng):
                th = gamma[g, i]
                n[row[i]] = hole * P * np.sin(th) ** 2
                P *= np.cos(th) ** 2
            n[row[ng]] = hole * P
        elif mapping == "softmax":
            m = max(0.0, float(np.max(gamma[g])))
            e = np.exp(gamma[g] - m)                  # every factor <= 1
            den = np.exp(-m) + e.sum()                # >= 1 term equal to 1
            n[row[0]] = np.exp(-m) / den
            n[row[1:]] = e / den
        else:
            raise ValueError(mapping)
    return n


def chain_rule(gamma, members, norb, mapping, dEdn):
    """dE/dgamma from dE/dn through the mapping's Jacobian (written out)."""
    gamma = np.asarray(gamma, dtype=np.float64)
    ns, ng = gamma.shape
    out = np.zeros_like(gamma)
    n = occupations(gamma, members, norb, mapping)
    for g in range(ns):
        row = members[g]
        gn = dEdn[row]
        if mapping == "softmax":
            nn_ = n[row]
            gbar = np.dot(gn, nn_)
            out[g] = nn_[1:] * (gn[1:] - gbar)
            continue
        cg, sg = np.cos(gamma[g, 0]), np.sin(gamma[g, 0])
        hole = 0.5 * sg * sg
        # weak part: n_{p_i} = hole * Pprev_i * t_i
        c = np.cos(gamma[g, 1:]); s = np.sin(gamma[g, 1:])
        t = np.append(s * s, 1.0)                     # t_i, i = 1..ng
        Pprev = np.ones(ng)                           # prod_{l < i} c_l^2
        for i in range(1, ng):
            Pprev[i] = Pprev[i - 1] * c[i - 1] ** 2
        gw = gn[1:]
        dE_dhole = float(np.sum(gw * Pprev * t))
        out[g, 0] = cg * sg * (dE_dhole - gn[0])
        # theta_j (j = 1..ng-1): reverse accumulation
        R = gw[ng - 1]                                # R_{ng-1} = g_ng
        for j in range(ng - 1, 0, -1):                # j = ng-1 .. 1
            out[g, j] = 2.0 * s[j - 1] * c[j - 1] * hole * Pprev[j - 1] * (gw[j - 1] - R)
            R = gw[j - 1] * t[j - 1] + c[j - 1] ** 2 * R
    return out


def energy_and_grad(gamma, members, norb, mapping, hdiag, J, K, functional):
    n = occupations(gamma, members, norb, mapping)
    E = functionals.energy_of_n(n, hdiag, J, K, members, functional)
    dn = functionals.denergy_dn(n, hdiag, J, K, members, functional)
    return E, chain_rule(gamma, members, norb, mapping, dn), n


# The trigonometric variables live on a box (see optimize_lbfgs); the
# softmax variables are unbounded.
TRIG_EDGE = 1e-12          # faces of the weak-orbital angles, and pi/2 for all
TRIG_STRONG_EDGE = 1e-6    # lower face of the strong-orbital angle gamma_g


def variable_bounds(mapping, shape=None):
    """Box of the optimiser's variables: the trigonometric map is even and
    pi-periodic in every angle, so [0, pi/2]^n reaches every occupation vector
    once, and the only points where E is not differentiable in the angles
    (a weak amplitude sqrt(n_p) = |sqrt(h_g) cos.. sin..| crossing zero, which
    PNOF5's sqrt(n_p n_q) terms turn into a kink) lie on its faces.  The faces
    are held TRIG_EDGE inside, where E and its gradient are finite and equal
    the one-sided limits to O(TRIG_EDGE).  The strong angle's lower face
    (h_g -> 0, n_g -> 1) is held TRIG_STRONG_EDGE inside: E falls linearly
    moving away from it (every K_gp >= 0), so no minimum lies there, and at
    1e-12 the hole 1 - n_g would be lost to rounding in n_g (PNOF7's
    sqrt(n_g (1 - n_g))).  Returns scalars without `shape`, else arrays of
    that (ns, ng) shape."""
    if mapping != "trig":
        return -np.inf, np.inf
    if shape is None:
        return TRIG_EDGE, 0.5 * np.pi - TRIG_EDGE
    lo = np.full(shape, TRIG_EDGE)
    lo[:, 0] = TRIG_STRONG_EDGE
    return lo, np.full(shape, 0.5 * np.pi - TRIG_EDGE)


def projected_gradient(x, g, lo, hi):
    """g with the components that push a variable out through a face it sits
    on set to zero (the first-order optimality measure of a box problem)."""
    pg = g.copy()
    pg[(x <= lo) & (g > 0.0)] = 0.0
    pg[(x >= hi) & (g < 0.0)] = 0.0
    return pg


def optimize_lbfgs(gamma0, members, norb, mapping, hdiag, J, K, functional, maxit=2000,
                   tol=1e-8, etol=1e-14, loose=1e-5, memory=8, c1=1e-4, max_backtrack=50,
                   step0=0.1):
    """Limited-memory BFGS (Nocedal, Math. Comp. 35 (1980)) on the box of
    ``variable_bounds``: the two-loop recursion over the last `memory` (s, y)
    pairs with initial scaling s.y / y.y acts on the projected gradient, the
    direction is zeroed on the variables held at a face, and a backtracking
    Armijo line search from step 1 (from `step0` / max|pg| on the first
    iteration or after a reset) projects every trial point onto the box and
    tests E_t <= E + c1 g.(x_t - x) (Bertsekas, projected quasi-Newton).  With
    no bounds (softmax) this is plain L-BFGS.  Pairs with s.y <= 0 are skipped;
    a non-descent direction, or a line search that needed half of its
    halvings, resets the memory.  Converged when max|pg| <= tol, or when
    max|pg| <= loose and two consecutive steps change E by at most
    etol * max(1, |E|) (the FP64 floor of the energy).

    Returns (gamma, n, E, iterations, converged)."""
    shape = np.shape(gamma0)
    lo, hi = variable_bounds(mapping, shape)
    if np.ndim(lo):
        lo, hi = lo.ravel(), hi.ravel()
    x = np.clip(np.array(gamma0, dtype=np.float64).ravel(), lo, hi)

    def f(v):
        E, g, n = energy_and_grad(v.reshape(shape), members, norb, mapping, hdiag, J, K, functional)
        return E, g.ravel(), n

    E, g, n = f(x)
    S, Y = [], []
    it = 0
    flat = 0
    pg = projected_gradient(x, g, lo, hi)
    while it < maxit and np.max(np.abs(pg)) > tol and flat < 2:
        held = pg != g                          # at a face, pushed outwards
        q = pg.copy()
        al = []
        for s_, y_ in zip(reversed(S), reversed(Y)):
            a = np.dot(s_, q) / np.dot(s_, y_)
            al.append(a)
            q = q - a * y_
        if S:
            r = q * (np.dot(S[-1], Y[-1]) / np.dot(Y[-1], Y[-1]))
        else:
            r = q * (step0 / np.max(np.abs(pg)))
        for (s_, y_), a in zip(zip(S, Y), reversed(al)):
            bcoef = np.dot(y_, r) / np.dot(s_, y_)
            r = r + s_ * (a - bcoef)
        d = -r
        d[held] = 0.0
        gd = float(np.dot(g, d))
        if not gd < 0.0:
            S, Y = [], []
            d = -pg * (step0 / np.max(np.abs(pg)))
        t = 1.0
        nb = 0
        for nb in range(max_backtrack):
            xt = np.clip(x + t * d, lo, hi)
            Et, gt, nt = f(xt)
            if Et <= E + c1 * float(np.dot(g, xt - x)):
                break
            t *= 0.5
        s_ = xt - x
        y_ = gt - g
        if nb >= max_backtrack // 2:
            S, Y = [], []                      # poor direction: restart the memory
        elif np.dot(s_, y_) > 0.0:
            S.append(s_); Y.append(y_)
            if len(S) > memory:
                S.pop(0); Y.pop(0)
        pgt = projected_gradient(xt, gt, lo, hi)
        small = np.max(np.abs(pgt)) <= loose
        flat = flat + 1 if (small and abs(Et - E) <= etol * max(1.0, abs(E))) else 0
        x, E, g, n, pg = xt, Et, gt, nt, pgt
        it += 1
    return x.reshape(shape), n, E, it, bool(np.max(np.abs(pg)) <= tol or flat >= 2)


def aufbau_members(hdiag, ns, ng):
    """Orbital roles from the one-electron energies: the ns lowest h_pp are the
    strong orbitals (ascending), the next ns*ng the weak ones, paired in the
    mirrored order of the pairing figure."""
    order = np.argsort(hdiag, kind="stable")
    members = np.zeros((ns, ng + 1), dtype=np.int64)
    for g in range(ns):
        members[g, 0] = order[g]
        for i in range(ng):
            members[g, 1 + i] = order[ns + (ns - 1 - g) + i * ns]
    return members


def inverse_trig(n, members, ng):
    """gamma with occupations(gamma) = n for a feasible n (n_g >= 1/2)."""
    gamma = np.zeros((len(members), ng))
    for g, row in enumerate(members):
        ngv = n[row[0]]
        gamma[g, 0] = np.arccos(np.sqrt(np.clip(2.0 * ngv - 1.0, 0.0, 1.0)))
        hole = 1.0 - ngv
        rem = hole
        for i in range(1, ng):
            frac = n[row[i]] / rem if rem > 0 else 0.0
            gamma[g, i] = np.arcsin(np.sqrt(np.clip(frac, 0.0, 1.0)))
            rem -= n[row[i]]
    return gamma
