"""Pins of the finite-field NLOP step (oracle/nlop.py).

- Polynomial dipoles: for mu(F) a polynomial of degree 5 the centred
  differences carry errors in h^2 and h^4 only, so the third Romberg column is
  exact and the selected values equal alpha = mu'(0), beta = mu''(0) and
  gamma = mu'''(0) to rounding.
- A smooth non-polynomial mu(F) = a sin(wF) + b F^2 e^F: the selected values
  approach the analytic derivatives far below the first-column error.
- The selection rule on a hand-made triangle (smallest vertical difference,
  value from the next column, ties to the smallest magnitude).
- The dipole formula against Hellmann-Feynman: at the closed-shell SCF
  minimum mu(F) = -dE/dF, checked by a centred difference of SCF energies.
- Isotropic average and anisotropy closed forms.
"""
import math

import numpy as np
import pytest

from oracle import nlop
from paper_2512_13550_amd import inputs
from _scf import scf_energy, scf_orbitals


def ladder(f, step, npoint):
    mu_p = [f(step * 2.0 ** k) for k in range(npoint + 1)]
    mu_m = [f(-step * 2.0 ** k) for k in range(npoint + 1)]
    return f(0.0), mu_p, mu_m


def test_polynomial_dipole_is_exact():
    c = [0.3, 4.2, -1.7, 35.0, 11.0, -80.0]          # mu = sum c_i F^i
    f = lambda F: sum(ci * F ** i for i, ci in enumerate(c))
    mu0, mp, mm = ladder(f, 1e-3, 5)
    res = nlop.nlop(mu0, mp, mm, 1e-3, 5)
    exact = [c[1], 2.0 * c[2], 6.0 * c[3]]
    for r, e in zip(res, exact):
        assert abs(r["value"] - e) <= 1e-6 * max(1.0, abs(e)), (r["value"], e)
        assert abs(r["table"][0, 2] - e) <= 1e-6 * max(1.0, abs(e))


def test_smooth_dipole_converges():
    a, w, b = 1.3, 2.0, 0.7
    f = lambda F: a * math.sin(w * F) + b * F * F * math.exp(F)
    exact = [a * w, 2.0 * b, -a * w ** 3 + 6.0 * b]   # derivatives at 0
    mu0, mp, mm = ladder(f, 1e-2, 6)
    res = nlop.nlop(mu0, mp, mm, 1e-2, 6)
    for r, e in zip(res, exact):
        first_col_err = abs(r["table"][0, 0] - e)
        assert abs(r["value"] - e) <= max(1e-3 * first_col_err, 1e-7 * abs(e)), (r["value"], e)


def test_selection_rule():
    R = np.full((3, 3), np.nan)
    R[:, 0] = [1.0, 1.5, 3.0]          # vertical differences 0.5, 1.5
    R[:2, 1] = [0.75, 1.0]             # difference 0.25 (smallest)
    R[0, 2] = 0.875
    v, d, k, j = nlop.select(R)
    assert (v, d, k, j) == (0.875, 0.25, 0, 1)
    # a tie between two pairs: the smaller candidate value wins
    R = np.full((3, 3), np.nan)
    R[:, 0] = [1.0, 1.25, 1.5]         # two pairs, both 0.25
    R[:2, 1] = [2.0, -0.5]             # candidates of column 0: 2.0 (k=0), -0.5 (k=1); difference 2.5
    R[0, 2] = 7.0
    v, d, k, j = nlop.select(R)
    assert (v, d, k, j) == (-0.5, 0.25, 1, 0)
    # the Romberg recursion itself: a first column D(h) = A + c h^2 with
    # h doubling down the column extrapolates to A in the second column
    A, c = 2.5, 3.0
    D = np.array([A + c * (0.1 * 2 ** k) ** 2 for k in range(4)])
    assert np.allclose(nlop.romberg(D)[:3, 1], A, rtol=0, atol=1e-14)


def test_dipole_is_minus_energy_derivative_at_scf_minimum():
    nbf, nocc = 16, 4
    B = inputs.make_B_grid(nbf, 64, seed=2)
    H = inputs.make_H(2, nbf)
    d = inputs.make_dipoles(2, nbf)[2]
    h = 1e-4
    Ep = scf_energy(B, H + h * d, nocc)
    Em = scf_energy(B, H - h * d, nocc)
    # orbitals of the field-free SCF minimum (the occupied eigenvectors of F)
    C, n = scf_orbitals(B, H, nocc)
    mu = nlop.dipole(C, n, d)
    assert abs(mu - (-(Ep - Em) / (2.0 * h))) <= 1e-7 * max(1.0, abs(mu))


def test_isotropic_closed_forms():
    mean, aniso = nlop.isotropic(4.58, 4.58, 6.40)
    assert abs(mean - (4.58 * 2 + 6.40) / 3) < 1e-15
    assert abs(aniso - abs(6.40 - 4.58)) < 1e-14          # axial: |a_par - a_perp|
    assert nlop.isotropic(3.0, 3.0, 3.0) == (3.0, 0.0)


def test_single_point_ladder_is_the_centred_difference():
    """With one step there is no vertical pair to select from: the value is
    the centred difference itself (mu quadratic in F: alpha and beta exact)."""
    f = lambda F: 0.25 + 3.0 * F - 0.5 * F * F      # dyadic: every step exact
    mu0, mp, mm = ladder(f, 0.25, 1)
    res = nlop.nlop(mu0, mp, mm, 0.25, 1)
    assert res[0]["value"] == 3.0 and res[1]["value"] == -1.0 and res[2]["value"] == 0.0
    assert all(math.isnan(r["uncertainty"]) and (r["k"], r["j"]) == (0, 0) for r in res)


def test_printed_stencils_and_romberg_constants():
    """The oracle's finite differences and Romberg recursion against the
    constants the paper prints (tests/golden/nlop_formulas.json): each
    stencil's weights are read off the oracle by feeding it unit dipoles, the
    Romberg denominators by a first column with one unit entry."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "nlop_formulas.json")))
    h = 0.5                       # a power of two: the weights come back exact
    offsets_all = [0, 1, -1, 2, -2]
    for prop, name in enumerate(("alpha", "beta", "gamma")):
        st = g["stencils"][name]
        got = {}
        for off in offsets_all:
            mu = {o: 0.0 for o in offsets_all}
            mu[off] = 1.0
            val = nlop.estimates(prop, mu[0], (mu[1], mu[-1]), (mu[2], mu[-2]), h)
            got[off] = val * st["divisor"] * h ** st["power"]
        ref = {o: 0.0 for o in offsets_all}
        for o, w in zip(st["offsets"], st["weights"]):
            ref[o] = float(w)
        assert got == ref, (name, got, ref)
    # R(1, j) from a first column that is 1 at k = 1 and 0 elsewhere: column j
    # (1-based) scales the previous one by 1 + 1/(4^(j-1) - 1)
    D = np.zeros(9)
    D[0] = 1.0
    R = nlop.romberg(D)
    for j, den in enumerate(g["romberg"]["denominators_j2_to_j9"], start=1):
        assert abs(R[0, j] / R[0, j - 1] - (1.0 + 1.0 / den)) <= 4e-16
    # ladder
    lad = g["ladder"]
    hk = [lad["default_STEP"] * 2.0 ** k for k in range(lad["default_NPOINT"])]
    assert np.allclose(hk, lad["h_default"], rtol=0, atol=1e-18)
