"""Finite-field NLOP step on the GPU against the oracle.

- nof_nlop_romberg on the same dipoles: tables equal to 1e-13 relative
  (the same arithmetic in another order), identical selections.
- nof_dipole against the oracle's formula to 1e-12 relative.
- End to end, closed-shell HF on a kernel-on-grid tensor: nof_solve at each
  field of the ladder, nof_dipole, nof_nlop_romberg, against a Roothaan SCF
  at each field with the oracle's dipole and Romberg step.  The dipoles agree
  to the convergence of the two methods (~1e-10), which the differences
  amplify by 1/h, 1/h^2, 1/h^3 of the steps the selection uses; the bars are
  stated in the test.
"""
import numpy as np
import pytest
import torch

from oracle import nlop
from paper_2512_13550_amd import inputs
from gpu_util import dev, host, need_gpu
from _scf import scf_orbitals

pytestmark = pytest.mark.gpu


def test_romberg_matches_oracle():
    nof = need_gpu()
    print("case nlop romberg", flush=True)
    a, w, b = 1.3, 2.0, 0.7
    f = lambda F: a * np.sin(w * F) + b * F * F * np.exp(F) + 0.25
    for npoint, step in ((5, 1e-2), (3, 2e-3), (9, 1e-4), (1, 1e-2)):
        mu_p = np.array([f(step * 2.0 ** k) for k in range(npoint + 1)])
        mu_m = np.array([f(-step * 2.0 ** k) for k in range(npoint + 1)])
        ref = nlop.nlop(f(0.0), mu_p, mu_m, step, npoint)
        table, result = nof.nlop_romberg(dev(np.array(f(0.0))), dev(mu_p), dev(mu_m), step)
        torch.cuda.synchronize()
        T, Rs = host(table), host(result)
        for p in range(3):
            Rr = ref[p]["table"]
            assert np.array_equal(np.isnan(T[p]), np.isnan(Rr))
            ok = ~np.isnan(Rr)
            assert np.allclose(T[p][ok], Rr[ok], rtol=1e-13, atol=0)
            assert abs(Rs[p, 0] - ref[p]["value"]) <= 1e-13 * abs(ref[p]["value"])
            if npoint > 1:
                assert (int(Rs[p, 2]), int(Rs[p, 3])) == (ref[p]["k"], ref[p]["j"])
                # a difference of two table entries: compare on the scale of the entries
                assert abs(Rs[p, 1] - ref[p]["uncertainty"]) <= 1e-13 * np.max(np.abs(Rr[ok]))


def test_dipole_matches_oracle():
    nof = need_gpu()
    print("case nlop dipole", flush=True)
    nbf, norb = 70, 50
    C = inputs.make_C(4, nbf, norb)
    n = inputs.make_occupations(4, norb, 12)
    d = inputs.make_dipoles(4, nbf)[1]
    mu = float(nof.dipole(dev(C), dev(n), dev(d)))
    ref = nlop.dipole(C, n, d)
    assert abs(mu - ref) <= 1e-12 * max(1.0, abs(ref))


def test_hf_finite_field_end_to_end():
    nof = need_gpu()
    print("case nlop hf end to end", flush=True)
    nbf, naux, nocc = 16, 64, 4
    npoint, step = 3, 4e-3
    B = inputs.make_B_grid(nbf, naux, seed=2)
    H0 = inputs.make_H(2, nbf)
    d = inputs.make_dipoles(2, nbf)[2]
    fields = [0.0] + [s * step * 2.0 ** k for k in range(npoint + 1) for s in (1.0, -1.0)]
    members = torch.from_numpy(np.array(inputs.pairing(nbf, nocc, 1), dtype=np.int32)).cuda()
    C0, _ = scf_orbitals(B, H0, nocc)                 # start every field from the field-free minimum
    Bd, dd = dev(B), dev(d)
    mu_gpu, mu_ref = {}, {}
    for F in fields:
        H = H0 + F * d
        C = dev(C0)
        gamma = dev(np.zeros((nocc, 1)))
        n = torch.empty(nbf, dtype=torch.float64, device="cuda")
        # warm start at the field-free minimum: ADAM's first steps move every
        # component by ~lr whatever the gradient, so the rate is small here
        r = nof.solve(Bd, C, dev(H), members, nof.MAP_TRIG, nof.FUNC_HF, gamma, n=n, max_outer=3,
                      no_steps=4000, tol_lambda=1e-11, on_maxit=0, lr=1e-3)
        assert r["converged"] == 1, (F, r)
        mu_gpu[F] = float(nof.dipole(C, n, dd))
        Cs, ns = scf_orbitals(B, H, nocc)
        mu_ref[F] = nlop.dipole(Cs, ns, d)
    dmu = max(abs(mu_gpu[F] - mu_ref[F]) for F in fields)
    print("max |dmu|", dmu, flush=True)
    assert dmu <= 1e-9
    mp = np.array([mu_gpu[step * 2.0 ** k] for k in range(npoint + 1)])
    mm = np.array([mu_gpu[-step * 2.0 ** k] for k in range(npoint + 1)])
    table, result = nof.nlop_romberg(dev(np.array(mu_gpu[0.0])), dev(mp), dev(mm), step)
    Rs = host(result)
    ref = nlop.nlop(mu_ref[0.0], [mu_ref[step * 2.0 ** k] for k in range(npoint + 1)],
                    [mu_ref[-step * 2.0 ** k] for k in range(npoint + 1)], step, npoint)
    for p, name in enumerate(("alpha", "beta", "gamma")):
        print(name, Rs[p, 0], ref[p]["value"], "uncertainty", ref[p]["uncertainty"], flush=True)
    # bars: a dipole error e moves the estimates at step h by ~e/h, e/h^2, e/h^3;
    # with e <= 1e-9 and h >= step that is <= 2.5e-7, 6.3e-5, 1.6e-2
    e = 1e-9
    for p, scale in enumerate((1.0 / step, 1.0 / step ** 2, 1.0 / step ** 3)):
        assert abs(Rs[p, 0] - ref[p]["value"]) <= 4.0 * e * scale


def test_isotropic_matches_oracle():
    nof = need_gpu()
    print("case nlop isotropic", flush=True)
    for a in ((4.58, 4.58, 6.40), (1.0, 2.0, 3.0), (3.0, 3.0, 3.0)):
        out = host(nof.nlop_isotropic(dev(np.array(a))))
        ref = nlop.isotropic(*a)
        assert abs(out[0] - ref[0]) <= 1e-15 * abs(ref[0]) and abs(out[1] - ref[1]) <= 1e-14
