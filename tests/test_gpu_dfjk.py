"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Bar (FP64): normwise relative error <= 1e-10 for b, D, h, J, K, lambda, g and
|dE|/|E| <= 1e-10.  FP32 storage + FP32 matrix-core arithmetic: the stated
per-result bounds below.
"""
import numpy as np
import pytest
import torch

from oracle import dfjk
from paper_2512_13550_amd import inputs
from gpu_util import case, dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10

SHAPES = [
    # (nbf, naux, norb, seed): tiny workload, ragged multi-tile, rectangular C, degenerate
    (48, 192, 48, 0),
    (300, 40, 260, 1),
    (257, 9, 129, 2),
    (5, 2, 3, 3),
    (130, 1, 130, 4),
    (1, 3, 1, 5),
    # Norb = 820: the FP64 exchange-type term's per-q products G^q take two
    # chunks of q (798 + 22 within 4 GiB)
    (830, 4, 820, 6),
]


@pytest.mark.parametrize("nbf,naux,norb,seed", SHAPES)
def test_transform_jk_fock_energy_fp64(nbf, naux, norb, seed):
    nof = need_gpu()
    print(f"case fp64 nbf={nbf} naux={naux} norb={norb} seed={seed}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    ref = dfjk.iteration(B, C, H, n, cJ, cK)
    Bd, Cd, Hd = dev(B), dev(C), dev(H)
    b, D = nof.mo_transform(Bd, Cd)
    h = nof.one_electron(Hd, Cd)
    J, K = nof.jk_diag(b, D)
    lam, g, K2 = nof.gen_fock(b, D, dev(n), h, dev(cJ), dev(cK), want_K=True)
    E = nof.energy(dev(n), h, J, K, dev(cJ), dev(cK))
    torch.cuda.synchronize()
    bh = host(b)
    assert np.array_equal(bh, np.swapaxes(bh, 1, 2)), "b must be exactly symmetric"
    assert normwise(bh, ref["b"]) <= FP64_TOL
    assert normwise(host(D), ref["D"]) <= FP64_TOL
    assert normwise(host(h), ref["h"]) <= FP64_TOL
    assert normwise(host(J), ref["J"]) <= FP64_TOL
    assert normwise(host(K), ref["K"]) <= FP64_TOL
    assert np.array_equal(host(K), host(K2)), "fused K must equal the K-only pass"
    assert normwise(host(lam), ref["lam"]) <= FP64_TOL
    assert normwise(host(g), ref["g"]) <= FP64_TOL
    assert abs(float(E) - ref["E"]) <= FP64_TOL * abs(ref["E"])
    F2 = nof.exchange_fock(b, dev(cK))
    assert normwise(host(F2), ref["F2"]) <= FP64_TOL
    # the same build as its steps (F = F2 - F1, then lambda and g): identical
    # to the fused call bit for bit
    F = nof.fock_terms(b, D, dev(cJ), dev(cK))
    lam3, g3 = nof.lambda_grad(dev(n), h, None, F)
    torch.cuda.synchronize()
    assert normwise(host(F), ref["F2"] - ref["F1"]) <= FP64_TOL
    assert np.array_equal(host(lam3), host(lam)) and np.array_equal(host(g3), host(g))
    # the Coulomb-type term alone (HBM pass with K) with the exchange-type term
    # alone give the same lambda and g
    F1, K3 = nof.coulomb_fock(b, D, dev(cJ))
    lam4, g4 = nof.lambda_grad(dev(n), h, F1, F2)
    torch.cuda.synchronize()
    assert normwise(host(F1), ref["F1"]) <= FP64_TOL
    assert np.array_equal(host(K3), host(K2))
    assert normwise(host(lam4), ref["lam"]) <= FP64_TOL and normwise(host(g4), ref["g"]) <= FP64_TOL


def test_structured_coefficients_hf_closed_form():
    """Hartree-Fock occupations (0/1, Delta = Pi = 0): E equals the closed form."""
    nof = need_gpu()
    w = inputs.WORKLOADS["tiny"]
    B = inputs.make_B(w.seed, w.nbf, w.naux, w.decay)
    C = inputs.make_C(w.seed, w.nbf, w.norb)
    H = inputs.make_H(w.seed, w.nbf)
    n = np.zeros(w.norb)
    n[: w.nstrong] = 1.0
    Z = np.zeros((w.norb, w.norb))
    cJ, cK = nof.coeffs_from_cumulant(dev(n), dev(Z), dev(Z))
    Bd, Cd = dev(B), dev(C)
    b, D = nof.mo_transform(Bd, Cd)
    h = nof.one_electron(dev(H), Cd)
    J, K = nof.jk_diag(b, D)
    E = float(nof.energy(dev(n), h, J, K, cJ, cK))
    ref = dfjk.iteration(B, C, H, n, *dfjk.coeffs_from_cumulant(n, Z, Z))
    hh, Jh, Kh = ref["h"], ref["J"], ref["K"]
    o = slice(0, w.nstrong)
    E_hf = 2 * np.trace(hh[o, o]) + np.sum(2 * Jh[o, o] - Kh[o, o])
    assert abs(E - E_hf) <= FP64_TOL * abs(E_hf)


def test_coeffs_from_cumulant():
    nof = need_gpu()
    rng = np.random.default_rng(0)
    m = 37
    n = rng.uniform(0, 1, m)
    Dl = inputs.make_symmetric(1, m)
    Pi = inputs.make_symmetric(2, m)
    cJ, cK = nof.coeffs_from_cumulant(dev(n), dev(Dl), dev(Pi))
    rJ, rK = dfjk.coeffs_from_cumulant(n, Dl, Pi)
    assert normwise(host(cJ), rJ) <= 1e-15
    assert normwise(host(cK), rK) <= 1e-15


def test_deterministic_repeat():
    nof = need_gpu()
    B, C, H, n, cJ, cK = case(200, 64, 180, 7)
    Bd, Cd = dev(B), dev(C)
    outs = []
    for _ in range(2):
        b, D = nof.mo_transform(Bd, Cd)
        J, K = nof.jk_diag(b, D)
        lam, g, _ = nof.gen_fock(b, D, dev(n), dev(np.eye(180)), dev(cJ), dev(cK))
        outs.append([host(x) for x in (b, J, K, lam, g)])
    for a, c in zip(*outs):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("nbf,naux,norb,seed", [(48, 192, 48, 0), (300, 40, 260, 1)])
def test_fp32_form(nbf, naux, norb, seed):
    """FP32-stored B and b with FP32 matrix-core products (FP64 accumulation
    across auxiliary slabs and in every reduction).  Bounds: b, J, K, lambda
    normwise <= 2e-6; |dE|/|E| <= 1e-6."""
    nof = need_gpu()
    print(f"case fp32 nbf={nbf} naux={naux} norb={norb}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    ref = dfjk.iteration(B, C, H, n, cJ, cK)
    Bd = dev(B, torch.float32)
    Cd = dev(C)
    b, D = nof.mo_transform(Bd, Cd, prec=nof.P_F32)
    assert b.dtype == torch.float32
    h = nof.one_electron(dev(H), Cd)
    J, K = nof.jk_diag(b, D)
    lam, g, _ = nof.gen_fock(b, D, dev(n), h, dev(cJ), dev(cK), prec=nof.P_F32)
    E = float(nof.energy(dev(n), h, J, K, dev(cJ), dev(cK)))
    errs = dict(b=normwise(host(b), ref["b"]), J=normwise(host(J), ref["J"]),
                K=normwise(host(K), ref["K"]), lam=normwise(host(lam), ref["lam"]),
                E=abs(E - ref["E"]) / abs(ref["E"]))
    print("fp32 errors", errs, flush=True)
    for k in ("b", "J", "K", "lam"):
        assert errs[k] <= 2e-6, (k, errs[k])
    assert errs["E"] <= 1e-6


PASS_SHAPES = [(1, 1), (2, 3), (17, 5), (33, 127), (40, 130), (64, 257), (300, 64)]


@pytest.mark.parametrize("naux,norb", PASS_SHAPES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_k_and_coulomb_pass_shapes(naux, norb, dt):
    """The pass over the unique half of b (K and the Coulomb-type term F1) on
    degenerate, odd (unaligned pairs) and ragged shapes, FP64 and FP32 b, fed
    directly with symmetric slabs: K = sum_P b^2 and F1 against the oracle on
    the same values, FP64 accumulation: 1e-13.  With cK = 0 lambda = n h + F1,
    where nof_gen_fock forms F1 inside the exchange-type product: 1e-13 in
    FP64; with FP32 b that product runs in FP32 (W rounded to FP32, each
    product b_rs W_Ps rounded once, slab partials added in FP64), so the
    bound is 2 * 2^-24 * max_rs sum_P |b_rs W_Ps| beside 1e-13 of max|lambda|."""
    nof = need_gpu()
    print(f"case pass naux={naux} norb={norb} {dt}", flush=True)
    rng = np.random.default_rng(naux * 1000 + norb)
    b = rng.standard_normal((naux, norb, norb))
    b = b + np.swapaxes(b, 1, 2)
    if dt == "f32":
        b = b.astype(np.float32).astype(np.float64)
    D = np.ascontiguousarray(np.diagonal(b, axis1=1, axis2=2))
    n = rng.uniform(0.0, 1.0, norb)
    h = rng.standard_normal((norb, norb)); h = h + h.T
    cJ = rng.standard_normal((norb, norb)); cJ = cJ + cJ.T
    cK = np.zeros((norb, norb))
    tdt = torch.float64 if dt == "f64" else torch.float32
    prec = nof.P_F64 if dt == "f64" else nof.P_F32
    bd = dev(b, tdt)
    _, K = nof.jk_diag(bd, dev(D), want_J=False)
    lam, g, K2 = nof.gen_fock(bd, dev(D), dev(n), dev(h), dev(cJ), dev(cK), want_K=True, prec=prec)
    F1, K3 = nof.coulomb_fock(bd, dev(D), dev(cJ))
    torch.cuda.synchronize()
    Kref = np.einsum("Ppq,Ppq->pq", b, b)
    lam_ref, _, F1_ref, _ = dfjk.gen_fock(b, n, h, cJ, cK)
    assert normwise(host(K), Kref) <= 1e-13
    assert np.array_equal(host(K), host(K2)) and np.array_equal(host(K), host(K3))
    assert normwise(host(F1), F1_ref) <= 1e-13
    if dt == "f64":
        assert normwise(host(lam), lam_ref) <= 1e-13
    else:
        W = D @ cJ
        mag = np.max(np.einsum("Prs,Ps->rs", np.abs(b), np.abs(W)))
        err = np.max(np.abs(host(lam) - lam_ref))
        assert err <= 2 * 2.0 ** -24 * mag + 1e-13 * np.max(np.abs(lam_ref)), (err, mag)
