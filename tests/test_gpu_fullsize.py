"""Parity at the benchmark's full sizes, in its launch configuration.

c500 (Nbf=500, Naux=2000, Norb=500): the whole iteration (stage 1, stage 2,
h, J, generalized Fock with fused K, energy) against the complete FP64
oracle, element by element, for the FP64, FP32, BF16 x6 and BF16 x10 (B
split once into fixed-point planes) forms.

chain1000 (Nbf=1000, Naux=4000, Norb=1000): one whole iteration in the
benchmark's call sequence (stages, h, J, Coulomb-type pass with K,
exchange-type term, lambda and g, energy) against the oracle run slab by slab
over all 4000 slabs: E, J, K, lambda and g to 1e-10 normwise in FP64; the x10
forms (B as planes of the FP64 B; B stored in FP32, whose rounding alone
moves E by about 6e-7 Eh here) and the INT8 form within 1e-6 Eh of the
oracle's E and lambda within 3e-7 normwise; also the orthogonal sum rules,
which hold at any size.
"""
import numpy as np
import pytest
import torch

from oracle import dfjk
from paper_2512_13550_amd import inputs
from gpu_util import dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu


def gpu_step(nof, B, C, H, n, cJ, cK, prec, dt):
    naux, nbf, _ = B.shape
    norb = C.shape[1]
    T = torch.empty((naux, nbf, norb), dtype=dt, device="cuda")
    b = torch.empty((naux, norb, norb), dtype=dt, device="cuda")
    D = torch.empty((naux, norb), dtype=torch.float64, device="cuda")
    nof.transform_stage1(B, C, T, prec=prec)
    nof.transform_stage2(T, C, b, D, prec=prec)
    del T
    h = nof.one_electron(H, C)
    J, _ = nof.jk_diag(b, D, want_K=False)
    lam, g, K = nof.gen_fock(b, D, n, h, cJ, cK, want_K=True, prec=prec)
    E = nof.energy(n, h, J, K, cJ, cK)
    torch.cuda.synchronize()
    return b, D, dict(h=host(h), J=host(J), K=host(K), lam=host(lam), g=host(g), E=float(E))


def test_c500_full_iteration_all_forms():
    nof = need_gpu()
    w = inputs.WORKLOADS["c500"]
    print("case c500 full", flush=True)
    B = inputs.make_B(w.seed, w.nbf, w.naux, w.decay, threads=16)
    C = inputs.make_C(w.seed, w.nbf, w.norb)
    H = inputs.make_H(w.seed, w.nbf)
    n = inputs.make_occupations(w.seed, w.norb, w.nstrong)
    nn = np.outer(n, n)
    cJ, cK = 2.0 * nn, nn
    ref = dfjk.iteration(B, C, H, n, cJ, cK)
    print("oracle E", ref["E"], flush=True)
    Cd, Hd, nd, cJd, cKd = dev(C), dev(H), dev(n), dev(cJ), dev(cK)
    bounds = {"f64": (1e-10, 1e-10), "f32": (2e-6, 1e-8), "bf16x6": (5e-7, 2e-9), "bf16x10": (3e-7, 1e-9)}
    # g = 4 (lambda - lambda^T) is normed by its own (smaller) maximum
    gbounds = {"f64": 1e-10, "f32": 5e-5, "bf16x6": 2e-6, "bf16x10": 2e-6}
    for form, prec, dt in (("f64", nof.P_F64, torch.float64), ("f32", nof.P_F32, torch.float32),
                           ("bf16x6", nof.P_BF16X6, torch.float32), ("bf16x10", nof.P_BF16X10, torch.float32)):
        Bd = dev(B, torch.float64 if form in ("f64", "bf16x10") else torch.float32)
        if form == "bf16x10":
            Bd = nof.SplitB(Bd)
        b, D, got = gpu_step(nof, Bd, Cd, Hd, nd, cJd, cKd, prec, dt)
        del Bd
        errs = {k: normwise(got[k], ref[k]) for k in ("h", "J", "K", "lam", "g")}
        errs["b"] = normwise(host(b), ref["b"])
        errs["D"] = normwise(host(D), ref["D"])
        errs["E"] = abs(got["E"] - ref["E"]) / abs(ref["E"])
        print(form, {k: f"{v:.2e}" for k, v in errs.items()}, "dE Eh", got["E"] - ref["E"], flush=True)
        del b, D
        torch.cuda.empty_cache()
        tol, tolE = bounds[form]
        for k in ("b", "D", "J", "K", "lam"):
            assert errs[k] <= tol, (form, k, errs[k])
        assert errs["g"] <= gbounds[form], (form, errs["g"])
        assert errs["E"] <= tolE, (form, errs["E"])


def bench_step(nof, B, C, H, n, cJ, cK, prec, dt):
    """One iteration in bench.py's call sequence: the stages (one
    nof_mo_transform call for x10), h, J; then K alone and both Fock terms in
    one contraction (FP64), or K with the Coulomb-type term in one pass and
    the exchange-type term (x10, INT8); lambda and g, E."""
    naux, nbf, _ = B.shape
    norb = C.shape[1]
    b = torch.empty((naux, norb, norb), dtype=dt, device="cuda")
    D = torch.empty((naux, norb), dtype=torch.float64, device="cuda")
    fixed = prec in (nof.P_BF16X10, nof.P_I8X10)
    if fixed:
        nof.mo_transform(B, C, prec=prec, b=b, D=D)
    else:
        T = torch.empty((naux, nbf, norb), dtype=dt, device="cuda")
        nof.transform_stage1(B, C, T, prec=prec)
        nof.transform_stage2(T, C, b, D, prec=prec)
        del T
    h = nof.one_electron(H, C)
    if fixed:
        J, _ = nof.jk_diag(b, D, want_K=False)
        F1, K = nof.coulomb_fock(b, D, cJ)
        F2 = nof.exchange_fock(b, cK, prec=prec)
        lam, g = nof.lambda_grad(n, h, F1, F2)
    else:
        J, K = nof.jk_diag(b, D)
        F = nof.fock_terms(b, D, cJ, cK, prec=prec)
        lam, g = nof.lambda_grad(n, h, None, F)
    E = nof.energy(n, h, J, K, cJ, cK)
    torch.cuda.synchronize()
    del b, D
    torch.cuda.empty_cache()
    return dict(h=host(h), J=host(J), K=host(K), lam=host(lam), g=host(g), E=float(E))


def test_chain1000_against_oracle_all_forms():
    nof = need_gpu()
    w = inputs.WORKLOADS["chain1000"]
    print("case chain1000", flush=True)
    B = inputs.make_B(w.seed, w.nbf, w.naux, w.decay, threads=16)
    C = inputs.make_C(w.seed, w.nbf, w.norb)
    H = inputs.make_H(w.seed, w.nbf)
    n = inputs.make_occupations(w.seed, w.norb, w.nstrong)
    nn = np.outer(n, n)
    cJ, cK = 2.0 * nn, nn
    Cd, Hd, nd, cJd, cKd = dev(C), dev(H), dev(n), dev(cJ), dev(cK)
    Bd = dev(B)
    got64 = bench_step(nof, Bd, Cd, Hd, nd, cJd, cKd, nof.P_F64, torch.float64)
    planes = nof.SplitB(Bd)
    del Bd
    torch.cuda.empty_cache()
    gotx = bench_step(nof, planes, Cd, Hd, nd, cJd, cKd, nof.P_BF16X10, torch.float32)
    del planes
    torch.cuda.empty_cache()
    Bd = dev(B, torch.float32)
    gotx32 = bench_step(nof, Bd, Cd, Hd, nd, cJd, cKd, nof.P_BF16X10, torch.float32)
    del Bd
    torch.cuda.empty_cache()
    # INT8 form: its exchange-type planes (33 GB here) are split and multiplied
    # in chunks of groups that fit the 8 GiB plane budget (four chunks)
    planes8 = nof.SplitBI8(dev(B))
    got8 = bench_step(nof, planes8, Cd, Hd, nd, cJd, cKd, nof.P_I8X10, torch.float32)
    del planes8
    torch.cuda.empty_cache()
    print("gpu done; oracle over all slabs", flush=True)
    ref = dfjk.streamed_iteration(lambda lo, hi: B[lo:hi], w.naux, C, H, n, cJ, cK, pblock=100)
    errs = {k: normwise(got64[k], ref[k]) for k in ("h", "J", "K", "lam", "g")}
    errs["E"] = abs(got64["E"] - ref["E"]) / abs(ref["E"])
    print("chain1000 FP64 vs oracle", {k: f"{v:.2e}" for k, v in errs.items()}, "E", ref["E"], flush=True)
    for k, v in errs.items():
        assert v <= 1e-10, (k, v)
    for name, got in (("x10 planes of FP64 B", gotx), ("x10 FP32 B", gotx32), ("INT8 planes of FP64 B", got8)):
        dE = got["E"] - ref["E"]
        print("chain1000", name, "dE (Eh)", dE, "max dJ", np.abs(got["J"] - ref["J"]).max(),
              "max dK", np.abs(got["K"] - ref["K"]).max(), "lambda normwise", normwise(got["lam"], ref["lam"]),
              flush=True)
        assert abs(dE) <= 1e-6, (name, dE)
        assert normwise(got["lam"], ref["lam"]) <= 3e-7, name
    # orthogonal sum rules (Norb = Nbf): sum K = sum_P ||B^P||_F^2, sum J = sum_P (tr B^P)^2
    sK = float(np.einsum("Pmn,Pmn->", B, B))
    sJ = float(np.sum(np.trace(B, axis1=1, axis2=2) ** 2))
    assert abs(got64["K"].sum() - sK) <= 1e-10 * sK
    assert abs(got64["J"].sum() - sJ) <= 1e-10 * sJ
