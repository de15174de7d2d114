"""Split-precision BF16 form of the transform and exchange-type Fock term
against the FP64 oracle.

Bounds (normwise, derived from the arithmetic): a BF16 piece keeps 8 bits, so
one piece leaves a relative residual <= 2^-8 per operand, two pieces 2^-16 and
three pieces 2^-24; products of pieces are exact in FP32 and are accumulated in
FP32 within one auxiliary slab (about sqrt(K/32) roundings of 2^-24).  With a
safety factor of ~10 on the observed errors:
  x1: 2e-2,   x3: 1e-4,   x6: 2e-6 (the FP32 form's bar),
and the energy |dE|/|E| <= 2e-2, 1e-5, 5e-8 respectively.  B stored in BF16 is
compared against the oracle evaluated on the BF16-rounded B (the arithmetic
error alone), with the x6 bounds.
"""
import numpy as np
import pytest
import torch

from oracle import dfjk
from gpu_util import case, dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu

BOUNDS = {"x1": (2e-2, 2e-2), "x3": (1e-4, 1e-5), "x6": (2e-6, 5e-8)}


def run_gpu(nof, Bd, C, H, n, cJ, cK, prec):
    Cd = dev(C)
    b, D = nof.mo_transform(Bd, Cd, prec=prec)
    assert b.dtype == torch.float32
    h = nof.one_electron(dev(H), Cd)
    J, K = nof.jk_diag(b, D)
    lam, g, _ = nof.gen_fock(b, D, dev(n), h, dev(cJ), dev(cK), prec=prec)
    E = float(nof.energy(dev(n), h, J, K, dev(cJ), dev(cK)))
    torch.cuda.synchronize()
    return dict(b=host(b), J=host(J), K=host(K), lam=host(lam), g=host(g), E=E)


@pytest.mark.parametrize("mode", ["x1", "x3", "x6"])
@pytest.mark.parametrize("nbf,naux,norb,seed", [(48, 192, 48, 0), (300, 40, 260, 1), (130, 7, 97, 5)])
def test_bf16_split_forms(mode, nbf, naux, norb, seed):
    nof = need_gpu()
    prec = {"x1": nof.P_BF16X1, "x3": nof.P_BF16X3, "x6": nof.P_BF16X6}[mode]
    print(f"case bf16 {mode} nbf={nbf} naux={naux} norb={norb}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    ref = dfjk.iteration(B, C, H, n, cJ, cK)
    got = run_gpu(nof, dev(B, torch.float32), C, H, n, cJ, cK, prec)
    errs = {k: normwise(got[k], ref[k]) for k in ("b", "J", "K", "lam", "g")}
    errs["E"] = abs(got["E"] - ref["E"]) / abs(ref["E"])
    print(mode, errs, flush=True)
    tol, tolE = BOUNDS[mode]
    for k in ("b", "J", "K", "lam"):
        assert errs[k] <= tol, (k, errs[k])
    assert errs["E"] <= tolE


@pytest.mark.parametrize("nbf,naux,norb,seed", [(48, 192, 48, 0), (300, 40, 260, 1)])
def test_bf16_stored_B(nbf, naux, norb, seed):
    nof = need_gpu()
    print(f"case bf16-stored B nbf={nbf} naux={naux} norb={norb}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    Bb = torch.from_numpy(B).to(torch.bfloat16)
    B_rounded = Bb.to(torch.float64).numpy()
    ref = dfjk.iteration(B_rounded, C, H, n, cJ, cK)
    got = run_gpu(nof, Bb.to("cuda"), C, H, n, cJ, cK, nof.P_BF16X6)
    errs = {k: normwise(got[k], ref[k]) for k in ("b", "J", "K", "lam")}
    errs["E"] = abs(got["E"] - ref["E"]) / abs(ref["E"])
    print("bf16-stored", errs, flush=True)
    tol, tolE = BOUNDS["x6"]
    for k in ("b", "J", "K", "lam"):
        assert errs[k] <= tol, (k, errs[k])
    assert errs["E"] <= tolE
