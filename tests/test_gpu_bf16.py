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

x10 (fixed-point pieces, exact leading products) is compared against the
oracle on the FP32-rounded B, so that only the arithmetic remains: the
representation error of four pieces is 2^-33 of a stage's largest element and
the dropped products are of order 2^-32, so what is left is the FP32 storage of
T and b (unit roundoff u = 2^-24, twice: normwise <= 2u = 1.2e-7), bound 3e-7;
the energy, a sum over those stored values, |dE|/|E| <= 2e-8 (observed <= 4.3e-9) where many
orbitals average the roundings, and |dE| <= 4u sum|terms| (the worst case) for one or two.
A cancellation case pins the exactness itself: with paired rows whose products
cancel, the exact result is zero and x10 must return it to 2^-30 of the sum of
the |products| (element-wise split pieces with the matrix cores' alignment
leave errors of order 2^-24 of the largest product there).
"""
import numpy as np
import pytest
import torch

from oracle import dfjk
from gpu_util import case, dev, host, need_gpu, normwise
from paper_2512_13550_amd import inputs

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


@pytest.mark.parametrize("nbf,naux,norb,seed", [(48, 192, 48, 0), (300, 40, 260, 1), (130, 7, 97, 5),
                                               (1, 3, 1, 6), (2, 5, 2, 7)])
def test_bf16_x10_fixed_point(nbf, naux, norb, seed):
    nof = need_gpu()
    print(f"case bf16 x10 nbf={nbf} naux={naux} norb={norb}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    B32 = B.astype(np.float32)
    ref = dfjk.iteration(B32.astype(np.float64), C, H, n, cJ, cK)
    got = run_gpu(nof, dev(B32, torch.float32), C, H, n, cJ, cK, nof.P_BF16X10)
    errs = {k: normwise(got[k], ref[k]) for k in ("b", "J", "K", "lam", "g")}
    errs["E"] = abs(got["E"] - ref["E"]) / abs(ref["E"])
    print("x10", errs, flush=True)
    for k in ("b", "J", "K", "lam"):
        assert errs[k] <= 3e-7, (k, errs[k])
    # E sums products of the stored T and b values: with many orbitals the
    # roundings average (2e-8 of |E|); with one or two nothing averages and
    # the bound is the worst case, 4u of the sum of the terms' magnitudes
    if norb >= 48:
        assert errs["E"] <= 2e-8
    else:
        terms = (2 * np.sum(np.abs(n * np.diag(ref["h"]))) + np.sum(np.abs(cJ * ref["J"]))
                 + np.sum(np.abs(cK * ref["K"])))
        assert abs(got["E"] - ref["E"]) <= 4 * 2.0 ** -24 * terms
    b32 = dev(ref["b"], torch.float32)
    F2 = nof.exchange_fock(b32, dev(cK), prec=nof.P_BF16X10)
    assert normwise(host(F2), ref["F2"]) <= 3e-7


@pytest.mark.parametrize("src", ["f32", "f64"])
@pytest.mark.parametrize("nbf,naux,norb,seed", [(48, 192, 48, 0), (300, 40, 260, 1), (130, 7, 97, 5)])
def test_bf16_x10_split_B(src, nbf, naux, norb, seed):
    """B split once into fixed-point planes (nof_split_B), from FP32 or FP64."""
    nof = need_gpu()
    print(f"case bf16 x10 split B from {src} nbf={nbf} naux={naux} norb={norb}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    Bin = B.astype(np.float32).astype(np.float64) if src == "f32" else B
    ref = dfjk.iteration(Bin, C, H, n, cJ, cK)
    planes = nof.SplitB(dev(Bin, torch.float32 if src == "f32" else torch.float64))
    got = run_gpu(nof, planes, C, H, n, cJ, cK, nof.P_BF16X10)
    errs = {k: normwise(got[k], ref[k]) for k in ("b", "J", "K", "lam", "g")}
    errs["E"] = abs(got["E"] - ref["E"]) / abs(ref["E"])
    print("x10 split B", src, errs, flush=True)
    for k in ("b", "J", "K", "lam"):
        assert errs[k] <= 3e-7, (k, errs[k])
    assert errs["E"] <= 2e-8


def test_bf16_x10_long_contraction():
    """Nbf > 1024: the order-0 sums are added to FP64 every 1024 terms."""
    nof = need_gpu()
    nbf, naux, norb = 1100, 3, 150
    print(f"case bf16 x10 long contraction nbf={nbf} naux={naux} norb={norb}", flush=True)
    B = inputs.make_B(9, nbf, naux, 25.0)
    C = inputs.make_C(9, nbf, norb)
    B32 = B.astype(np.float32)
    b_ref, D_ref = dfjk.mo_transform(B32.astype(np.float64), C)
    for Bd in (dev(B32, torch.float32), nof.SplitB(dev(B32, torch.float32))):
        b, D = nof.mo_transform(Bd, dev(C), prec=nof.P_BF16X10)
        torch.cuda.synchronize()
        eb, eD = normwise(host(b), b_ref), normwise(host(D), D_ref)
        print("x10 long", eb, eD, flush=True)
        assert eb <= 3e-7 and eD <= 3e-7


@pytest.mark.parametrize("nbf,naux,norb,seed", [(48, 192, 48, 0), (300, 40, 260, 1), (130, 7, 97, 5),
                                               (1100, 3, 150, 9)])
def test_bf16_x10_fused_grids_equal_two_stage(nbf, naux, norb, seed):
    """nof_mo_transform (x10) takes the column grids of T from the maxima that
    the first stage's epilogue writes per row tile; the two separate stage
    calls find them with a pass over T.  Same grids, so b and D agree bit for
    bit (row tiles: 1, 3, 2 and 9; ragged columns; K > 1024 in the last)."""
    nof = need_gpu()
    print(f"case bf16 x10 fused grids nbf={nbf} naux={naux} norb={norb}", flush=True)
    B = inputs.make_B(seed, nbf, naux, 25.0).astype(np.float32)
    Cd = dev(inputs.make_C(seed, nbf, norb))
    for Bd in (dev(B, torch.float32), nof.SplitB(dev(B, torch.float32))):
        b1, D1 = nof.mo_transform(Bd, Cd, prec=nof.P_BF16X10)
        T = torch.empty((naux, nbf, norb), dtype=torch.float32, device="cuda")
        nof.transform_stage1(Bd, Cd, T, prec=nof.P_BF16X10)
        b2 = torch.empty_like(b1)
        D2 = torch.empty_like(D1)
        nof.transform_stage2(T, Cd, b2, D2, prec=nof.P_BF16X10)
        torch.cuda.synchronize()
        assert torch.equal(b1, b2) and torch.equal(D1, D2)


def paired(rng, nrow, ncol, sign):
    """Rows 2k and 2k+1 equal (sign=+1) or opposite (sign=-1), entries with
    magnitudes spread over 2^-12..1."""
    half = rng.standard_normal((nrow // 2, ncol)) * 2.0 ** rng.uniform(-12, 0, (nrow // 2, ncol))
    out = np.empty((nrow, ncol))
    out[0::2] = half
    out[1::2] = sign * half
    return out


def test_bf16_x10_cancellation():
    nof = need_gpu()
    print("case bf16 x10 cancellation", flush=True)
    rng = np.random.default_rng(7)
    naux, nbf, norb = 3, 96, 80
    # stage 1: B = V M V^T with V_k = e_2k - e_2k+1 (symmetric, B[:, 2k+1] = -B[:, 2k]);
    # C with rows 2k and 2k+1 equal, so V^T C = 0 and T = B C = 0 exactly.
    M = rng.standard_normal((naux, nbf // 2, nbf // 2)) * 2.0 ** rng.uniform(-12, 0, (naux, nbf // 2, nbf // 2))
    M = 0.5 * (M + M.transpose(0, 2, 1))
    V = np.zeros((nbf, nbf // 2))
    V[0::2, np.arange(nbf // 2)] = 1.0
    V[1::2, np.arange(nbf // 2)] = -1.0
    B = np.einsum("ak,Pkl,bl->Pab", V, M, V).astype(np.float32)
    C = paired(rng, nbf, norb, +1.0)
    T = torch.empty((naux, nbf, norb), dtype=torch.float32, device="cuda")
    nof.transform_stage1(dev(B, torch.float32), dev(C), T, prec=nof.P_BF16X10)
    scale1 = np.einsum("Pab,bq->Paq", np.abs(B.astype(np.float64)), np.abs(C))
    r1 = float(np.max(np.abs(host(T)) / scale1))
    nof.transform_stage1(nof.SplitB(dev(B, torch.float32)), dev(C), T, prec=nof.P_BF16X10)
    r1 = max(r1, float(np.max(np.abs(host(T)) / scale1)))
    # stage 2: T with rows 2k+1 = -(rows 2k), C with rows 2k and 2k+1 equal: b = C^T T = 0
    T2 = np.stack([paired(rng, nbf, norb, -1.0) for _ in range(naux)]).astype(np.float32)
    b = torch.empty((naux, norb, norb), dtype=torch.float32, device="cuda")
    D = torch.empty((naux, norb), dtype=torch.float64, device="cuda")
    nof.transform_stage2(dev(T2, torch.float32), dev(C), b, D, prec=nof.P_BF16X10)
    torch.cuda.synchronize()
    scale2 = np.einsum("ap,Paq->Ppq", np.abs(C), np.abs(T2.astype(np.float64)))
    r2 = float(np.max(np.abs(host(b)) / scale2))
    r2d = float(np.max(np.abs(host(D)) / np.diagonal(scale2, axis1=1, axis2=2)))
    print("x10 cancellation |out| / sum|products|:", r1, r2, r2d, flush=True)
    assert r1 <= 2.0 ** -30 and r2 <= 2.0 ** -30 and r2d <= 2.0 ** -30


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


def test_split_B_pieces_meet_documented_bounds():
    """nof_split_B's planes read back: per row (P, mu), with 2^E the smallest
    power of two above the row's largest |value|, piece q is an integer
    n_q times 2^(E-7-8q) with |n_q| <= 128, the four pieces leave
    |v - sum| <= 2^(E-32), and the padding columns are zero."""
    nof = need_gpu()
    nbf, naux = 50, 3
    B = inputs.make_B(11, nbf, naux, 8.0)
    B[1, 7, :] *= 1e-9            # rows far below the others keep their own grid
    B[1, :, 7] *= 1e-9
    B[2, 3, :] = 0.0              # an all-zero row
    B[2, :, 3] = 0.0
    planes = nof.SplitB(dev(B))
    torch.cuda.synchronize()
    ldk = (nbf + 31) // 32 * 32
    pl = planes.planes.view(torch.bfloat16)[: 4 * naux * nbf * ldk].view(4, naux, nbf, ldk)
    P = pl.to(torch.float64).cpu().numpy()
    assert np.all(P[:, :, :, nbf:] == 0.0)
    P = P[:, :, :, :nbf]
    m = np.max(np.abs(B), axis=2)                       # [naux][nbf]
    E = np.where(m > 0, np.frexp(m)[1], 0)
    for q in range(4):
        unit = np.ldexp(1.0, E - 7 - 8 * q)[:, :, None]
        nq = P[q] / unit
        assert np.array_equal(nq, np.rint(nq)), q
        assert np.max(np.abs(nq)) <= 128, q
    resid = np.abs(B - P.sum(axis=0))
    assert np.all(resid <= np.ldexp(1.0, E - 32)[:, :, None])


@pytest.mark.parametrize("mode", ["f32", "x1", "x3", "x6", "x10", "i8"])
def test_fock_terms_reduced_precision(mode):
    """Both Fock terms in one call (nof_fock_terms: F = F2 - F1) on FP32 b
    against the oracle on the same FP32 values.  F32, x1 and x3 take the
    Coulomb-type term into the exchange-type product's right operand (each
    b_rs W_Ps then rounded once in that product's arithmetic); x6, x10 and
    the INT8 form take F1 from the FP64 pass over b.  Bounds, relative to
    the larger of max|F1| and max|F2|: the forms' normwise bounds above (f32:
    the FP32 form's 2e-6, x10: 3e-7)."""
    nof = need_gpu()
    prec = {"f32": nof.P_F32, "x1": nof.P_BF16X1, "x3": nof.P_BF16X3, "x6": nof.P_BF16X6,
            "x10": nof.P_BF16X10, "i8": nof.P_I8X10}[mode]
    tol = {"f32": 2e-6, "x10": 3e-7, "i8": 3e-7}.get(mode, BOUNDS.get(mode, (0, 0))[0])
    nbf, naux, norb, seed = 150, 11, 133, 8
    print(f"case fock terms {mode} naux={naux} norb={norb}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    b64 = dfjk.iteration(B, C, H, n, cJ, cK)["b"]
    b32 = b64.astype(np.float32).astype(np.float64)
    _, _, F1, F2 = dfjk.gen_fock(b32, n, np.zeros((norb, norb)), cJ, cK)
    D = np.ascontiguousarray(np.diagonal(b32, axis1=1, axis2=2))
    F = nof.fock_terms(dev(b32, torch.float32), dev(D), dev(cJ), dev(cK), prec=prec)
    torch.cuda.synchronize()
    scale = max(np.max(np.abs(F1)), np.max(np.abs(F2)))
    err = float(np.max(np.abs(host(F) - (F2 - F1)))) / scale
    print(mode, "fock terms error", err, flush=True)
    assert err <= tol, (mode, err)
