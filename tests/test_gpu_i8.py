"""INT8 fixed-point form of the transform (NOF_P_I8X10) against the FP64
oracle.

Bounds (normwise, derived from the arithmetic): the four INT8 pieces of a
row or column leave a residual of at most 2^-29 of its largest element and
the dropped products of order 4..6 are below 2^-28 of |x|max |y|max per
term, so what dominates is the FP32 storage of T and b (unit roundoff
u = 2^-24, twice: normwise <= 2u = 1.2e-7); bound 3e-7 for b, D, J, K and
lambda (whose exchange-type term is the x10 one), |dE|/|E| <= 2e-8 where
many orbitals average the roundings, and the worst case 4u sum|terms| with
one or two orbitals.  The integer sums are exact: products that cancel in
exact arithmetic cancel exactly (a zero result is returned as zero).
"""
import numpy as np
import pytest
import torch

from oracle import dfjk
from gpu_util import case, dev, host, need_gpu, normwise
from paper_2512_13550_amd import inputs

pytestmark = pytest.mark.gpu


def run_gpu(nof, planes, C, H, n, cJ, cK):
    Cd = dev(C)
    b, D = nof.mo_transform(planes, Cd, prec=nof.P_I8X10)
    assert b.dtype == torch.float32
    h = nof.one_electron(dev(H), Cd)
    J, K = nof.jk_diag(b, D)
    lam, g, _ = nof.gen_fock(b, D, dev(n), h, dev(cJ), dev(cK), prec=nof.P_I8X10)
    E = float(nof.energy(dev(n), h, J, K, dev(cJ), dev(cK)))
    torch.cuda.synchronize()
    return dict(b=host(b), D=host(D), J=host(J), K=host(K), lam=host(lam), g=host(g), E=E)


def test_split_B_i8_pieces_meet_documented_bounds():
    """nof_split_B_i8 read back: per row (P, mu), E is the smallest exponent
    with max|v| 2^(7-E) < 127.5; the INT8 pieces satisfy |n_0| <= 127,
    |n_1..3| <= 64, sum_q n_q 2^(E-7-7q) leaves |v - sum| <= 2^(E-29), and the
    padding columns are zero."""
    nof = need_gpu()
    nbf, naux = 70, 3
    B = inputs.make_B(12, nbf, naux, 8.0)
    B[1, 7, :] *= 1e-9            # a row far below the others keeps its own grid
    B[1, :, 7] *= 1e-9
    B[2, 3, :] = 0.0              # an all-zero row
    B[2, :, 3] = 0.0
    B[0, 5, :] *= 127.75 / 128 / np.max(np.abs(B[0, 5, :]))   # max just above 127.5 / 128
    B[0, :, 5] = B[0, 5, :]
    sp = nof.SplitBI8(dev(B))
    torch.cuda.synchronize()
    ldk = (nbf + 63) // 64 * 64
    rows = naux * nbf
    raw = sp.planes.cpu().numpy()
    P = raw[: 4 * rows * ldk].view(np.int8).reshape(4, naux, nbf, ldk).astype(np.float64)
    eoff = (4 * rows * ldk + 255) // 256 * 256
    E = raw[eoff: eoff + 4 * rows].view(np.int32).reshape(naux, nbf)
    assert np.all(P[:, :, :, nbf:] == 0.0)
    P = P[:, :, :, :nbf]
    m = np.max(np.abs(B), axis=2)
    Eref = np.frexp(m)[1]
    Eref = np.where(np.ldexp(m, 7 - Eref) >= 127.5, Eref + 1, Eref)
    nz = m > 0
    assert np.array_equal(E[nz], Eref[nz])
    assert E[0, 5] == Eref[0, 5]
    assert np.max(np.abs(P[0])) <= 127 and np.max(np.abs(P[1:])) <= 64
    rec = sum(P[q] * np.ldexp(1.0, E - 7 - 7 * q)[:, :, None] for q in range(4))
    resid = np.abs(B - rec)
    assert np.all(resid <= np.ldexp(1.0, E - 29)[:, :, None])
    assert np.all(rec[2, 3, :] == 0.0)


@pytest.mark.parametrize("nbf,naux,norb,seed", [(48, 192, 48, 0), (300, 40, 260, 1), (130, 7, 97, 5),
                                               (1, 3, 1, 6), (2, 5, 2, 7), (257, 9, 129, 2)])
def test_i8x10_against_oracle(nbf, naux, norb, seed):
    nof = need_gpu()
    print(f"case i8x10 nbf={nbf} naux={naux} norb={norb}", flush=True)
    B, C, H, n, cJ, cK = case(nbf, naux, norb, seed)
    ref = dfjk.iteration(B, C, H, n, cJ, cK)
    got = run_gpu(nof, nof.SplitBI8(dev(B)), C, H, n, cJ, cK)
    errs = {k: normwise(got[k], ref[k]) for k in ("b", "D", "J", "K", "lam", "g")}
    errs["E"] = abs(got["E"] - ref["E"]) / abs(ref["E"])
    print("i8x10", errs, flush=True)
    assert np.array_equal(got["b"], np.swapaxes(got["b"], 1, 2)), "b must be exactly symmetric"
    for k in ("b", "D", "J", "K", "lam"):
        assert errs[k] <= 3e-7, (k, errs[k])
    if norb >= 48:
        assert errs["E"] <= 2e-8
    else:
        terms = (2 * np.sum(np.abs(n * np.diag(ref["h"]))) + np.sum(np.abs(cJ * ref["J"]))
                 + np.sum(np.abs(cK * ref["K"])))
        assert abs(got["E"] - ref["E"]) <= 4 * 2.0 ** -24 * terms


def test_i8x10_from_fp32_B():
    """B split from FP32 storage: the oracle on the FP32-rounded B."""
    nof = need_gpu()
    B, C, H, n, cJ, cK = case(200, 30, 180, 3)
    B32 = B.astype(np.float32)
    ref = dfjk.iteration(B32.astype(np.float64), C, H, n, cJ, cK)
    got = run_gpu(nof, nof.SplitBI8(dev(B32, torch.float32)), C, H, n, cJ, cK)
    errs = {k: normwise(got[k], ref[k]) for k in ("b", "J", "K", "lam")}
    print("i8x10 fp32 B", errs, flush=True)
    for k, v in errs.items():
        assert v <= 3e-7, (k, v)


def test_i8x10_long_contraction():
    """Nbf = 2100: the int32 sums stay exact at this depth (no FP64 flush)."""
    nof = need_gpu()
    nbf, naux, norb = 2100, 2, 140
    print(f"case i8x10 long contraction nbf={nbf} naux={naux} norb={norb}", flush=True)
    B = inputs.make_B(9, nbf, naux, 25.0)
    C = inputs.make_C(9, nbf, norb)
    b_ref, D_ref = dfjk.mo_transform(B, C)
    b, D = nof.mo_transform(nof.SplitBI8(dev(B)), dev(C), prec=nof.P_I8X10)
    torch.cuda.synchronize()
    eb, eD = normwise(host(b), b_ref), normwise(host(D), D_ref)
    print("i8x10 long", eb, eD, flush=True)
    assert eb <= 3e-7 and eD <= 3e-7


def test_i8x10_exact_cancellation():
    """B = V M V^T with V_k = e_2k - e_2k+1 (so B[:, 2k+1] = -B[:, 2k]) and C
    with rows 2k and 2k+1 equal: V^T C = 0, so T = B C = 0 and b = C^T T = 0
    in exact arithmetic.  The negated and equal values have negated and equal
    pieces on one grid, and the int32 sums are exact, so b and D come out as
    zeros (the BF16 form leaves ~2^-30 of the summed magnitudes here)."""
    nof = need_gpu()
    rng = np.random.default_rng(7)
    naux, nbf, norb = 3, 128, 90
    M = rng.standard_normal((naux, nbf // 2, nbf // 2)) * 2.0 ** rng.uniform(-12, 0, (naux, nbf // 2, nbf // 2))
    M = 0.5 * (M + M.transpose(0, 2, 1))
    V = np.zeros((nbf, nbf // 2))
    V[0::2, np.arange(nbf // 2)] = 1.0
    V[1::2, np.arange(nbf // 2)] = -1.0
    B = np.einsum("ak,Pkl,bl->Pab", V, M, V)
    half = rng.standard_normal((nbf // 2, norb)) * 2.0 ** rng.uniform(-12, 0, (nbf // 2, norb))
    C = np.repeat(half, 2, axis=0)
    b, D = nof.mo_transform(nof.SplitBI8(dev(B)), dev(C), prec=nof.P_I8X10)
    torch.cuda.synchronize()
    assert float(host(b).__abs__().max()) == 0.0
    assert float(host(D).__abs__().max()) == 0.0


@pytest.mark.parametrize("naux,norb,seed", [(600, 256, 11), (450, 300, 12), (5, 70, 13), (65600, 8, 14)])
def test_i8x10_exchange_groups(naux, norb, seed):
    """The INT8 exchange-type term with slabs far below the others.  Up to the
    exact int32 depth (Naux <= 65536) it runs through the per-q symmetric
    products G^q_rs = sum_P b^P[q][r] b^P[q][s], one INT8 product over all
    slabs per q with one grid per (q, r); beyond it (Naux = 65600) as one
    INT8 product per group of slabs whose joint contraction (slabs x 64-padded
    rows) stays within 65536 (norb = 8: 1024 slabs a group, 65 groups).  A slab
    far below the others only loses digits below 2^-29 of its grid's maximum,
    which the normwise bound of 3e-7 (relative to max|F1|, max|F2|) covers."""
    nof = need_gpu()
    print(f"case i8x10 exchange groups naux={naux} norb={norb}", flush=True)
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((naux, norb, norb))
    b = 0.5 * (b + b.transpose(0, 2, 1))
    b[1::7] *= 1e-6                       # slabs far below the others in the same group
    b32 = b.astype(np.float32).astype(np.float64)
    n = rng.uniform(0.0, 1.0, norb)
    cJ = rng.standard_normal((norb, norb))
    cK = rng.standard_normal((norb, norb))
    cJ, cK = cJ + cJ.T, cK + cK.T         # the coupling matrices are symmetric
    _, _, F1, F2 = dfjk.gen_fock(b32, n, np.zeros((norb, norb)), cJ, cK)
    D = np.ascontiguousarray(np.diagonal(b32, axis1=1, axis2=2))
    F = nof.fock_terms(dev(b32, torch.float32), dev(D), dev(cJ), dev(cK), prec=nof.P_I8X10)
    torch.cuda.synchronize()
    scale = max(np.max(np.abs(F1)), np.max(np.abs(F2)))
    err = float(np.max(np.abs(host(F) - (F2 - F1)))) / scale
    print("i8x10 exchange groups error", err, flush=True)
    assert err <= 3e-7, err


def test_i8x10_stage_entry_points_reject():
    """The INT8 form exists as the fused transform only."""
    nof = need_gpu()
    B, C, H, n, cJ, cK = case(40, 4, 30, 1)
    sp = nof.SplitBI8(dev(B))
    T = torch.empty((4, 40, 30), dtype=torch.float32, device="cuda")
    with pytest.raises(nof.NofError):
        nof.transform_stage1(sp, dev(C), T, prec=nof.P_I8X10)
