"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before launching anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    path = os.path.join(ROOT, "paper_2512_13550_amd", "libnof.so")
    if not os.path.exists(path):
        pytest.fail("libnof.so not built (run __graft_entry__.build())")
    import paper_2512_13550_amd.nof as nof
    return nof


def declared_symbols():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(nof_[A-Za-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    nof = _lib()
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(nof.lib, s), s
    assert set(nof.DECLARED) <= set(syms)


FAKE = ctypes.c_void_p(4096)   # never dereferenced: validation fails before any launch


def test_status_strings():
    nof = _lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -99, 12345):
        assert isinstance(nof.lib.nof_status_str(code), bytes)


def test_transform_validation():
    nof = _lib()
    L = nof.lib
    assert L.nof_mo_transform(0, 4, 4, FAKE, 0, FAKE, FAKE, 0, None, 0, FAKE, 1 << 20, None) == nof.E_DIM
    assert L.nof_mo_transform(2, 4, 4, None, 0, FAKE, FAKE, 0, None, 0, FAKE, 1 << 20, None) == nof.E_NULL
    assert L.nof_mo_transform(2, 4, 4, FAKE, 0, FAKE, FAKE, 2, None, 0, FAKE, 1 << 20, None) == nof.E_DTYPE
    assert L.nof_mo_transform(2, 4, 4, FAKE, 0, FAKE, FAKE, 1, None, 0, FAKE, 1 << 20, None) == nof.E_PREC
    assert L.nof_mo_transform(2, 4, 4, FAKE, 0, FAKE, FAKE, 0, None, 1, FAKE, 1 << 20, None) == nof.E_PREC
    assert L.nof_mo_transform(2, 4, 4, FAKE, 0, FAKE, FAKE, 0, None, 7, FAKE, 1 << 20, None) == nof.E_PREC
    need = L.nof_mo_transform_ws(2, 4, 4, 0, 0, 0)
    assert need >= 2 * 4 * 4 * 8
    assert L.nof_mo_transform(2, 4, 4, FAKE, 0, FAKE, FAKE, 0, None, 0, FAKE, need - 1, None) == nof.E_WORKSPACE
    assert L.nof_mo_transform(2, 4, 4, FAKE, 0, FAKE, FAKE, 0, None, 0, None, need, None) == nof.E_WORKSPACE


def test_jk_and_fock_validation():
    nof = _lib()
    L = nof.lib
    assert L.nof_jk_diag(-1, 4, FAKE, 0, FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == nof.E_DIM
    assert L.nof_jk_diag(3, 4, None, 0, FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == nof.E_NULL
    assert L.nof_jk_diag(3, 4, FAKE, 2, FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == nof.E_DTYPE
    assert L.nof_jk_diag(3, 4, FAKE, 0, FAKE, FAKE, FAKE, FAKE, 8, None) == nof.E_WORKSPACE
    args = [FAKE] * 6   # D, n, h, cJ, cK, lambda
    assert L.nof_gen_fock(3, 4, FAKE, 0, *args, None, None, 0, FAKE, 8, None) == nof.E_WORKSPACE
    assert L.nof_gen_fock(3, 4, FAKE, 0, FAKE, FAKE, FAKE, FAKE, None, FAKE, None, None, 0, FAKE, 1 << 30, None) == nof.E_NULL
    assert L.nof_gen_fock(3, 4, FAKE, 0, *args, None, None, 1, FAKE, 1 << 30, None) == nof.E_PREC
    assert L.nof_energy(0, *([FAKE] * 7), FAKE, 1 << 20, None) == nof.E_DIM
    assert L.nof_energy(4, FAKE, FAKE, None, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == nof.E_NULL
    assert L.nof_energy_ws(4) > 0 and L.nof_energy_ws(0) == 0
    assert L.nof_energy(4, *([FAKE] * 7), FAKE, L.nof_energy_ws(4) - 1, None) == nof.E_WORKSPACE
    assert L.nof_coeffs_from_cumulant(4, FAKE, None, FAKE, FAKE, FAKE, None) == nof.E_NULL
    need = L.nof_coulomb_fock_ws(3, 4, 0)
    assert need > 0 and L.nof_coulomb_fock_ws(3, 4, 2) == 0 and L.nof_coulomb_fock_ws(0, 4, 0) == 0
    assert L.nof_coulomb_fock(3, 4, FAKE, 0, FAKE, FAKE, FAKE, None, FAKE, need - 1, None) == nof.E_WORKSPACE
    assert L.nof_coulomb_fock(3, 4, FAKE, 0, None, FAKE, FAKE, None, FAKE, need, None) == nof.E_NULL
    assert L.nof_coulomb_fock(3, 4, FAKE, 2, FAKE, FAKE, FAKE, None, FAKE, need, None) == nof.E_DTYPE
    assert L.nof_coulomb_fock(0, 4, FAKE, 0, FAKE, FAKE, FAKE, None, FAKE, need, None) == nof.E_DIM
    assert L.nof_lambda_grad(4, FAKE, FAKE, FAKE, None, FAKE, None, None) == nof.E_NULL
    assert L.nof_lambda_grad(0, FAKE, FAKE, FAKE, FAKE, FAKE, None, None) == nof.E_DIM


def test_exchange_split_and_stage_validation():
    nof = _lib()
    L = nof.lib
    big = 1 << 30
    assert L.nof_exchange_fock(0, 4, FAKE, 0, FAKE, FAKE, 0, FAKE, big, None) == nof.E_DIM
    assert L.nof_exchange_fock(3, 4, None, 0, FAKE, FAKE, 0, FAKE, big, None) == nof.E_NULL
    assert L.nof_exchange_fock(3, 4, FAKE, 0, None, FAKE, 0, FAKE, big, None) == nof.E_NULL
    assert L.nof_exchange_fock(3, 4, FAKE, 2, FAKE, FAKE, 0, FAKE, big, None) == nof.E_DTYPE
    assert L.nof_exchange_fock(3, 4, FAKE, 0, FAKE, FAKE, 1, FAKE, big, None) == nof.E_PREC
    assert L.nof_exchange_fock(3, 4, FAKE, 1, FAKE, FAKE, 0, FAKE, big, None) == nof.E_PREC
    assert L.nof_exchange_fock(3, 4, FAKE, 0, FAKE, FAKE, 0, FAKE, 8, None) == nof.E_WORKSPACE
    assert L.nof_exchange_fock_ws(3, 4, 0, 1) == 0
    assert L.nof_exchange_fock_ws(3, 4, 1, nof.P_BF16X10) >= 3 * 4 * 4 * 8 // 3
    # fixed-point planes of B: [4][naux][nbf][ldk], ldk = nbf rounded up to 32
    assert L.nof_split_B_bytes(2, 33) == 4 * 2 * 33 * 64 * 2
    assert L.nof_split_B_bytes(0, 33) == 0
    assert L.nof_split_B(2, 4, FAKE, nof.BF16, FAKE, big, None) == nof.E_DTYPE
    assert L.nof_split_B(2, 4, None, nof.F32, FAKE, big, None) == nof.E_NULL
    assert L.nof_split_B(2, 4, FAKE, nof.F32, FAKE, 8, None) == nof.E_WORKSPACE
    # planes are accepted by the x10 transform only
    assert L.nof_mo_transform(2, 4, 4, FAKE, nof.BF16X4, FAKE, FAKE, 1, None, nof.P_BF16X6, FAKE, big, None) == nof.E_DTYPE
    # stage workspace: FP64/FP32 need none of substance; x10 holds C planes and grid exponents
    assert L.nof_mo_transform_stage_ws(2, 40, 30, nof.P_F64) > 0
    x10 = L.nof_mo_transform_stage_ws(2, 40, 30, nof.P_BF16X10)
    assert x10 >= 4 * 30 * 64 * 2 + 2 * 40 * 4
    assert L.nof_mo_transform_stage_ws(0, 40, 30, nof.P_BF16X10) == 0
    assert L.nof_mo_transform_stage1(2, 40, 30, FAKE, nof.F32, FAKE, FAKE, nof.F32, nof.P_BF16X10,
                                     FAKE, x10 - 1, None) == nof.E_WORKSPACE


def test_solve_validation():
    import ctypes
    nof = _lib()
    L = nof.lib
    prm = nof.SolveParams(10, 30, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10)
    res = nof.SolveResult()
    args = lambda B, p, ws_bytes: (2, 4, 4, B, 0, FAKE, FAKE, 1, 1, FAKE, 1, 1, FAKE, None, 0,
                                   ctypes.byref(p), ctypes.byref(res), FAKE, ws_bytes, None)
    assert L.nof_solve(*args(None, prm, 1 << 30)) == nof.E_NULL
    bad = nof.SolveParams(0, 30, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10)
    assert L.nof_solve(*args(FAKE, bad, 1 << 30)) == nof.E_ARG
    bad = nof.SolveParams(10, 30, 0.0, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10)
    assert L.nof_solve(*args(FAKE, bad, 1 << 30)) == nof.E_ARG
    bad = nof.SolveParams(10, 30, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, -1.0)
    assert L.nof_solve(*args(FAKE, bad, 1 << 30)) == nof.E_ARG
    assert L.nof_solve(*args(FAKE, prm, 8)) == nof.E_WORKSPACE
    assert L.nof_solve_ws(2, 4, 4, 1, 1, 0, nof.P_BF16X1) == 0
    # iterative diagonalization needs a positive off-diagonal bound
    bad = nof.SolveParams(10, 30, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10, 1, 0.0)
    assert L.nof_solve(*args(FAKE, bad, 1 << 30)) == nof.E_ARG


def test_pseudo_fock_diag_validation():
    nof = _lib()
    L = nof.lib
    need = L.nof_pseudo_fock_diag_ws(5)
    assert need >= 3 * 6 * 6 * 8 and L.nof_pseudo_fock_diag_ws(0) == 0 and L.nof_pseudo_fock_diag_ws(70000) == 0
    assert L.nof_pseudo_fock_diag(0, FAKE, None, 1.0, FAKE, None, None, FAKE, need, None) == nof.E_DIM
    assert L.nof_pseudo_fock_diag(5, None, None, 1.0, FAKE, None, None, FAKE, need, None) == nof.E_NULL
    assert L.nof_pseudo_fock_diag(5, FAKE, None, 1.0, None, None, None, FAKE, need, None) == nof.E_NULL
    assert L.nof_pseudo_fock_diag(5, FAKE, None, 0.0, FAKE, None, None, FAKE, need, None) == nof.E_ARG
    assert L.nof_pseudo_fock_diag(5, FAKE, None, float("nan"), FAKE, None, None, FAKE, need, None) == nof.E_ARG
    assert L.nof_pseudo_fock_diag(5, FAKE, None, 1.0, FAKE, None, None, FAKE, need - 1, None) == nof.E_WORKSPACE
    assert L.nof_solve_ws(2, 4, 4, 1, 1, 0, nof.P_F64) > 2 * 4 * 4 * 8


def test_nlop_validation():
    nof = _lib()
    L = nof.lib
    assert L.nof_dipole(0, 4, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == nof.E_DIM
    assert L.nof_dipole(4, 4, None, FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == nof.E_NULL
    assert L.nof_dipole(4, 4, FAKE, FAKE, FAKE, FAKE, FAKE, 8, None) == nof.E_WORKSPACE
    assert L.nof_dipole_ws(4, 4) > 4 * 4 * 8
    assert L.nof_nlop_romberg(0, 1e-3, FAKE, FAKE, FAKE, FAKE, FAKE, None) == nof.E_DIM
    assert L.nof_nlop_romberg(17, 1e-3, FAKE, FAKE, FAKE, FAKE, FAKE, None) == nof.E_DIM
    assert L.nof_nlop_romberg(3, 0.0, FAKE, FAKE, FAKE, FAKE, FAKE, None) == nof.E_ARG
    assert L.nof_nlop_romberg(3, 1e-3, None, FAKE, FAKE, FAKE, FAKE, None) == nof.E_NULL
    assert L.nof_nlop_isotropic(None, FAKE, None) == nof.E_NULL


def test_plan_solve_validation():
    import ctypes
    nof = _lib()
    L = nof.lib
    plan = ctypes.c_void_p()
    assert L.nof_plan_create(ctypes.byref(plan), 3, 16, 8, 8, nof.P_F64) == nof.OK
    try:
        need = L.nof_plan_solve_ws(plan, 2, 1)
        assert need > L.nof_plan_ws(plan) + 3 * 9 * 8 * 8 * 8   # plan + nine norb^2 arrays per instance
        assert L.nof_plan_solve_ws(plan, 3, 2) == 0                # 3 x (2+1) > norb
        assert L.nof_plan_solve_ws(None, 2, 1) == 0
        prm = nof.SolveParams(10, 30, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10)
        res = (nof.SolveResult * 3)()
        args = lambda pl, B, p, ws_bytes: (pl, B, FAKE, FAKE, 2, 1, FAKE, 1, 1, FAKE, None,
                                           ctypes.byref(p), res, FAKE, ws_bytes, None)
        assert L.nof_plan_solve(*args(None, FAKE, prm, need)) == nof.E_NULL
        assert L.nof_plan_solve(*args(plan, None, prm, need)) == nof.E_NULL
        bad = nof.SolveParams(10, 0, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10)
        assert L.nof_plan_solve(*args(plan, FAKE, bad, need)) == nof.E_ARG
        bad = nof.SolveParams(10, 30, 0.01, 1.0, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10)
        assert L.nof_plan_solve(*args(plan, FAKE, bad, need)) == nof.E_ARG
        bad = nof.SolveParams(10, 30, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, float("nan"))
        assert L.nof_plan_solve(*args(plan, FAKE, bad, need)) == nof.E_ARG
        bad = nof.SolveParams(10, 30, 0.01, 0.9, 0.999, 1e-8, 1e-5, 1e-9, 100, 1e-8, 1e-10, 1, 1.0)
        assert L.nof_plan_solve(*args(plan, FAKE, bad, need)) == nof.E_ARG
        assert L.nof_plan_solve(*args(plan, FAKE, prm, need - 1)) == nof.E_WORKSPACE
    finally:
        L.nof_plan_destroy(plan)


def test_orthonormalize_validation():
    nof = _lib()
    L = nof.lib
    need = L.nof_orthonormalize_ws(40, 30)
    assert need > 2 * 30 * 30 * 8 + 40 * 30 * 8
    assert L.nof_orthonormalize_ws(0, 30) == 0
    assert L.nof_orthonormalize(0, 30, FAKE, None, 1e-10, None, FAKE, need, None) == nof.E_DIM
    assert L.nof_orthonormalize(40, 30, None, None, 1e-10, None, FAKE, need, None) == nof.E_NULL
    assert L.nof_orthonormalize(40, 30, FAKE, None, -1.0, None, FAKE, need, None) == nof.E_ARG
    assert L.nof_orthonormalize(40, 30, FAKE, None, float("nan"), None, FAKE, need, None) == nof.E_ARG
    assert L.nof_orthonormalize(40, 30, FAKE, None, 1e-10, None, FAKE, need - 1, None) == nof.E_WORKSPACE


# ---- host-side bounds check of the batched plans' workspace layouts ----
PLAN_REGIONS = ["Call", "T", "b", "D", "TH", "h", "J", "K", "W", "Kpart", "F1part", "F2part", "F1", "F2",
                "Epart", "Cplanes", "Tcolmax", "Texp", "cKT", "Tplanes"]


@pytest.mark.parametrize("ninst,naux,nbf,norb", [(25, 1200, 300, 300), (3, 7, 33, 17), (1, 1, 1, 1),
                                                 (4, 40, 130, 97), (2, 300, 1100, 150)])
@pytest.mark.parametrize("prec", ["f64", "f32", "x10", "i8x10"])
def test_plan_layout_regions_fit_the_workspace(ninst, naux, nbf, norb, prec):
    """Every region of every plan layout (field300 x10 included) is 256-byte
    aligned, disjoint from the others, ends inside nof_plan_ws, and is at least
    as large as what the iteration writes there (computed here from the
    documented layout), also for the largest exchange split the tuner may set."""
    import ctypes
    nof = _lib()
    L = nof.lib
    p = {"f64": nof.P_F64, "f32": nof.P_F32, "x10": nof.P_BF16X10, "i8x10": nof.P_I8X10}[prec]
    plan = ctypes.c_void_p()
    assert L.nof_plan_create(ctypes.byref(plan), ninst, naux, nbf, norb, p) == 0
    try:
        total = L.nof_plan_ws(plan)
        off = (ctypes.c_size_t * 32)()
        size = (ctypes.c_size_t * 32)()
        n = L.nof_plan_layout(plan, off, size, 32)
        assert n == len(PLAN_REGIONS)
        regions = [(PLAN_REGIONS[i], off[i], size[i]) for i in range(n)]
        for name, o, sz in regions:
            assert o % 256 == 0, name
            assert o + sz <= total, (name, o, sz, total)
        spans = sorted((o, o + sz, name) for name, o, sz in regions if sz > 0)
        for (a0, a1, na), (b0, b1, nb) in zip(spans, spans[1:]):
            assert a1 <= b0, (na, nb)
        # the largest exchange-term split the tuner may set (host-only calls)
        cfg = (ctypes.c_int * 4)()
        assert L.nof_plan_get_config(plan, cfg) == 0
        gmax = 1
        while True:
            cfg[3] = gmax + 1
            if L.nof_plan_set_config(plan, cfg) != 0:
                break
            gmax += 1
        es = 8 if prec == "f64" else 4
        n2 = norb * norb * 8
        ldc = ninst * norb
        need = {"Call": nbf * ldc * 8, "T": naux * nbf * ldc * es, "b": ninst * naux * norb * norb * es,
                "D": ninst * naux * norb * 8, "TH": ninst * nbf * norb * 8, "h": ninst * n2, "J": ninst * n2,
                "K": ninst * n2, "W": ninst * naux * norb * 8, "Kpart": ninst * n2,
                "F2part": ninst * gmax * n2, "F2": ninst * n2, "Epart": ninst * 8}
        if prec == "f64":
            # the per-q symmetric products of every instance, q values at a
            # time within 4 GiB, in place of the exchange-term partials
            gq = min(norb, max(1, (4 << 30) // (ninst * n2)))
            need["F2part"] = ninst * gq * n2
        if prec in ("x10", "i8x10", "f64"):
            need.update({"F1part": ninst * n2, "F1": ninst * n2})
        else:
            # FP32: the Coulomb-type term rides in the exchange-type product
            # (F2 holds F2 - F1): its partials and sum need no space
            assert size[PLAN_REGIONS.index("F1part")] == 0 and size[PLAN_REGIONS.index("F1")] == 0
        if prec == "x10":
            ldk = (nbf + 31) // 32 * 32
            need.update({"Cplanes": 4 * ldc * ldk * 2, "Tcolmax": naux * ((nbf + 127) // 128) * ldc * 4,
                         "Texp": naux * ldc * 4, "cKT": ninst * norb * norb * 4})
        if prec == "i8x10":
            ldk8 = (nbf + 63) // 64 * 64
            need.update({"Cplanes": 4 * ldc * ldk8 + ldc * 4, "Tcolmax": naux * ((nbf + 127) // 128) * ldc * 4,
                         "Texp": naux * ldc * 4, "cKT": ninst * norb * norb * 4, "Tplanes": 4 * naux * ldc * ldk8})
        else:
            assert size[PLAN_REGIONS.index("Tplanes")] == 0
        for name, o, sz in regions:
            assert sz >= need.get(name, 0), (name, sz, need.get(name))
    finally:
        L.nof_plan_destroy(plan)
