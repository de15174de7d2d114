"""Batched finite-field form: one plan for many instances sharing B, checked
against the single-instance C ABI (same library, already pinned to the
oracle) and directly against the oracle; every tile configuration, the
autotuner, and graph capture with several replays."""
import numpy as np
import pytest
import torch

from oracle import dfjk, functionals
from paper_2512_13550_amd import inputs
from gpu_util import dev, host, need_gpu, normwise

pytestmark = pytest.mark.gpu


def instances(nbf, naux, norb, ninst, seed, ns):
    B = inputs.make_B(seed, nbf, naux, 25.0)
    fi = inputs.field_instances(seed, nbf, norb, ns, ninst)
    ng = max(1, (norb - ns) // ns)
    members = np.array(inputs.pairing(norb, ns, ng))
    cJ = np.empty((ninst, norb, norb)); cK = np.empty_like(cJ)
    for i in range(ninst):
        cJ[i], cK[i] = functionals.coefficients(fi["n"][i], members, "pnof5")
    return B, fi["C"], fi["H"], fi["n"], cJ, cK


def single(nof, Bd, C, H, n, cJ, cK, prec):
    Cd = dev(C)
    b, D = nof.mo_transform(Bd, Cd, prec=prec)
    h = nof.one_electron(dev(H), Cd)
    J, K = nof.jk_diag(b, D)
    lam, g, _ = nof.gen_fock(b, D, dev(n), h, dev(cJ), dev(cK), prec=prec)
    E = nof.energy(dev(n), h, J, K, dev(cJ), dev(cK))
    return float(E), host(lam), host(g)


@pytest.mark.parametrize("prec_name", ["f64", "f32"])
def test_batch_matches_single_instance_every_config(prec_name):
    nof = need_gpu()
    ninst, nbf, naux, norb = 6, 130, 90, 110
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3001, 27)
    tdt = torch.float64 if prec_name == "f64" else torch.float32
    prec = nof.P_F64 if prec_name == "f64" else nof.P_F32
    Bd = dev(B, tdt)
    plan = nof.BatchPlan(Bd, dev(C), dev(H), dev(n), dev(cJ), dev(cK), prec=prec)
    ref = [single(nof, Bd, C[i], H[i], n[i], cJ[i], cK[i], prec) for i in range(ninst)]
    tol = 1e-12 if prec_name == "f64" else 2e-6
    # the last two: one P per exchange group (fold 1, the default split of small
    # plans), where the partials of instance i must not land on instance 0's
    for cfg in ([128, 128, 128, 1], [64, 64, 64, 2], [64, 128, 64, 1], [128, 64, 128, 3],
                [128, 128, 128, naux], [64, 64, 64, naux]):
        plan.config = cfg
        E, lam, g = plan.iteration()
        torch.cuda.synchronize()
        for i in range(ninst):
            assert abs(float(E[i]) - ref[i][0]) <= tol * abs(ref[i][0]), (cfg, i)
            assert normwise(host(lam[i]), ref[i][1]) <= tol, (cfg, i)
            assert normwise(host(g[i]), ref[i][2]) <= tol * 10, (cfg, i)
    if prec_name == "f64":
        for i in (0, ninst - 1):
            o = dfjk.iteration(B, C[i], H[i], n[i], cJ[i], cK[i])
            assert abs(float(E[i]) - o["E"]) <= 1e-10 * abs(o["E"])
            assert normwise(host(lam[i]), o["lam"]) <= 1e-10


@pytest.mark.parametrize("src", ["f32", "f64"])
def test_batch_x10_matches_single_instance(src):
    """The fixed-point (x10) plan: B as planes, the packed C split once, stage
    2 and the exchange-type term instance by instance; every instance equals
    the single-instance x10 path (same grids and products; only the grouping
    of FP64 partial sums differs), for several exchange splits and after the
    autotuner, and one instance against the oracle on the FP32-rounded B."""
    nof = need_gpu()
    print(f"case batched x10 from {src}", flush=True)
    ninst, nbf, naux, norb = 5, 130, 90, 110
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3002, 27)
    Bin = B.astype(np.float32).astype(np.float64) if src == "f32" else B
    Bs = nof.SplitB(dev(Bin, torch.float32 if src == "f32" else torch.float64))
    plan = nof.BatchPlan(Bs, dev(C), dev(H), dev(n), dev(cJ), dev(cK))
    assert plan.prec == nof.P_BF16X10
    ref = [single(nof, Bs, C[i], H[i], n[i], cJ[i], cK[i], nof.P_BF16X10) for i in range(ninst)]
    same = {}
    for cfg in ([128, 128, 128, 1], [128, 128, 128, 3], [128, 128, 128, naux], [64, 64, 64, 3],
                [64, 128, 64, 1], [128, 64, 128, naux], None):
        if cfg is None:
            plan.autotune()
        else:
            plan.config = cfg
        E, lam, g = plan.iteration()
        torch.cuda.synchronize()
        if cfg is not None:
            # every output element is summed in the same order at either tile
            # edge: configurations with the same exchange split agree exactly
            got = (host(E), host(lam), host(g))
            if cfg[3] in same:
                for u, v in zip(got, same[cfg[3]]):
                    assert np.array_equal(u, v), cfg
            same[cfg[3]] = got
        for i in range(ninst):
            assert abs(float(E[i]) - ref[i][0]) <= 1e-12 * abs(ref[i][0]), (cfg, i)
            assert normwise(host(lam[i]), ref[i][1]) <= 1e-12, (cfg, i)
            assert normwise(host(g[i]), ref[i][2]) <= 1e-10, (cfg, i)
    o = dfjk.iteration(Bin, C[1], H[1], n[1], cJ[1], cK[1])
    assert abs(float(E[1]) - o["E"]) <= 2e-8 * abs(o["E"])
    assert normwise(host(lam[1]), o["lam"]) <= 3e-7


def test_batch_i8x10_matches_single_instance():
    """The INT8 fixed-point plan: B as INT8 planes, the packed C split once,
    T split into planes of its columns and stage 2 for all instances.  The
    INT8 sums are exact and every instance gets the same grids as alone, so b
    is bit-identical to the single-instance INT8 path and E (from J and K)
    equal to 1e-12.  The plan takes the exchange-type term as the x10 product
    of the batched fixed-point plans (one launch for every instance), the
    single-instance INT8 path as INT8 products over groups of slabs: lambda
    and g agree within the forms' shared bound of 3e-7, for several exchange
    splits and after the autotuner; one instance against the oracle."""
    nof = need_gpu()
    print("case batched i8x10", flush=True)
    ninst, nbf, naux, norb = 5, 130, 90, 110
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3003, 27)
    Bs = nof.SplitBI8(dev(B))
    plan = nof.BatchPlan(Bs, dev(C), dev(H), dev(n), dev(cJ), dev(cK))
    assert plan.prec == nof.P_I8X10
    ref = [single(nof, Bs, C[i], H[i], n[i], cJ[i], cK[i], nof.P_I8X10) for i in range(ninst)]
    same = {}
    for cfg in ([128, 128, 128, 1], [128, 128, 128, 3], [128, 128, 64, 3], [64, 64, 64, 1], None):
        if cfg is None:
            plan.autotune()
        else:
            plan.config = cfg
        E, lam, g = plan.iteration()
        torch.cuda.synchronize()
        if cfg is not None:
            # the exchange-type product at a 64 or 128 tile edge (the INT8
            # transform has one): same exchange split, same results
            got = (host(E), host(lam), host(g))
            if cfg[3] in same:
                for u, v in zip(got, same[cfg[3]]):
                    assert np.array_equal(u, v), cfg
            same[cfg[3]] = got
        for i in range(ninst):
            assert abs(float(E[i]) - ref[i][0]) <= 1e-12 * abs(ref[i][0]), (cfg, i)
            assert normwise(host(lam[i]), ref[i][1]) <= 3e-7, (cfg, i)
            assert normwise(host(g[i]), ref[i][2]) <= 8 * 3e-7 * np.max(np.abs(ref[i][1])) / np.max(np.abs(ref[i][2])), \
                (cfg, i)
    o = dfjk.iteration(B, C[2], H[2], n[2], cJ[2], cK[2])
    assert abs(float(E[2]) - o["E"]) <= 2e-8 * abs(o["E"])
    assert normwise(host(lam[2]), o["lam"]) <= 3e-7


def test_batch_x10_tile_edges_long_contraction():
    """Nbf above 1024: both transform stages of the x10 plan add their
    order-0 FP32 sums to FP64 every 1024 terms.  The 64-wide tiles (two
    workgroups per CU, four waves) give exactly the 128-wide tiles' results
    there too, with ragged edges in every tiled dimension (Nbf = 1100, Norb =
    70, two instances: 140 packed columns)."""
    nof = need_gpu()
    print("case batched x10 tile edges, nbf 1100", flush=True)
    ninst, nbf, naux, norb = 2, 1100, 6, 70
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3004, 9)
    Bs = nof.SplitB(dev(B))
    plan = nof.BatchPlan(Bs, dev(C), dev(H), dev(n), dev(cJ), dev(cK))
    out = []
    for cfg in ([128, 128, 128, 2], [64, 64, 64, 2], [64, 128, 128, 2], [128, 64, 64, 2]):
        plan.config = cfg
        E, lam, g = plan.iteration()
        torch.cuda.synchronize()
        out.append((host(E), host(lam), host(g)))
    for o in out[1:]:
        for u, v in zip(o, out[0]):
            assert np.array_equal(u, v)
    ref = single(nof, Bs, C[1], H[1], n[1], cJ[1], cK[1], nof.P_BF16X10)
    assert abs(float(out[0][0][1]) - ref[0]) <= 1e-12 * abs(ref[0])
    assert normwise(out[0][1][1], ref[1]) <= 1e-12


@pytest.mark.parametrize("prec_name", ["f64", "f32", "x10", "i8x10"])
def test_plan_writes_stay_inside_workspace(prec_name):
    """Every region of a plan's workspace lies inside the nof_plan_ws bytes it
    reports: the workspace is a view into a larger buffer whose tail holds a
    sentinel, and after iterations, the autotuner, a capture and graph replays
    the tail is unchanged and the replayed energies equal the eager ones."""
    nof = need_gpu()
    print(f"case plan workspace bounds {prec_name}", flush=True)
    ninst, nbf, naux, norb = 4, 100, 70, 96
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3002, 24)
    if prec_name == "x10":
        Bp = nof.SplitB(dev(B))
    elif prec_name == "i8x10":
        Bp = nof.SplitBI8(dev(B))
    else:
        Bp = dev(B, torch.float32 if prec_name == "f32" else torch.float64)
    plan = nof.BatchPlan(Bp, dev(C), dev(H), dev(n), dev(cJ), dev(cK))
    need = plan.ws.numel()
    tail = 64 << 20
    big = torch.empty(need + tail, dtype=torch.uint8, device=plan.ws.device)
    big[need:] = 0xA5
    plan.ws = big[:need]
    E0 = plan.iteration()[0].clone()
    plan.autotune()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
        for _ in range(2):
            plan.launch(s)
    s.synchronize()
    Eg = plan.E.clone()
    E1 = plan.iteration()[0].clone()
    torch.cuda.synchronize()
    assert bool((big[need:] == 0xA5).all())
    assert torch.equal(Eg, E1)
    # the tuner may change the FP32 tiles (summation order of the products)
    tol = 1e-6 if prec_name == "f32" else 1e-10
    assert float((E0 - E1).abs().max()) <= tol * float(E1.abs().max())


def test_autotune_and_graph_replays():
    nof = need_gpu()
    ninst, nbf, naux, norb = 9, 100, 70, 96
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3002, 24)
    Cd = dev(C)
    plan = nof.BatchPlan(dev(B), Cd, dev(H), dev(n), dev(cJ), dev(cK))
    cfg = plan.autotune()
    print("tuned config", cfg, flush=True)
    assert cfg[0] in (64, 128) and cfg[1] in (64, 128) and cfg[2] in (64, 128) and cfg[3] >= 1
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
    s.synchronize()
    rng = np.random.default_rng(0)
    for rep in range(3):
        # eager work between replays: new orbitals written in place
        y = inputs.make_antisym(7, rep, norb, 0.05)
        C2 = np.stack([C[i] @ np.asarray(__import__("scipy").linalg.expm(y)) for i in range(ninst)])
        Cd.copy_(dev(C2))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            plan.launch(s)
        s.synchronize()
        Eg, lg, gg = host(plan.E).copy(), host(plan.lam).copy(), host(plan.g).copy()
        E2, l2, g2 = plan.iteration()
        torch.cuda.synchronize()
        assert np.array_equal(Eg, host(E2)), rep
        assert np.array_equal(lg, host(l2)), rep
        assert np.array_equal(gg, host(g2)), rep
        o = dfjk.iteration(B, C2[rep], H[rep], n[rep], cJ[rep], cK[rep])
        assert abs(Eg[rep] - o["E"]) <= 1e-10 * abs(o["E"])


def test_field_workload_fp32_against_oracle():
    """The 25-instance field workload (Nbf=300, Naux=1200, Norb=300) in FP32
    with tuned tiles, checked on two instances against the FP64 oracle."""
    nof = need_gpu()
    w = inputs.WORKLOADS["field300"]
    print("case field300 fp32", flush=True)
    B, C, H, n, cJ, cK = instances(w.nbf, w.naux, w.norb, 25, w.seed, w.nstrong)
    plan = nof.BatchPlan(dev(B, torch.float32), dev(C), dev(H), dev(n), dev(cJ), dev(cK),
                         prec=nof.P_F32)
    plan.autotune()
    E, lam, g = plan.iteration()
    torch.cuda.synchronize()
    for i in (0, 24):
        o = dfjk.iteration(B, C[i], H[i], n[i], cJ[i], cK[i])
        print("field instance", i, "dE", float(E[i]) - o["E"], flush=True)
        assert abs(float(E[i]) - o["E"]) <= 1e-7 * abs(o["E"])
        assert normwise(host(lam[i]), o["lam"]) <= 2e-6


@pytest.mark.parametrize("prec_name", ["f64", "f32"])
def test_batch_odd_norb_default_and_fold1(prec_name):
    """Odd Norb (the pass takes its unaligned-pair path), three instances, the
    plan's default split and one P per exchange group, against the
    single-instance entry points."""
    nof = need_gpu()
    ninst, nbf, naux, norb = 3, 40, 20, 37
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3003, 9)
    tdt = torch.float64 if prec_name == "f64" else torch.float32
    prec = nof.P_F64 if prec_name == "f64" else nof.P_F32
    Bd = dev(B, tdt)
    plan = nof.BatchPlan(Bd, dev(C), dev(H), dev(n), dev(cJ), dev(cK), prec=prec)
    ref = [single(nof, Bd, C[i], H[i], n[i], cJ[i], cK[i], prec) for i in range(ninst)]
    tol = 1e-12 if prec_name == "f64" else 2e-6
    for cfg in (None, [64, 64, 64, naux]):
        if cfg is not None:
            plan.config = cfg
        E, lam, g = plan.iteration()
        torch.cuda.synchronize()
        for i in range(ninst):
            assert abs(float(E[i]) - ref[i][0]) <= tol * abs(ref[i][0]), (cfg, i)
            assert normwise(host(lam[i]), ref[i][1]) <= tol, (cfg, i)


@pytest.mark.parametrize("prec_name", ["x10", "i8x10"])
@pytest.mark.parametrize("nbf", [40, 100])
def test_batch_fixed_point_stage1_layouts(prec_name, nbf):
    """Stage 1 of the fixed-point plans takes the rows of all slabs as one
    product when a slab holds a whole tile of rows (Nbf >= the tile edge: the
    x10 plan at 64 for Nbf = 100), else one product per slab (Nbf = 40, and
    Nbf = 100 at 128 or in the INT8 plan); T's column grids come from the
    per-slab maxima either way.  Against the single-instance path (which
    never folds): E to 1e-12; lambda to 1e-12 (x10: same products) or the
    forms' 3e-7 (INT8: the plan's exchange-type term is the x10 one); the
    x10 plan's two layouts agree exactly."""
    nof = need_gpu()
    print(f"case batched {prec_name} stage-1 layouts nbf {nbf}", flush=True)
    ninst, naux, norb = 3, 20, 37
    B, C, H, n, cJ, cK = instances(nbf, naux, norb, ninst, 3005, 9)
    Bs = nof.SplitB(dev(B)) if prec_name == "x10" else nof.SplitBI8(dev(B))
    prec = nof.P_BF16X10 if prec_name == "x10" else nof.P_I8X10
    plan = nof.BatchPlan(Bs, dev(C), dev(H), dev(n), dev(cJ), dev(cK))
    ref = [single(nof, Bs, C[i], H[i], n[i], cJ[i], cK[i], prec) for i in range(ninst)]
    tl = 1e-12 if prec_name == "x10" else 3e-7
    out = []
    for cfg in ([128, 128, 128, 2], [64, 128, 128, 2]):
        plan.config = cfg
        E, lam, g = plan.iteration()
        torch.cuda.synchronize()
        out.append((host(E), host(lam), host(g)))
        for i in range(ninst):
            assert abs(float(E[i]) - ref[i][0]) <= 1e-12 * abs(ref[i][0]), (cfg, i)
            assert normwise(host(lam[i]), ref[i][1]) <= tl, (cfg, i)
    for u, v in zip(out[0], out[1]):
        assert np.array_equal(u, v)
