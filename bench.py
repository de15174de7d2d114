#!/usr/bin/env python
"""Benchmark of one orbital-optimisation iteration of the density-fitted JK +
generalized-Fock build on one MI355X.

Workload (default "c500"): Nbf=500, Naux=2000, Norb=500, synthetic
hydrogen-chain-shaped inputs (see paper_2512_13550_amd/inputs.py), 125
strongly occupied orbitals each paired with three weak ones, ten iterations
each preceded by a small random orthogonal rotation of C.

One step = one iteration: C <- C exp(eps Y_i) (FP64 rotation on the GPU),
b = C^T B C and D, h = C^T H C, J, and in one call lambda, g and K, then E.
All inputs are resident in HBM before the timed region starts.

Prints ONE JSON line.  `value` is the algorithmic TFLOP/s of the FP64 path;
`forms` holds the FP32 form on the same workload with its error against the
FP64 GPU result; `roofline` describes the dominant kernel (the first stage of
the orbital transformation) timed with HIP events on the launch stream;
`cpu_baseline` is the FP64 CPU oracle timed on a bounded slab sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # dense MFMA TFLOP/s (MI355X datasheet)
HBM_PEAK_GBS = 8000.0


def algorithmic_flops(nbf, naux, norb):
    a1 = 2.0 * naux * nbf * nbf * norb                 # T^P = B^P C
    a2 = 1.0 * naux * nbf * norb * (norb + 1)          # b^P = C^T T^P, symmetric half
    a6 = 2.0 * naux * norb ** 3                        # exchange-type Fock contraction
    small = 6.0 * naux * norb * norb                   # J, K, W, F1
    dense = a1 + 2.0 * naux * nbf * norb * norb + a6   # the three products as dense GEMMs
    return dict(a1=a1, a2=a2, a6=a6, small=small, total=a1 + a2 + a6 + small, dense=dense)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c500")
    ap.add_argument("--forms", default="f32,bf16x3,bf16x6,bf16x10,bf16x10f32,bf16B",
                    help="comma list of extra forms: f32, bf16x1, bf16x3, bf16x6, bf16x10 (B split "
                         "once into fixed-point planes from FP64), bf16x10f32 (FP32 B split in the "
                         "loader), bf16B (B stored in BF16)")
    ap.add_argument("--cpu-slabs", type=int, default=160,
                    help="auxiliary slabs in the CPU-oracle sample (0 = skip)")
    ap.add_argument("--batched", type=int, default=1,
                    help="1: also time the 25-instance finite-field batch (graph launch); "
                         "2: time only that batch and print its record (for kernel profiles)")
    ap.add_argument("--precision-workload", default="chain1000",
                    help="also time FP64 against the x10 forms on this workload in a child run "
                         "('' = skip)")
    ap.add_argument("--warmstart", type=int, default=0,
                    help="train the warm-start network on this many instances and evaluate it")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="bytes of a plain read+write kernel run 3 times after timing "
                         "(counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--traffic-file", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                           "profiles", "traffic_fp64_c500.json"))
    return ap.parse_args()


def kernel_source_digest():
    """Digest of the sources of the timed kernel (the traffic figure is stale
    once they change)."""
    import hashlib
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2512_13550_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(root, "gemm_tn.hip"), "rb") as f:
        h.update(f.read())
    with open(os.path.join(root, "common.h"), "rb") as f:      # the descriptor it reads
        txt = f.read()
    i = txt.index(b"struct GemmDesc {")
    h.update(txt[i:txt.index(b"};", i)])
    return h.hexdigest()[:16]


def load_traffic(path, kernel):
    """HBM bytes per launch of a kernel from a committed counter summary, or
    None when absent or taken on other kernel sources."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != kernel_source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return k.get("bytes_per_launch") if k else None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2512_13550_amd.nof as nof
    from paper_2512_13550_amd import inputs

    if args.batched == 2:
        rec = run_batched(nof, inputs, torch.device("cuda:0"), steps=args.steps)
        print(json.dumps({"batched": rec}))
        return
    w = inputs.WORKLOADS[args.workload]
    nbf, naux, norb = w.nbf, w.naux, w.norb
    t0 = time.time()
    print(f"# generating {w.name}: nbf={nbf} naux={naux} norb={norb}", file=sys.stderr, flush=True)
    B_h = inputs.make_B(w.seed, nbf, naux, w.decay, threads=16)
    C0 = inputs.make_C(w.seed, nbf, norb)
    H_h = inputs.make_H(w.seed, nbf)
    n_h = inputs.make_occupations(w.seed, norb, w.nstrong)
    total_iters = max(args.warmup + args.steps, w.iters)
    Ys = [inputs.make_antisym(w.seed, it, norb) for it in range(total_iters)]
    print(f"# inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    B64 = torch.from_numpy(B_h).to(dev)
    H = torch.from_numpy(H_h).to(dev)
    n = torch.from_numpy(n_h).to(dev)
    Yd = [torch.from_numpy(Y).to(dev) for Y in Ys]
    Z = torch.zeros((norb, norb), dtype=torch.float64, device=dev)
    # HF-like reconstruction (Delta = Pi = 0): dense coefficient matrices
    cJ, cK = nof.coeffs_from_cumulant(n, Z, Z)

    flops = algorithmic_flops(nbf, naux, norb)

    PRECS = {"f64": nof.P_F64, "f32": nof.P_F32, "bf16x1": nof.P_BF16X1, "bf16x3": nof.P_BF16X3,
             "bf16x6": nof.P_BF16X6, "bf16x10": nof.P_BF16X10, "bf16x10f32": nof.P_BF16X10,
             "bf16B": nof.P_BF16X6}

    def run(B, prec_name, steps, warmup):
        dt = torch.float64 if prec_name == "f64" else torch.float32
        prec = PRECS[prec_name]
        C = torch.from_numpy(C0).to(dev)
        Cn = torch.empty_like(C)
        # x10: both stages in one nof_mo_transform call (the first stage's
        # epilogue gives the second its column grids); the others call the
        # stages separately, so that each is timed on its own
        fused = prec == nof.P_BF16X10
        names = (["rotate"] + (["a1_a2_transform"] if fused else ["a1_transform_stage1", "a2_transform_stage2"])
                 + ["h_and_J", "fock_K_lambda_grad", "energy"])
        if fused:
            T = None
            ws_t = nof.workspace(nof.lib.nof_mo_transform_ws(naux, nbf, norb, nof._b_arg(B)[0], nof._TDT[dt], prec),
                                 dev)
        else:
            T = torch.empty((naux, nbf, norb), dtype=dt, device=dev)
        b = torch.empty((naux, norb, norb), dtype=dt, device=dev)
        D = torch.empty((naux, norb), dtype=torch.float64, device=dev)
        out = {"lam": torch.empty_like(Z), "g": torch.empty_like(Z), "K": torch.empty_like(Z)}
        J = torch.empty_like(Z)
        E = torch.empty((), dtype=torch.float64, device=dev)
        rot = nof.Rotation(norb, nbf, dev)
        ws_f = nof.workspace(nof.lib.nof_gen_fock_ws(naux, norb, nof._TDT[dt], prec), dev)
        ws_j = nof.workspace(nof.lib.nof_jk_diag_ws(naux, norb, nof._TDT[dt]), dev)
        ws_e = nof.workspace(nof.lib.nof_energy_ws(norb), dev)
        Es = []
        nev = len(names) + 1
        evs = []

        def one(it, record):
            nonlocal C, Cn
            e = [torch.cuda.Event(enable_timing=True) for _ in range(nev)] if record else []
            mark = iter(e)

            def tick():
                if record:
                    next(mark).record()
            tick()
            rot.apply(C, Yd[it], Cn)                                  # A9: C <- C exp(eps Y)
            C, Cn = Cn, C
            tick()
            if fused:
                nof.mo_transform(B, C, prec=prec, b=b, D=D, ws=ws_t)   # A1 + A2
            else:
                nof.transform_stage1(B, C, T, prec=prec)              # A1
                tick()
                nof.transform_stage2(T, C, b, D, prec=prec)           # A2
            tick()
            h = nof.one_electron(H, C)
            nof.jk_diag(b, D, want_J=True, want_K=False, J=J, ws=ws_j)   # A3
            tick()
            nof.gen_fock(b, D, n, h, cJ, cK, want_grad=True, want_K=True, prec=prec,
                         out=out, ws=ws_f)                            # A4-A7
            tick()
            nof.energy(n, h, J, out["K"], cJ, cK, E=E, ws=ws_e)      # A8
            tick()
            return e

        for it in range(warmup):
            one(it, False)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for k in range(steps):
            evs.append(one(warmup + k, True))
            Es.append(E.clone())
        stop.record()
        torch.cuda.synchronize()
        total_ms = start.elapsed_time(stop)
        seg = np.array([[ev[i].elapsed_time(ev[i + 1]) for i in range(nev - 1)] for ev in evs])
        per_step = [ev[0].elapsed_time(ev[nev - 1]) for ev in evs]
        res = dict(ms_per_step=total_ms / steps, seg_ms=seg.mean(axis=0).tolist(), seg_names=names,
                   step_median_ms=float(np.median(per_step)), step_min_ms=float(np.min(per_step)),
                   E=[float(x) for x in Es], J=J.clone(), K=out["K"].clone(),
                   lam=out["lam"].clone(), g=out["g"].clone())
        # the exchange-type Fock kernel alone (inside nof_gen_fock above), same
        # inputs and launch configuration, timed with events on its stream
        ws_x = nof.workspace(nof.lib.nof_exchange_fock_ws(naux, norb, nof._TDT[dt], prec), dev)
        F2 = torch.empty_like(Z)
        nof.exchange_fock(b, cK, prec=prec, F2=F2, ws=ws_x)
        ex = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ex[0].record()
        for _ in range(steps):
            nof.exchange_fock(b, cK, prec=prec, F2=F2, ws=ws_x)
        ex[1].record()
        torch.cuda.synchronize()
        res["exchange_ms"] = ex[0].elapsed_time(ex[1]) / steps
        # the K pass alone (A4: one HBM pass over the unique half of b + the
        # fixed-order reduction of its chunk partials)
        Kk = torch.empty_like(Z)
        nof.jk_diag(b, D, want_J=False, want_K=True, K=Kk, ws=ws_j)
        ex[0].record()
        for _ in range(steps):
            nof.jk_diag(b, D, want_J=False, want_K=True, K=Kk, ws=ws_j)
        ex[1].record()
        torch.cuda.synchronize()
        res["k_pass_ms"] = ex[0].elapsed_time(ex[1]) / steps
        del T, b, ws_x
        if fused:
            del ws_t
        torch.cuda.empty_cache()
        return res

    print("# timing fp64", file=sys.stderr, flush=True)
    r64 = run(B64, "f64", args.steps, args.warmup)
    ms = r64["ms_per_step"]
    value = flops["total"] / (ms * 1e-3) / 1e12
    a1_ms = r64["seg_ms"][1]
    a2_ms = r64["seg_ms"][2]
    a6_ms = r64["exchange_ms"]
    # dominant kernel of the FP64 step: transform stage 1 or the exchange-type Fock term
    if a6_ms > a1_ms:
        dom = dict(key="k_exchange_fock", name="exchange-type Fock term F2 (sum_P b^P (cK o b^P)), FP64 MFMA",
                   ms=a6_ms, flops=flops["a6"], bytes=8.0 * (naux * norb * norb + norb * norb))
    else:
        dom = dict(key="k_transform_stage1", name="transform stage 1 (T^P = B^P C), FP64 MFMA",
                   ms=a1_ms, flops=flops["a1"], bytes=8.0 * (naux * nbf * nbf + naux * nbf * norb + nbf * norb))
    dom_tf = dom["flops"] / (dom["ms"] * 1e-3) / 1e12

    forms = {}
    B32 = None
    for f in [x for x in args.forms.split(",") if x]:
        print(f"# timing {f}", file=sys.stderr, flush=True)
        if f == "bf16B":
            Bf = B64.to(torch.bfloat16)
        elif f == "bf16x10":
            Bf = nof.SplitB(B64)          # fixed-point planes of the FP64 B, split once
        else:
            if B32 is None:
                B32 = B64.to(torch.float32)
            Bf = B32
        r = run(Bf, f, args.steps, args.warmup)
        del Bf
        torch.cuda.empty_cache()
        dE = max(abs(a - b_) for a, b_ in zip(r["E"], r64["E"]))
        forms[f] = dict(
            ms_per_step=r["ms_per_step"],
            tflops=flops["total"] / (r["ms_per_step"] * 1e-3) / 1e12,
            speedup_vs_f64=ms / r["ms_per_step"],
            max_abs_dE_Eh=dE,
            max_abs_dJ=float((r["J"] - r64["J"]).abs().max()),
            max_abs_dK=float((r["K"] - r64["K"]).abs().max()),
            max_abs_dlambda=float((r["lam"] - r64["lam"]).abs().max()),
            stage_ms=dict(zip(r["seg_names"], r["seg_ms"])),
            meets_dE_1e6=bool(dE <= 1e-6),
        )
        if "a1_a2_transform" in r["seg_names"]:
            # the fused x10 transform as BF16 matrix-core work: ten products of
            # pieces per algorithmic flop of either stage
            t = r["seg_ms"][r["seg_names"].index("a1_a2_transform")]
            tf = 10.0 * (flops["a1"] + flops["a2"]) / (t * 1e-3) / 1e12
            forms[f]["transform_matrix_core"] = dict(products_per_flop=10, tflops_bf16=tf,
                                                     peak=PEAK["bf16"], frac=tf / PEAK["bf16"])
    del B32
    torch.cuda.empty_cache()

    batched = run_batched(nof, inputs, dev) if args.batched else None
    warm = run_warmstart(nof, args.warmstart) if args.warmstart > 0 else None
    if args.copy_calib > 0:
        n_el = args.copy_calib // 4
        src = torch.ones(n_el, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if args.cpu_slabs > 0:
        cpu = cpu_baseline(B_h, C0, H_h, n_h, w, args.cpu_slabs)

    precision = None
    if args.precision_workload and args.precision_workload != args.workload:
        del B64
        torch.cuda.empty_cache()
        precision = run_precision_workload(args.precision_workload)

    line = {
        "metric": "JK+gen-Fock build ms/iter and TFLOP/s; BF16 vs FP64 on one GPU at |dE|<=1e-6 Eh",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: Nbf={nbf} Naux={naux} Norb={norb}, one orbital-optimisation "
                               f"iteration (rotation + transform + J/K + gen-Fock + energy), "
                               f"{w.nstrong} strong orbitals x {w.ng} weak partners",
                   "nbf": nbf, "naux": naux, "norb": norb, "seed": w.seed},
        "E_last": r64["E"][-1],
        "ms_per_step_median": r64["step_median_ms"],
        "ms_per_step_min": r64["step_min_ms"],
        "algorithmic_flops_per_step": flops["total"],
        "tflops_dense_equivalent": flops["dense"] / (ms * 1e-3) / 1e12,
        "k_pass": {"ms": r64["k_pass_ms"],
                   "bytes": 8.0 * naux * norb * (norb + 1) / 2,
                   "gbs": 8.0 * naux * norb * (norb + 1) / 2 / (r64["k_pass_ms"] * 1e-3) / 1e9,
                   "frac_of_8tbs": 8.0 * naux * norb * (norb + 1) / 2 / (r64["k_pass_ms"] * 1e-3) / 1e9
                   / HBM_PEAK_GBS},
        "stage_ms": dict(zip(r64["seg_names"], r64["seg_ms"])),
        "roofline": {"bound": "mfma", "kernel": dom["name"],
                     "achieved": dom_tf, "peak": PEAK["f64"], "unit": "TFLOP/s",
                     "frac": dom_tf / PEAK["f64"], "traffic": load_traffic(args.traffic_file, dom["key"]),
                     "flops_per_launch": dom["flops"], "avg_launch_ms": dom["ms"],
                     "algorithmic_bytes_per_launch": dom["bytes"],
                     "other": {"transform_stage1_ms": a1_ms, "exchange_fock_ms": a6_ms,
                               "transform_stage1_frac": flops["a1"] / (a1_ms * 1e-3) / 1e12 / PEAK["f64"],
                               "exchange_fock_frac": flops["a6"] / (a6_ms * 1e-3) / 1e12 / PEAK["f64"],
                               # both transform stages (A1 + A2, symmetric half of A2 counted)
                               "transform_ms": a1_ms + a2_ms,
                               "transform_frac": (flops["a1"] + flops["a2"]) / ((a1_ms + a2_ms) * 1e-3) / 1e12
                               / PEAK["f64"]}},
        "forms": forms,
        "batched": batched,
        "precision_workload": precision,
        "warmstart": warm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def run_precision_workload(name, steps=3, warmup=1):
    """FP64 against the x10 forms (B as fixed-point planes of the FP64 B, and
    FP32 B split in the loader) on another workload, in a child process of
    this script (its inputs do not fit beside this run's)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", name, "--forms", "bf16x10,bf16x10f32",
           "--batched", "0", "--cpu-slabs", "0", "--precision-workload", "", "--steps", str(steps),
           "--warmup", str(warmup), "--traffic-file", ""]
    print(f"# precision workload {name}: child run", file=sys.stderr, flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"workload": name, "error": f"child exited {r.returncode}", "stderr_tail": r.stderr[-400:]}
    d = json.loads(lines[-1])
    keep = ("ms_per_step", "speedup_vs_f64", "max_abs_dE_Eh", "max_abs_dJ", "max_abs_dK", "meets_dE_1e6")
    return {"workload": d["config"]["workload"], "fp64_ms_per_step": d["ms_per_step"],
            "E_fp64": d["E_last"], "steps": steps,
            "forms": {k: {q: v[q] for q in keep} for k, v in d["forms"].items()}}


def run_batched(nof, inputs, dev, steps=5):
    """25 finite-field instances sharing B (Nbf=300, Naux=1200, Norb=300), FP32
    products: one graph launch per iteration versus 25 single-instance
    iterations through the per-instance entry points."""
    import torch
    w = inputs.WORKLOADS["field300"]
    nbf, naux, norb = w.nbf, w.naux, w.norb
    B = inputs.make_B(w.seed, nbf, naux, w.decay, threads=16)
    fi = inputs.field_instances(w.seed, nbf, norb, w.nstrong, 25)
    members = np.array(inputs.pairing(norb, w.nstrong, w.ng), dtype=np.int32)
    d = lambda x, t=torch.float64: torch.from_numpy(np.ascontiguousarray(x)).to(dev, t)
    Bd = d(B, torch.float32)
    Cd, Hd, nd = d(fi["C"]), d(fi["H"]), d(fi["n"])
    occ = nof.Occupations(norb, torch.from_numpy(members).to(dev), nof.MAP_TRIG, nof.FUNC_PNOF5)
    cJd = torch.empty((25, norb, norb), dtype=torch.float64, device=dev)
    cKd = torch.empty_like(cJd)
    for i in range(25):
        cJd[i], cKd[i] = occ.coefficients(nd[i])
    plan = nof.BatchPlan(Bd, Cd, Hd, nd, cJd, cKd, prec=nof.P_F32)
    cfg = plan.autotune()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(s)
        plan.launch(s)
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record(s)
        for _ in range(steps):
            plan.launch(s)
        e1.record(s)
    s.synchronize()
    ms_batch = e0.elapsed_time(e1) / steps
    # the same work as 25 separate single-instance iterations
    T = torch.empty((naux, nbf, norb), dtype=torch.float32, device=dev)
    b = torch.empty((naux, norb, norb), dtype=torch.float32, device=dev)
    D = torch.empty((naux, norb), dtype=torch.float64, device=dev)
    def single_all():
        for i in range(25):
            nof.transform_stage1(Bd, Cd[i], T, prec=nof.P_F32)
            nof.transform_stage2(T, Cd[i], b, D, prec=nof.P_F32)
            h = nof.one_electron(Hd[i], Cd[i])
            J, _ = nof.jk_diag(b, D, want_K=False)
            lam, g, K = nof.gen_fock(b, D, nd[i], h, cJd[i], cKd[i], want_K=True, prec=nof.P_F32)
            nof.energy(nd[i], h, J, K, cJd[i], cKd[i])
    single_all()
    torch.cuda.synchronize()
    e0.record()
    single_all()
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1)
    f = algorithmic_flops(nbf, naux, norb)["total"] * 25
    E32 = plan.E.clone()
    C_start = Cd.clone()
    solve = run_batched_solve(nof, plan, Bd, Cd, Hd, members, w, dev, s)
    Cd.copy_(C_start)                     # the solve leaves its orbitals in C
    # the same batch in the fixed-point x10 form (B split once into planes from
    # FP64) and in FP64, both autotuned and replayed from a graph; energies
    # of the three against the FP64 batch
    del T, b, D
    torch.cuda.empty_cache()
    B64 = d(B)
    out = {}
    for name, Bp in (("x10", nof.SplitB(B64)), ("f64", B64)):
        pl = nof.BatchPlan(Bp, Cd, Hd, nd, cJd, cKd)
        pl.autotune()
        with torch.cuda.stream(s):
            pl.capture(s)
            pl.launch(s)
        s.synchronize()
        with torch.cuda.stream(s):
            e0.record(s)
            for _ in range(steps):
                pl.launch(s)
            e1.record(s)
        s.synchronize()
        out[name] = (e0.elapsed_time(e1) / steps, pl.E.clone())
        del pl, Bp
        torch.cuda.empty_cache()
    ms_x10, Ex10 = out["x10"]
    ms_64, E64 = out["f64"]
    return {"workload": "field300: 25 finite-field instances, Nbf=300 Naux=1200 Norb=300, FP32 products",
            "ms_per_iteration_batched_graph": ms_batch, "ms_per_iteration_25_single": ms_single,
            "speedup": ms_single / ms_batch, "tflops_batched": f / (ms_batch * 1e-3) / 1e12,
            "tuned_config": {"tile_stage1": cfg[0], "tile_stage2": cfg[1], "tile_exchange": cfg[2],
                             "exchange_p_split": cfg[3]},
            "max_abs_dE_Eh_vs_f64": float((E32 - E64).abs().max()),
            "x10": {"ms_per_iteration_batched_graph": ms_x10, "tflops": f / (ms_x10 * 1e-3) / 1e12,
                    "speedup_vs_fp32_batch": ms_batch / ms_x10, "speedup_vs_f64_batch": ms_64 / ms_x10,
                    "max_abs_dE_Eh_vs_f64": float((Ex10 - E64).abs().max())},
            "f64": {"ms_per_iteration_batched_graph": ms_64},
            "solve": solve}


def run_batched_solve(nof, plan, Bd, Cd, Hd, members, w, dev, stream, outer=2, steps=10):
    """The NO + ON loop for all 25 instances (nof_plan_solve: per-instance ON
    steps, one graph replay per NO step of all instances) against 25
    single-instance solves (nof_solve), both for `outer` outer iterations of
    `steps` NO steps (PNOF5, trigonometric map, cold start n_g = 0.98)."""
    import torch
    ns, ng, norb = w.nstrong, w.ng, w.norb
    g0 = np.zeros((ns, ng))
    g0[:, 0] = np.arccos(np.sqrt(2 * 0.98 - 1))
    for i in range(1, ng):
        g0[:, i] = np.arcsin(np.sqrt(1.0 / (ng - i + 1)))
    mem = torch.from_numpy(members).to(dev)
    kw = dict(max_outer=outer, no_steps=steps, tol_lambda=0.0, tol_energy=0.0, on_maxit=500)
    C0 = Cd.clone()
    gam = torch.from_numpy(np.stack([g0] * 25)).to(dev)
    plan.inputs[1].copy_(C0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.solve(mem, nof.MAP_TRIG, nof.FUNC_PNOF5, gam, stream=stream, **kw)
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    for i in range(25):
        C = C0[i].clone()
        g = torch.from_numpy(g0.copy()).to(dev)
        nof.solve(Bd, C, Hd[i], mem, nof.MAP_TRIG, nof.FUNC_PNOF5, g, prec=nof.P_F32, **kw)
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3
    return {"outer": outer, "no_steps_per_outer": steps, "on_maxit": kw["on_maxit"],
            "ms_batched": ms_b, "ms_25_single": ms_s, "speedup": ms_s / ms_b,
            "statuses_ok": all(r["status"] == 0 for r in res),
            "on_iters_per_instance_mean": float(np.mean([r["on_iters"] for r in res]))}


def run_warmstart(nof, ntrain, nheld=20):
    """Warm start: train on converged ONs of ntrain instances (Nbf = Norb in
    {100, 200}, Naux = 4 Nbf, 15-50 strong orbitals), evaluate on held-out
    Nbf = 500 instances with 125 strong orbitals."""
    from paper_2512_13550_amd import warmstart
    t0 = time.time()
    fac = warmstart.InstanceFactory(nof, gap=0.5)
    rng = np.random.default_rng(4000)
    log = lambda m: print(f"# warmstart {m}", file=sys.stderr, flush=True)
    X, T, it_train = warmstart.build_dataset(nof, fac, range(4000, 4000 + ntrain), (100, 200), (15, 50), rng,
                                             log=log)
    t_data = time.time() - t0
    params, hist = warmstart.train(nof, X, T, epochs=40, batch=4096, lr=2e-3, seed=1, log=log)
    t_train = time.time() - t0 - t_data
    rows = warmstart.evaluate(nof, fac, params, range(9000, 9000 + nheld), 500, 125)
    cold = np.array([r["iters_cold"] for r in rows]); warm = np.array([r["iters_warm"] for r in rows])
    return {"train_instances": ntrain, "train_rows": int(X.shape[0]), "loss_first_last": [hist[0], hist[-1]],
            "data_s": t_data, "train_s": t_train, "held_out": nheld,
            "iters_cold_mean": float(cold.mean()), "iters_warm_mean": float(warm.mean()),
            "iters_saved_mean": float(cold.mean() - warm.mean()),
            "iters_restart_mean": float(np.mean([r["iters_restart"] for r in rows])),
            "max_abs_dE_Eh": float(max(abs(r["E_warm"] - r["E_cold"]) for r in rows)),
            "all_converged": bool(all(r["converged"] for r in rows))}


def cpu_baseline(B_h, C0, H_h, n_h, w, slabs):
    """The FP64 oracle, as it stands, on the first `slabs` auxiliary slabs."""
    from oracle import dfjk
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    slabs = min(slabs, w.naux)
    Bs = B_h[:slabs]
    nn = np.outer(n_h, n_h)
    cJ, cK = 2.0 * nn, nn
    print(f"# cpu oracle sample: {slabs} slabs", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    dfjk.iteration(Bs, C0, H_h, n_h, cJ, cK)
    dt = time.perf_counter() - t0
    f = algorithmic_flops(w.nbf, slabs, w.norb)["total"]
    one = None
    try:                                   # the same sample on one host core
        from threadpoolctl import threadpool_limits
        s1 = max(1, slabs // 8)
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            dfjk.iteration(B_h[:s1], C0, H_h, n_h, cJ, cK)
            d1 = time.perf_counter() - t1
        one = {"value": algorithmic_flops(w.nbf, s1, w.norb)["total"] / d1 / 1e12, "unit": "TFLOP/s",
               "sample": f"{s1} slabs, {d1:.2f} s"}
    except Exception:  # pragma: no cover
        pass
    return {"value": f / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{slabs} of {w.naux} auxiliary slabs of {w.name}, one iteration, "
                      f"{dt:.2f} s; full-iteration estimate {dt * w.naux / slabs:.1f} s",
            "one_core": one}


if __name__ == "__main__":
    main()
