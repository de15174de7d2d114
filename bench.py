#!/usr/bin/env python
"""Benchmark of one orbital-optimisation iteration of the density-fitted JK +
generalized-Fock build on one MI355X.

Workload (default "chain1000"): Nbf=1000, Naux=4000, Norb=1000, synthetic
hydrogen-chain-shaped inputs (see paper_2512_13550_amd/inputs.py), 500
strongly occupied orbitals each paired with one weak orbital.

One step = one iteration: C <- C exp(eps Y_i) (FP64 rotation on the GPU),
b = C^T B C and D, h = C^T H C, J, the Coulomb-type Fock term with K (one pass
over the upper half of b), the exchange-type Fock term, lambda and g, then E.
Every step is bracketed by HIP events per call (on the stream of the
launches), so each large kernel is timed inside the timed region.  All inputs
are resident in HBM before the timed region starts.

Prints ONE JSON line.  `value` is the algorithmic TFLOP/s of the FP64 path;
`forms` holds the reduced-precision forms on the same workload with their
errors against the FP64 GPU result; `roofline` describes the dominant kernel;
`cpu_baseline` is the FP64 CPU oracle timed on a bounded slab sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "i8": 5000.0}   # dense MFMA TFLOP/s / TOP/s (MI355X datasheet)
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))


def algorithmic_flops(nbf, naux, norb):
    a1 = 2.0 * naux * nbf * nbf * norb                 # T^P = B^P C
    a2 = 1.0 * naux * nbf * norb * (norb + 1)          # b^P = C^T T^P, symmetric half
    a6 = 1.0 * naux * norb * norb * (norb + 1)         # exchange-type Fock term: the per-q
                                                       # products G^q are symmetric (half)
    small = 6.0 * naux * norb * norb                   # J, K, W, F1
    dense = a1 + 2.0 * naux * nbf * norb * norb + 2.0 * naux * norb ** 3   # the three products as dense GEMMs
    return dict(a1=a1, a2=a2, a6=a6, small=small, total=a1 + a2 + a6 + small, dense=dense)


def k_bytes(naux, norb, esz):
    """Algorithmic bytes of the K pass: the upper half of b."""
    return esz * naux * norb * (norb + 1) / 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="chain1000")
    ap.add_argument("--forms", default="i8x10,bf16x10,bf16x10f32,f32,bf16B",
                    help="comma list of extra forms: f32, bf16x1, bf16x3, bf16x6, bf16x10 (B split "
                         "once into fixed-point planes from FP64), bf16x10f32 (FP32 B split in the "
                         "loader), i8x10 (B split once into INT8 fixed-point planes from FP64), "
                         "bf16B (B stored in BF16; also compared with FP64 on the BF16-rounded B)")
    ap.add_argument("--cpu-slabs", type=int, default=800,
                    help="auxiliary slabs in the CPU-oracle sample (0 = skip)")
    ap.add_argument("--batched", type=int, default=1,
                    help="1: also time the 25-instance finite-field batch (graph launch) and its "
                         "solve; 2: time only that batch and print its record (for kernel profiles)")
    ap.add_argument("--secondary", default="c500",
                    help="also time FP64 against FP32 on this workload in a child run ('' = skip)")
    ap.add_argument("--warmstart", type=int, default=4000,
                    help="train the warm-start network on this many instances and evaluate it (0 = skip)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="bytes of a plain read+write kernel run 3 times after timing "
                         "(counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "traffic_fp64_chain1000.json"))
    return ap.parse_args()


# the sources that decide each timed kernel's code and launch configuration
KERNEL_SOURCES = {"k_exchange_fock": ("gemm_tn.hip", "api.hip", "common.h"),
                  "k_transform_stage1": ("gemm_tn.hip", "api.hip", "common.h"),
                  "k_transform_stage2": ("gemm_tn.hip", "api.hip", "common.h"),
                  "k_kf1": ("passes.hip", "api.hip", "common.h")}


def kernel_source_digest(kernel):
    """Digest of a kernel's sources (its counter traffic is stale once they change)."""
    import hashlib
    root = os.path.join(ROOT, "paper_2512_13550_amd", "csrc")
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES[kernel]:
        with open(os.path.join(root, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(path, kernel):
    """HBM-side bytes per launch of a kernel from a committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel's readings), or None when
    absent or taken on other sources of that kernel."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k or k.get("source_digest") != kernel_source_digest(kernel):
        return None
    return k.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2512_13550_amd.nof as nof
    from paper_2512_13550_amd import inputs

    dev = torch.device("cuda:0")
    if args.batched == 2:
        rec = run_batched(nof, inputs, dev, steps=args.steps, solve=False)
        print(json.dumps({"batched": rec}))
        return
    w = inputs.WORKLOADS[args.workload]
    nbf, naux, norb = w.nbf, w.naux, w.norb
    t0 = time.time()
    log(f"generating {w.name}: nbf={nbf} naux={naux} norb={norb}")
    B_h = inputs.make_B(w.seed, nbf, naux, w.decay, threads=16)
    C0 = inputs.make_C(w.seed, nbf, norb)
    H_h = inputs.make_H(w.seed, nbf)
    n_h = inputs.make_occupations(w.seed, norb, w.nstrong)
    total_iters = max(args.warmup + args.steps, w.iters)
    Ys = [inputs.make_antisym(w.seed, it, norb) for it in range(total_iters)]
    log(f"inputs ready in {time.time() - t0:.1f}s")

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
             "bf16B": nof.P_BF16X6, "i8x10": nof.P_I8X10}

    def run(B, prec_name, steps, warmup):
        dt = torch.float64 if prec_name == "f64" else torch.float32
        prec = PRECS[prec_name]
        C = torch.from_numpy(C0).to(dev)
        Cn = torch.empty_like(C)
        # x10: both stages in one nof_mo_transform call (the first stage's
        # epilogue gives the second its column grids); the others call the
        # stages separately, so that each is timed on its own
        fused = prec in (nof.P_BF16X10, nof.P_I8X10)
        # the x1 / x3 split forms fold the Coulomb-type term into the
        # exchange-type product (the pass over b forms K alone); the FP64 and
        # FP32 (symmetric per-q products), x6, x10 and INT8 exchange-type
        # terms do not take it, so there the pass forms K and the Coulomb-type
        # term together
        folded = prec not in (nof.P_F64, nof.P_F32, nof.P_BF16X6, nof.P_BF16X10, nof.P_I8X10)
        names = (["rotate"] + (["a1_a2_transform"] if fused else ["a1_transform_stage1", "a2_transform_stage2"])
                 + ["h_and_J"]
                 + (["a4_k_pass", "a5_a6_fock_terms"] if folded else ["a4_a5_coulomb_pass", "a6_exchange"])
                 + ["a7_lambda_grad", "a8_energy"])
        if fused:
            T = None
            ws_t = nof.workspace(nof.lib.nof_mo_transform_ws(naux, nbf, norb, nof._b_arg(B)[0], nof._TDT[dt], prec),
                                 dev)
        else:
            T = torch.empty((naux, nbf, norb), dtype=dt, device=dev)
        b = torch.empty((naux, norb, norb), dtype=dt, device=dev)
        D = torch.empty((naux, norb), dtype=torch.float64, device=dev)
        lam, g, K, J, F, F1 = (torch.empty_like(Z) for _ in range(6))
        E = torch.empty((), dtype=torch.float64, device=dev)
        rot = nof.Rotation(norb, nbf, dev)
        if folded:
            ws_f = nof.workspace(nof.lib.nof_fock_terms_ws(naux, norb, nof._TDT[dt], prec), dev)
        else:
            ws_c = nof.workspace(nof.lib.nof_coulomb_fock_ws(naux, norb, nof._TDT[dt]), dev)
            ws_x = nof.workspace(nof.lib.nof_exchange_fock_ws(naux, norb, nof._TDT[dt], prec), dev)
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
            if folded:
                nof.jk_diag(b, D, want_J=False, want_K=True, K=K, ws=ws_j)   # A4
                tick()
                nof.fock_terms(b, D, cJ, cK, prec=prec, F=F, ws=ws_f)    # A5 + A6: F2 - F1
                tick()
                nof.lambda_grad(n, h, None, F, lam=lam, g=g)             # A7
            else:
                nof.coulomb_fock(b, D, cJ, F1=F1, K=K, ws=ws_c)          # A4 + A5
                tick()
                nof.exchange_fock(b, cK, prec=prec, F2=F, ws=ws_x)       # A6
                tick()
                nof.lambda_grad(n, h, F1, F, lam=lam, g=g)               # A7
            tick()
            nof.energy(n, h, J, K, cJ, cK, E=E, ws=ws_e)             # A8
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
                   E=[float(x) for x in Es], J=J.clone(), K=K.clone(), lam=lam.clone(), g=g.clone())
        del T, b
        if fused:
            del ws_t
        torch.cuda.empty_cache()
        return res

    log("timing fp64")
    r64 = run(B64, "f64", args.steps, args.warmup)
    seg64 = dict(zip(r64["seg_names"], r64["seg_ms"]))
    ms = r64["ms_per_step"]
    value = flops["total"] / (ms * 1e-3) / 1e12
    a1_ms, a2_ms, a6_ms = seg64["a1_transform_stage1"], seg64["a2_transform_stage2"], seg64["a6_exchange"]
    kf_ms = seg64["a4_a5_coulomb_pass"]
    # dominant kernel of the FP64 step: transform stage 1 or the exchange-type term
    if a6_ms > a1_ms:
        dom = dict(key="k_exchange_fock", name="exchange-type term through the symmetric per-q products "
                   "G^q = sum_P b^P[q]^T b^P[q] (FP64 MFMA) and their cK-weighted sum over q; the "
                   "segment includes the sum",
                   ms=a6_ms, flops=flops["a6"],
                   bytes=8.0 * (naux * norb * norb + norb * norb))
    else:
        dom = dict(key="k_transform_stage1", name="transform stage 1 (T^P = B^P C), FP64 MFMA",
                   ms=a1_ms, flops=flops["a1"], bytes=8.0 * (naux * nbf * nbf + naux * nbf * norb + nbf * norb))
    dom_tf = dom["flops"] / (dom["ms"] * 1e-3) / 1e12

    forms = {}
    B32 = None
    for f in [x for x in args.forms.split(",") if x]:
        log(f"timing {f}")
        if f == "bf16B":
            Bf = B64.to(torch.bfloat16)
        elif f == "bf16x10":
            Bf = nof.SplitB(B64)          # fixed-point planes of the FP64 B, split once
        elif f == "i8x10":
            Bf = nof.SplitBI8(B64)        # INT8 fixed-point planes of the FP64 B, split once
        else:
            if B32 is None:
                B32 = B64.to(torch.float32)
            Bf = B32
        r = run(Bf, f, args.steps, args.warmup)
        ref = dict(E=r64["E"], J=r64["J"], K=r64["K"], lam=r64["lam"])
        forms[f] = form_record(r, ref, flops, ms)
        if f == "bf16B":
            # the BF16 rounding of B is an input error: the same form against
            # FP64 on the BF16-rounded B isolates the arithmetic error
            del Bf
            torch.cuda.empty_cache()
            B64r = B64.to(torch.bfloat16).to(torch.float64)
            log("timing fp64 on the BF16-rounded B")
            rr = run(B64r, "f64", args.steps, args.warmup)
            del B64r
            forms[f]["vs_fp64_on_bf16_rounded_B"] = errors(r, rr)
            Bf = None
        if "a1_a2_transform" in r["seg_names"]:
            # the fused fixed-point transform as matrix-core work: ten products
            # of pieces per algorithmic operation of either stage (BF16 or INT8)
            t = r["seg_ms"][r["seg_names"].index("a1_a2_transform")]
            unit = "i8" if f == "i8x10" else "bf16"
            tf = 10.0 * (flops["a1"] + flops["a2"]) / (t * 1e-3) / 1e12
            forms[f]["transform_matrix_core"] = dict(products_per_flop=10, unit=unit, tops=tf,
                                                     peak=PEAK[unit], frac=tf / PEAK[unit])
        del Bf
        torch.cuda.empty_cache()
    del B32
    torch.cuda.empty_cache()

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
    del B64, B_h
    torch.cuda.empty_cache()

    secondary = None
    if args.secondary and args.secondary != args.workload:
        secondary = run_secondary(args.secondary)
    batched = run_batched(nof, inputs, dev) if args.batched else None
    warm = run_warmstart(nof, args.warmstart) if args.warmstart > 0 else None

    kfb = k_bytes(naux, norb, 8.0) + 8.0 * naux * norb   # the upper half of b and W
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
        "stage_ms": seg64,
        "k_pass": {"what": "K and the Coulomb-type term F1 in one pass over the upper half of b, the "
                           "W = D cJ product and the fixed-order reductions of the partials (the "
                           "a4_a5_coulomb_pass segment of the step)",
                   "ms": kf_ms, "bytes": kfb, "gbs": kfb / (kf_ms * 1e-3) / 1e9,
                   "frac_of_8tbs": kfb / (kf_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "roofline": {"bound": "mfma", "kernel": dom["name"],
                     "achieved": dom_tf, "peak": PEAK["f64"], "unit": "TFLOP/s",
                     "frac": dom_tf / PEAK["f64"], "traffic": load_traffic(args.traffic_file, dom["key"]),
                     "flops_per_launch": dom["flops"], "avg_launch_ms": dom["ms"],
                     "algorithmic_bytes_per_launch": dom["bytes"],
                     "other": {"transform_stage1_ms": a1_ms, "transform_stage2_ms": a2_ms,
                               "exchange_fock_ms": a6_ms,
                               "transform_stage1_frac": flops["a1"] / (a1_ms * 1e-3) / 1e12 / PEAK["f64"],
                               "transform_stage2_frac": flops["a2"] / (a2_ms * 1e-3) / 1e12 / PEAK["f64"],
                               "exchange_fock_frac": flops["a6"] / (a6_ms * 1e-3) / 1e12 / PEAK["f64"],
                               "transform_frac": (flops["a1"] + flops["a2"]) / ((a1_ms + a2_ms) * 1e-3) / 1e12
                               / PEAK["f64"]}},
        "forms": forms,
        "secondary": secondary,
        "batched": batched,
        "warmstart": warm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def errors(r, ref):
    dE = max(abs(a - b_) for a, b_ in zip(r["E"], ref["E"]))
    return dict(max_abs_dE_Eh=dE,
                max_abs_dJ=float((r["J"] - ref["J"]).abs().max()),
                max_abs_dK=float((r["K"] - ref["K"]).abs().max()),
                max_abs_dlambda=float((r["lam"] - ref["lam"]).abs().max()),
                meets_dE_1e6=bool(dE <= 1e-6))


def form_record(r, ref, flops, ms64):
    rec = dict(ms_per_step=r["ms_per_step"],
               tflops=flops["total"] / (r["ms_per_step"] * 1e-3) / 1e12,
               speedup_vs_f64=ms64 / r["ms_per_step"])
    rec.update(errors(r, ref))
    rec["stage_ms"] = dict(zip(r["seg_names"], r["seg_ms"]))
    return rec


def run_secondary(name, steps=10, warmup=3):
    """FP64 against FP32 on another workload (ten iterations, each after a
    small random rotation), in a child process of this script."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", name, "--forms", "f32",
           "--batched", "0", "--cpu-slabs", "0", "--secondary", "", "--warmstart", "0",
           "--steps", str(steps), "--warmup", str(warmup), "--traffic-file", ""]
    log(f"secondary workload {name}: child run")
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"workload": name, "error": f"child exited {r.returncode}", "stderr_tail": r.stderr[-400:]}
    d = json.loads(lines[-1])
    keep = ("ms_per_step", "speedup_vs_f64", "max_abs_dE_Eh", "max_abs_dJ", "max_abs_dK", "max_abs_dlambda",
            "meets_dE_1e6")
    return {"workload": d["config"]["workload"], "fp64_ms_per_step": d["ms_per_step"],
            "fp64_tflops": d["value"], "E_fp64": d["E_last"], "steps": steps, "stage_ms": d["stage_ms"],
            "roofline_other": d["roofline"]["other"], "k_pass": d["k_pass"],
            "forms": {k: {q: v[q] for q in keep} for k, v in d["forms"].items()}}


def run_batched(nof, inputs, dev, steps=5, solve=True):
    """25 finite-field instances sharing B (Nbf=300, Naux=1200, Norb=300): one
    graph launch per iteration as the fixed-point x10 plan (B split once into
    planes of the FP64 B), the FP32 plan and the FP64 plan, each autotuned;
    energies against the FP64 plan; the x10 plan against 25 single-instance
    x10 iterations; then the batched NO + ON solve."""
    import torch
    w = inputs.WORKLOADS["field300"]
    nbf, naux, norb = w.nbf, w.naux, w.norb
    B = inputs.make_B(w.seed, nbf, naux, w.decay, threads=16)
    fi = inputs.field_instances(w.seed, nbf, norb, w.nstrong, 25)
    members = np.array(inputs.pairing(norb, w.nstrong, w.ng), dtype=np.int32)
    d = lambda x, t=torch.float64: torch.from_numpy(np.ascontiguousarray(x)).to(dev, t)
    B64 = d(B)
    Cd, Hd, nd = d(fi["C"]), d(fi["H"]), d(fi["n"])
    occ = nof.Occupations(norb, torch.from_numpy(members).to(dev), nof.MAP_TRIG, nof.FUNC_PNOF5)
    cJd = torch.empty((25, norb, norb), dtype=torch.float64, device=dev)
    cKd = torch.empty_like(cJd)
    for i in range(25):
        cJd[i], cKd[i] = occ.coefficients(nd[i])
    s = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_plan(pl):
        cfg = pl.autotune()
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
        return e0.elapsed_time(e1) / steps, pl.E.clone(), cfg

    out = {}
    Bx = nof.SplitB(B64)
    Bi = nof.SplitBI8(B64)
    for name, Bp, prec in (("x10", Bx, None), ("i8x10", Bi, None), ("f32", None, nof.P_F32),
                           ("f64", B64, None)):
        if name == "f32":
            Bp = B64.to(torch.float32)
        pl = nof.BatchPlan(Bp, Cd, Hd, nd, cJd, cKd, prec=prec) if prec is not None else \
            nof.BatchPlan(Bp, Cd, Hd, nd, cJd, cKd)
        out[name] = time_plan(pl)
        del pl
        if name == "f32":
            del Bp
        torch.cuda.empty_cache()
    ms_x10, Ex10, cfg = out["x10"]
    ms_i8, Ei8, cfg_i8 = out["i8x10"]
    del Bi
    torch.cuda.empty_cache()
    ms_32, E32, _ = out["f32"]
    ms_64, E64, _ = out["f64"]
    # the same work as 25 separate single-instance x10 iterations
    b = torch.empty((naux, norb, norb), dtype=torch.float32, device=dev)
    D = torch.empty((naux, norb), dtype=torch.float64, device=dev)
    ws_t = nof.workspace(nof.lib.nof_mo_transform_ws(naux, nbf, norb, nof.BF16X4, nof.F32, nof.P_BF16X10), dev)

    def single_all():
        for i in range(25):
            nof.mo_transform(Bx, Cd[i], prec=nof.P_BF16X10, b=b, D=D, ws=ws_t)
            h = nof.one_electron(Hd[i], Cd[i])
            J, _ = nof.jk_diag(b, D, want_K=False)
            lam, g, K = nof.gen_fock(b, D, nd[i], h, cJd[i], cKd[i], want_K=True, prec=nof.P_BF16X10)
            nof.energy(nd[i], h, J, K, cJd[i], cKd[i])
    single_all()
    torch.cuda.synchronize()
    e0.record()
    single_all()
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1)
    del b, D, ws_t
    torch.cuda.empty_cache()
    f = algorithmic_flops(nbf, naux, norb)["total"] * 25
    rec = {"workload": "field300: 25 finite-field instances, Nbf=300 Naux=1200 Norb=300",
           "form": "x10 plan (B as fixed-point planes of the FP64 B)",
           "ms_per_iteration_batched_graph": ms_x10, "ms_per_iteration_25_single": ms_single,
           "speedup": ms_single / ms_x10, "tflops_batched": f / (ms_x10 * 1e-3) / 1e12,
           "tuned_config": {"tile_stage1": cfg[0], "tile_stage2": cfg[1], "tile_exchange": cfg[2],
                            "exchange_p_split": cfg[3]},
           "max_abs_dE_Eh_vs_f64": float((Ex10 - E64).abs().max()),
           "i8x10": {"ms_per_iteration_batched_graph": ms_i8, "tflops": f / (ms_i8 * 1e-3) / 1e12,
                     "tuned_config": {"tile_exchange": cfg_i8[2], "exchange_p_split": cfg_i8[3]},
                     "max_abs_dE_Eh_vs_f64": float((Ei8 - E64).abs().max())},
           "f32": {"ms_per_iteration_batched_graph": ms_32, "tflops": f / (ms_32 * 1e-3) / 1e12,
                   "max_abs_dE_Eh_vs_f64": float((E32 - E64).abs().max())},
           "f64": {"ms_per_iteration_batched_graph": ms_64, "tflops": f / (ms_64 * 1e-3) / 1e12}}
    if solve:
        rec["solve"] = run_batched_solve(nof, Bx, B64, Cd, Hd, w, dev, s)
    return rec


def solve_pair(nof, Bin, prec, C0, Hd, mem, g0, norb, dev, stream, kw):
    """One batched solve of the 25 instances (plan on Bin) and the 25
    single-instance solves in the plan's precision; returns both results and
    their wall times."""
    import torch
    Cs = C0.unsqueeze(0).repeat(25, 1, 1).contiguous()
    nd = torch.zeros((25, norb), dtype=torch.float64, device=dev)
    Z = torch.zeros((25, norb, norb), dtype=torch.float64, device=dev)
    plan = nof.BatchPlan(Bin, Cs, Hd, nd, Z, Z.clone())
    plan.autotune()
    gam = torch.from_numpy(np.stack([g0] * 25)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.solve(mem, nof.MAP_SOFTMAX, nof.FUNC_PNOF5, gam, stream=stream, **kw)
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    single = []
    for i in range(25):
        C = C0.clone()
        g = torch.from_numpy(g0.copy()).to(dev)
        single.append(nof.solve(Bin, C, Hd[i], mem, nof.MAP_SOFTMAX, nof.FUNC_PNOF5, g, prec=prec, **kw))
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3
    del plan
    torch.cuda.empty_cache()
    return res, single, ms_b, ms_s


def run_batched_solve(nof, Bx, B64, Cd, Hd, w, dev, stream, outer=2, steps=10, on_maxit=2000):
    """The NO + ON loop for all 25 finite-field instances as an x10 plan
    (nof_plan_solve: per-instance ON steps, one graph replay per NO step of
    all instances) against 25 single-instance solves (nof_solve), both for
    `outer` outer iterations of `steps` NO steps.  As in a finite-field
    calculation every instance starts from the same orbitals (the first
    instance's); the orbital roles follow the one-electron energies of the
    field-free H at those orbitals (aufbau); PNOF5, softmax map, cold start
    n_g = 0.98.  The same pair again with an FP64 plan and FP64 single
    solves (fp64_pair)."""
    import torch
    from paper_2512_13550_amd.warmstart import aufbau_members
    ns, ng, norb = w.nstrong, w.ng, w.norb
    C0 = Cd[0].clone()
    h0 = nof.one_electron(Hd[0], C0)
    members = aufbau_members(torch.diagonal(h0).cpu().numpy(), ns, ng)
    mem = torch.from_numpy(members).to(dev)
    g0 = np.full((ns, ng), np.log(0.02 / ng / 0.98))
    kw = dict(max_outer=outer, no_steps=steps, tol_lambda=0.0, tol_energy=0.0, on_maxit=on_maxit)
    res, single, ms_b, ms_s = solve_pair(nof, Bx, nof.P_BF16X10, C0, Hd, mem, g0, norb, dev, stream, kw)
    # the same pair as an FP64 plan and FP64 single solves, whose roundings
    # differ only in the order of some FP64 sums: how far the pairs drift
    # apart measures how much the trajectory amplifies rounding (ADAM's first
    # steps move every component by about lr sign(g), also where g is ~0)
    r64, s64, ms_b64, ms_s64 = solve_pair(nof, B64, nof.P_F64, C0, Hd, mem, g0, norb, dev, stream, kw)
    dE64 = [abs(a["E"] - b_["E"]) for a, b_ in zip(r64, s64)]
    # the two runs take the same steps in exact arithmetic; their roundings
    # differ (packed first stage, one launch for all ON steps), and the ON line
    # searches can turn such differences into different discrete choices
    dEs = [abs(a["E"] - b_["E"]) for a, b_ in zip(res, single)]
    return {"outer": outer, "no_steps_per_outer": steps, "on_maxit": on_maxit, "map": "softmax",
            "roles": "aufbau at the shared start orbitals", "form": "x10",
            "ms_batched": ms_b, "ms_25_single": ms_s, "speedup": ms_s / ms_b,
            "statuses_ok": all(r["status"] == 0 and r["on_unconverged"] == 0 for r in res),
            "on_unconverged_calls": int(sum(r["on_unconverged"] for r in res)),
            "on_iters_per_call_mean": float(np.mean([r["on_iters"] for r in res])) / outer,
            "on_iters_per_call_max_instance": float(max(r["on_iters"] for r in res)) / outer,
            "max_abs_dE_Eh_batched_vs_single": float(max(dEs)),
            "median_abs_dE_Eh_batched_vs_single": float(np.median(dEs)),
            "instances_dE_above_1e-6": int(sum(x > 1e-6 for x in dEs)),
            "fp64_pair": {"ms_batched": ms_b64, "ms_25_single": ms_s64, "speedup": ms_s64 / ms_b64,
                          "max_abs_dE_Eh_batched_vs_single": float(max(dE64))}}


def run_warmstart(nof, ntrain, nheld=20):
    """Warm start: train on converged ONs of ntrain instances (Nbf = Norb in
    {100, 200}, Naux = 4 Nbf, 15-50 strong orbitals), evaluate on held-out
    Nbf = 500 instances with 125 strong orbitals, for the softmax and the
    trigonometric map."""
    from paper_2512_13550_amd import warmstart
    t0 = time.time()
    fac = warmstart.InstanceFactory(nof, gap=0.5)
    rng = np.random.default_rng(4000)
    lg = lambda m: log(f"warmstart {m}")
    X, T, it_train = warmstart.build_dataset(nof, fac, range(4000, 4000 + ntrain), (100, 200), (15, 50), rng,
                                             log=lg)
    t_data = time.time() - t0
    params, hist = warmstart.train(nof, X, T, epochs=40, batch=4096, lr=2e-3, seed=1, log=lg)
    t_train = time.time() - t0 - t_data
    out = {"train_instances": ntrain, "train_rows": int(X.shape[0]), "loss_first_last": [hist[0], hist[-1]],
           "data_s": t_data, "train_s": t_train, "held_out": nheld, "held_out_nbf": 500}
    for mapping, name in ((1, "softmax"), (0, "trig")):
        rows = warmstart.evaluate(nof, fac, params, range(9000, 9000 + nheld), 500, 125, mapping=mapping)
        cold = np.array([r["iters_cold"] for r in rows])
        warm = np.array([r["iters_warm"] for r in rows])
        out[name] = {"iters_cold_mean": float(cold.mean()), "iters_warm_mean": float(warm.mean()),
                     "iters_saved_mean": float(cold.mean() - warm.mean()),
                     "iters_restart_mean": float(np.mean([r["iters_restart"] for r in rows])),
                     "max_abs_dE_Eh": float(max(abs(r["E_warm"] - r["E_cold"]) for r in rows)),
                     "all_converged": bool(all(r["converged"] for r in rows))}
    return out


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
    log(f"cpu oracle sample: {slabs} slabs")
    t0 = time.perf_counter()
    dfjk.iteration(Bs, C0, H_h, n_h, cJ, cK)
    dt = time.perf_counter() - t0
    f = algorithmic_flops(w.nbf, slabs, w.norb)["total"]
    one = None
    try:                                   # a smaller sample on one host core
        from threadpoolctl import threadpool_limits
        s1 = max(1, slabs // 16)
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            dfjk.iteration(B_h[:s1], C0, H_h, n_h, cJ, cK)
            d1 = time.perf_counter() - t1
        one = {"value": algorithmic_flops(w.nbf, s1, w.norb)["total"] / d1 / 1e12, "unit": "TFLOP/s",
               "sample": f"{s1} slabs, {d1:.2f} s"}
    except Exception:  # pragma: no cover
        pass
    return {"value": f / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{slabs} of {w.naux} auxiliary slabs of {w.name} (the whole iteration restricted to "
                      f"those slabs: transform, J, K, both Fock terms, lambda, E), {dt:.2f} s; "
                      f"full-iteration estimate {dt * w.naux / slabs:.1f} s",
            "one_core": one}


if __name__ == "__main__":
    main()
