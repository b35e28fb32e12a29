#!/usr/bin/env python
"""Benchmark of the Nystrom-Schur hot path on one MI355X.

One step = the whole path on one synthetic system already resident in HBM:
DBBD extraction, batched Cholesky of the interior and interface blocks, the
block CG on the shifted Schur system (k+p sketch columns, eps_SI = 0.1), the
Nystrom core, and the PCG solve of A x = b to relative residual 1e-8 with the
block LDL^T back-substitution.

Workload (default): 3D 7-point lognormal diffusion (sigma 2, correlation 8
cells) on a 64^3 grid, 4x4x4 box subdomains, k = 64, p = 16; inner block CG
in FP32 (FP32 factors and block vectors, MFMA), everything else FP64.  A plain
FP64 step is timed beside it for the "vs plain FP64" part of the metric.

Prints ONE JSON line.  `value` = seconds per step (setup + solve); lower is
better.  `roofline` is computed live from HIP events bracketing every launch
of the dominant kernel family inside the timed region; `cpu_baseline` times
the FP64 oracle on the host on a bounded sample of the same workload.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "setup+solve sec & PCG iters to rel.res 1e-8; Schur-BCG HBM GB/s vs plain FP64"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=64, help="grid side (64 = the benchmark workload)")
    ap.add_argument("--boxes", type=int, default=4)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32", help="inner block-CG precision")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trsm-cols", type=int, default=0)
    ap.add_argument("--workload", choices=["c2", "c3"], default="c2",
                    help="c2: the 64^3 lognormal system (default line); c3: the batched anisotropic set")
    ap.add_argument("--nprob", type=int, default=256, help="problems of the batched workload")
    return ap.parse_args()


def roofline(stats, steps):
    """Roofline of the dominant kernel family from the live HIP-event totals."""
    dom = max(stats, key=lambda f: stats[f]["ms"])
    d = stats[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    if dom.startswith("chol"):
        # factorisation: both kernel families together, flop bound (FP64 MFMA)
        fl = stats["chol_update"]["flops"] + stats["chol_panel"]["flops"]
        ms = stats["chol_update"]["ms"] + stats["chol_panel"]["ms"]
        ach = fl / (ms * 1e-3) / 1e12
        roof = {"kernel": "chol_update+chol_panel", "bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS["f64"],
                "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["f64"], "traffic": None}
    else:
        by_per = d["bytes"] / max(d["launches"], 1)
        fl_per = d["flops"] / max(d["launches"], 1)
        intensity = fl_per / by_per if by_per else 0.0
        prec = "f32" if dom.endswith("f32") else "f64"
        ridge = PEAK_TFLOPS[prec] * 1e3 / HBM_PEAK_GBS
        if intensity >= ridge:
            ach = fl_per / (avg_ms * 1e-3) / 1e12
            roof = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                    "frac": ach / PEAK_TFLOPS[prec], "traffic": None}
        else:
            ach = by_per / (avg_ms * 1e-3) / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": ach / HBM_PEAK_GBS, "traffic": None}
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_step"] = d["launches"] / steps
    return roof


def _c3_problem(i):
    from workloads import config_c3_problem

    return config_c3_problem(i)


def bench_c3(args):
    """Batched workload: nprob 2D anisotropic Q1 problems (L ~ U{128..512}, 4x4 boxes, k=32, p=8), one
    batched setup + one batched PCG solve per step."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1), mp_context=mp.get_context("spawn")) as ex:
        Ps = list(ex.map(_c3_problem, range(args.nprob)))
    print(f"generated {len(Ps)} problems in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_2101_12164_amd as ns

    assert torch.cuda.is_available(), "bench.py needs a GPU"

    def T(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")

    probs = [(T(P.row_ptr, torch.int64), T(P.col, torch.int32), T(P.val, torch.float64), T(P.part, torch.int32))
             for P in Ps]
    oms = [T(P.omega(), torch.float64) for P in Ps]
    bs = [T(P.b(), torch.float64) for P in Ps]
    torch.cuda.synchronize()
    k, p = Ps[0].k, Ps[0].p
    prec = ns.NS_FP32 if args.prec == "fp32" else ns.NS_FP64

    def step():
        h, infos = ns.nystrom_schur_setup_batched(probs, k=k, p=p, omegas=oms, tol_inner=0.1, prec_inner=prec)
        try:
            xs, outs = ns.nystrom_schur_pcg_solve_batched(h, bs, rtol=1e-8, maxit=2000)
        finally:
            ns.nystrom_schur_destroy(h)
        return infos, outs

    for _ in range(args.warmup):
        step()
        print("warmup step done", file=sys.stderr, flush=True)
    ns.nystrom_schur_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        infos, outs = step()
        print(f"step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    stats = {f: ns.nystrom_schur_kernel_stats(f) for f in ns.KERNEL_FAMILIES}
    ns.nystrom_schur_kernel_timing(False)
    its = np.array([o["it_pcg"] for o in outs])
    isi = np.array([i["it_inner"] for i in infos])
    line = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (inner block CG f32)" if prec == ns.NS_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(Ps)} 2D anisotropic Q1 problems (eps 1e-3, random angle), L ~ U{{128..512}}, "
                               f"4x4 box subdomains, k={k} p={p}, eps_SI=0.1, rtol 1e-8, one batched setup + "
                               "batched PCG per step",
                   "n_total": int(sum(P.n for P in Ps)), "n_gamma_total": int(sum(P.n_gamma for P in Ps)),
                   "inner_prec": args.prec},
        "problems_per_s": len(Ps) / sec,
        "it_SI": {"min": int(isi.min()), "mean": float(isi.mean()), "max": int(isi.max())},
        "it_PCG": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max())},
        "relres_true_max": max(o["relres_true"] for o in outs),
        "t_setup_s": infos[0]["t_total"],
        "t_solve_s": outs[0]["t_solve"],
        "t_phases_s": {kk: infos[0][kk] for kk in ("t_extract", "t_factor", "t_inner", "t_nystrom")},
        "roofline": roofline(stats, args.steps),
        "kernels": {f: {"ms_total": v["ms"], "launches": v["launches"]} for f, v in stats.items() if v["launches"]},
    }
    print(json.dumps(line))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is design-only "
                                   "(see DESIGN.md)", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "c3":
        bench_c3(args)
        return

    import numpy as np
    import torch

    import paper_2101_12164_amd as ns
    from workloads import config_c2

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda"
    P = config_c2(N=args.grid, nb=args.boxes)

    def T(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

    A = dict(row_ptr=T(P.row_ptr, torch.int64), col_idx=T(P.col, torch.int32), val=T(P.val, torch.float64),
             part=T(P.part, torch.int32))
    omega = T(P.omega(), torch.float64)
    b = T(P.b(), torch.float64)
    torch.cuda.synchronize()

    def step(prec):
        s = ns.NystromSchur(A["row_ptr"], A["col_idx"], A["val"], A["part"], k=P.k, p=P.p, omega=omega,
                            tol_inner=P.tol_inner, prec_inner=prec, trsm_cols=args.trsm_cols)
        x, info = s.solve(b, rtol=P.tol_outer, maxit=2000)
        si = s.setup_info
        s.close()
        return si, info

    main_prec = ns.NS_FP32 if args.prec == "fp32" else ns.NS_FP64
    for _ in range(args.warmup):
        step(main_prec)
        print("warmup step done", file=sys.stderr, flush=True)

    ns.nystrom_schur_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(step(main_prec))
        print(f"step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {f: ns.nystrom_schur_kernel_stats(f) for f in ns.KERNEL_FAMILIES}
    ns.nystrom_schur_kernel_timing(False)
    sec = (t1 - t0) / args.steps
    si, info = runs[-1]

    # factor bytes streamed per Schur apply (forward + backward sweep, algorithmic)
    bp = np.bincount(P.part[P.part >= 0])
    tri = float(np.sum(bp * (bp + 1) / 2))

    def bcg_gbs(si_, prec):
        napply = si_["it_inner"] + 1
        by = napply * 2.0 * tri * (4 if prec == ns.NS_FP32 else 8)
        return by / si_["t_inner"] / 1e9 if si_["t_inner"] > 0 else None

    out_extra = {
        "it_SI": si["it_inner"],
        "it_PCG": info["it_pcg"],
        "relres_true": info["relres_true"],
        "relres_schur": info["relres_schur"],
        "k_eff": si["k_eff"],
        "t_setup_s": si["t_total"],
        "t_solve_s": info["t_solve"],
        "t_phases_s": {k: si[k] for k in ("t_extract", "t_factor", "t_inner", "t_nystrom")},
        "schur_bcg_gbs": bcg_gbs(si, main_prec),
    }
    if not args.no_fp64_compare and main_prec != ns.NS_FP64:
        t2 = time.perf_counter()
        si64, info64 = step(ns.NS_FP64)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print("fp64 comparison step done", file=sys.stderr, flush=True)
        out_extra["plain_fp64"] = {
            "sec_per_step": t3 - t2,
            "it_SI": si64["it_inner"],
            "it_PCG": info64["it_pcg"],
            "relres_true": info64["relres_true"],
            "t_inner_s": si64["t_inner"],
            "schur_bcg_gbs": bcg_gbs(si64, ns.NS_FP64),
        }

    # dominant kernel family in the timed region -> roofline
    kern = {f: {"ms_total": v["ms"], "launches": v["launches"]} for f, v in stats.items() if v["launches"]}
    roof = roofline(stats, args.steps)

    line = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (inner block CG f32)" if main_prec == ns.NS_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"3D 7-point lognormal diffusion sigma=2 ell=8, {args.grid}^3 grid, "
                               f"{args.boxes}^3 box subdomains, k={P.k} p={P.p}, eps_SI=0.1, rtol 1e-8",
                   "n": P.n, "n_gamma": P.n_gamma, "inner_prec": args.prec},
        "roofline": roof,
        "kernels": kern,
    }
    line.update(out_extra)

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(P, si["it_inner"], info["it_pcg"])
    print(json.dumps(line))


def cpu_baseline(P, it_si, it_pcg):
    """FP64 oracle timed on the host on a bounded sample of the same workload.

    Sample: the oracle's factorisation (dense LAPACK Cholesky of every interior
    block, sparse factorisation of A_Gamma), one Schur-operator application
    with k+p columns and one outer PCG iteration (S apply + A_Gamma solve).
    Scaled to one full step: the block-CG applications x (it_SI + 1), the PCG
    iteration x it_PCG (the iteration counts measured on the GPU).
    """
    import numpy as np

    from oracle import DBBD, Operators

    t = {}
    t0 = time.perf_counter()
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ops = Operators(d, factor="dense", gamma_factor="sparse")
    t["extract_factor"] = time.perf_counter() - t0
    s = P.k + P.p
    X = np.random.default_rng(0).standard_normal((d.n_gamma, s))
    t0 = time.perf_counter()
    ops.S(X)
    ops.solve_G(X)
    t["bcg_apply"] = time.perf_counter() - t0
    r = np.random.default_rng(1).standard_normal(d.n_gamma)
    t0 = time.perf_counter()
    ops.S(r)
    ops.solve_G(r)
    t["pcg_iter"] = time.perf_counter() - t0
    est = t["extract_factor"] + (it_si + 1) * t["bcg_apply"] + it_pcg * t["pcg_iter"]
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": est, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle DBBD split + factorisation of all {d.n_sub} blocks and A_Gamma (x1), one block-CG "
                      f"application S and A_Gamma^-1 on {s} columns (x{it_si + 1}), one PCG iteration (x{it_pcg}); "
                      f"seconds {json.dumps({k: round(v, 3) for k, v in t.items()})}"}


if __name__ == "__main__":
    main()
