#!/usr/bin/env python
"""Benchmark of the Nystrom-Schur hot path on one MI355X.

One step = the whole path on one synthetic system already resident in HBM:
DBBD extraction, batched Cholesky of the interior and interface blocks, the
block CG on the shifted Schur system (k+p sketch columns, eps_SI = 0.1), the
Nystrom core, and the PCG solve of A x = b to relative residual 1e-8 with the
block LDL^T back-substitution.

Workload (default): 2D 5-point lognormal diffusion (sigma 2, correlation 8
cells) on a 2048^2 grid, 32x32 box subdomains (63^2 interiors), k = 128,
p = 32, everything FP64 (the value).  The same step with the inner block CG in
FP32 and with BF16 operator operands is timed beside it, each with its counts
and its preconditioner's distance to the FP64 one.  --workload c2 runs the
64^3 lognormal system, c3 the batched anisotropic set, c4 the learned proposal.

Prints ONE JSON line.  `value` = median seconds per step (setup + solve) over
the measured steps, which run untouched (no events; block-CG and PCG iterations
replayed from graphs); lower is better.  `roofline` is computed live from HIP
events bracketing every launch of the dominant kernel family (the one with the
most device time in the warm-up) over the same number of steps run again with
those events; `cpu_baseline` times the FP64 oracle on the host on a bounded
sample of the same workload.
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
    ap.add_argument("--prec", choices=["fp32", "fp64", "bf16"], default=None,
                    help="inner block-CG precision of the timed steps (default: fp64 for the single systems, the "
                         "other precision timed beside it; fp32 for the batched set)")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--trsm-cols", type=int, default=0)
    ap.add_argument("--timing", choices=["dominant", "all", "none"], default="dominant",
                    help="kernel families timed with HIP events in the measured steps")
    ap.add_argument("--pcg-graph", type=int, default=0,
                    help="PCG iterations per replayed HIP graph (0: library default, -1: plain launches)")
    ap.add_argument("--workload", choices=["c5", "c2", "c3", "c4"], default="c5",
                    help="c5: the 2048^2 lognormal system (default line); c2: the 64^3 lognormal system; "
                         "c3: the batched anisotropic set; c4: the learned proposal on the 48^3 lognormal family")
    ap.add_argument("--nprob", type=int, default=256, help="problems of the batched workload")
    ap.add_argument("--ntrain", type=int, default=2000, help="c4: training instances (seeds 0..ntrain-1)")
    ap.add_argument("--nheld", type=int, default=32, help="c4: held-out instances (seeds 10000..)")
    ap.add_argument("--epochs", type=int, default=6, help="c4: passes over the training instances")
    ap.add_argument("--nval", type=int, default=16, help="c4: validation seeds (5000..) for the threshold")
    args = ap.parse_args()
    if args.prec is None:
        args.prec = "fp32" if args.workload == "c3" else "fp64"
    return args


def dominant_families(stats, scope="dominant"):
    """Kernel families to time in the measured steps: the one with the most device time (the two
    factorisation families together), all of them, or none."""
    if scope == "none":
        return []
    if scope == "all":
        return list(stats)
    work = {f: v for f, v in stats.items() if v["bytes"] > 0 or v["flops"] > 0}
    dom = max(work or stats, key=lambda f: stats[f]["ms"])
    return ["chol_update", "chol_panel"] if dom.startswith("chol") else [dom]


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic_{}_{}.json")


def measured_traffic(family, workload):
    """HBM bytes per launch of a kernel family from the committed counter profile of this workload, or None
    when there is none or a source file it names has changed since the counters were taken."""
    import hashlib

    path = TRAFFIC_FILE.format(family, workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    root = os.path.dirname(os.path.abspath(__file__))
    for rel, digest in rec.get("sources", {}).items():
        fp = os.path.join(root, rel)
        if not os.path.exists(fp):
            return None
        with open(fp, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return rec.get("traffic_bytes_per_launch")


def roofline(stats, steps, workload=None):
    """Roofline of the dominant kernel family from the live HIP-event totals."""
    # the dominant family among those with algorithmic work (the one-workgroup s x s kernels carry none:
    # they are latency-bound and have no roofline of their own)
    work = {f: v for f, v in stats.items() if v["bytes"] > 0 or v["flops"] > 0}
    if not work:
        return None
    dom = max(work, key=lambda f: work[f]["ms"])
    d = stats[dom]
    if not d["launches"]:
        return None
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
    if workload is not None:
        roof["traffic"] = measured_traffic(roof["kernel"], workload)
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_step"] = d["launches"] / steps
    return roof


def _c3_problem(i):
    from workloads import config_c3_problem

    return config_c3_problem(i)


def _c4_problem(seed):
    import numpy as np

    from workloads import config_c4

    P = config_c4(seed=seed)
    N = P.shape[0]
    idx = np.indices(P.shape).reshape(3, -1).T[:, ::-1]
    coords = 2.0 * idx / (N - 1) - 1.0
    return P, coords


def bench_c4(args):
    """Learned proposal: train the network on the GPU with the Nystrom bases the method produces for the
    training seeds, then set up + solve held-out seeds with the network's proposal (judged by Rayleigh-Ritz,
    plain Nystrom on rejection) and with plain Nystrom."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    # the generator processes start before anything touches the GPU and serve every chunk
    ex = ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1), mp_context=mp.get_context("spawn"))

    def gen(seeds):
        return list(ex.map(_c4_problem, seeds, chunksize=4))

    t0 = time.perf_counter()
    held = gen(range(10000, 10000 + args.nheld))
    val = gen(range(5000, 5000 + args.nval))
    first_chunk = gen(range(0, min(100, args.ntrain)))
    print(f"generated first problems in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_2101_12164_amd as ns

    def T(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")

    def dev(P):
        return T(P.row_ptr, torch.int64), T(P.col, torch.int32), T(P.val, torch.float64), T(P.part, torch.int32)

    def setup(P, A, proposal=None, accept_tol=0.2):
        return ns.NystromSchur(*A, k=P.k, p=P.p, omega=T(P.omega(), torch.float64), tol_inner=P.tol_inner,
                               prec_inner=ns.NS_FP32, proposal=proposal, accept_tol=accept_tol)

    k, hidden = first_chunk[0][0].k, 256
    data = []
    t_collect = time.perf_counter()
    chunk = first_chunk
    for c0 in range(0, args.ntrain, 100):
        if c0 > 0:
            chunk = gen(range(c0, min(c0 + 100, args.ntrain)))
        for P, C in chunk:
            A = dev(P)
            h = setup(P, A)
            U, _ = ns.nystrom_schur_get_basis(h.handle)
            h.close()
            X = ns.nystrom_schur_features(*A, T(C, torch.float64))
            data.append((X, U.contiguous()))
        print(f"collected {len(data)} training bases", file=sys.stderr, flush=True)
    t_collect = time.perf_counter() - t_collect
    ex.shutdown()

    # initial weights, drawn here (He-normal weights, zero biases; order W1 b1 W2 b2 W3 b3, weights in x out)
    rng0 = np.random.default_rng(12345)
    init = []
    for fan_in, fan_out in ((16, hidden), (hidden, hidden), (hidden, k)):
        init += [rng0.standard_normal(fan_in * fan_out) * np.sqrt(2.0 / fan_in), np.zeros(fan_out)]
    m = ns.nystrom_schur_mlp_create(16, hidden, k, np.concatenate(init).astype(np.float32))
    ns.nystrom_schur_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    rng = np.random.default_rng(0)
    for ep in range(args.epochs):
        tot = 0.0
        for i in rng.permutation(len(data)):
            X, U = data[i]
            tot += ns.nystrom_schur_mlp_loss_grad(m, X, U)
            ns.nystrom_schur_mlp_adam_step(m, 1e-3)
        losses.append(tot / len(data))
        print(f"epoch {ep} loss {losses[-1]:.4f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    stats = {f: ns.nystrom_schur_kernel_stats(f) for f in ("mlp_forward_bf16", "mlp_backward_f32")}
    ns.nystrom_schur_kernel_timing(False)

    # acceptance threshold from validation seeds: proposals forced through, the largest eigen-residual up to
    # which every validation seed converges within one PCG iteration of plain Nystrom (never below 0.2)
    tune = []
    for P, C in val:
        A = dev(P)
        b = T(P.b(), torch.float64)
        Z0 = ns.nystrom_schur_mlp_forward(m, ns.nystrom_schur_features(*A, T(C, torch.float64)), k)
        hf = setup(P, A, Z0, accept_tol=1e30)
        rho = ns.nystrom_schur_get_basis(hf.handle)[1]
        _, of = hf.solve(b, rtol=P.tol_outer, maxit=2000)
        hf.close()
        hp = setup(P, A)
        _, op = hp.solve(b, rtol=P.tol_outer, maxit=2000)
        hp.close()
        tune.append((rho, of["it_pcg"], op["it_pcg"]))
    tau = 0.2
    for rho, itf, itp in sorted(tune):
        if itf > itp + 1:
            break
        tau = max(tau, rho)
    print(f"threshold {tau:.3f} from {len(tune)} validation seeds", file=sys.stderr, flush=True)

    rows = []
    for P, C in held:
        A = dev(P)
        b = T(P.b(), torch.float64)
        Cd = T(C, torch.float64)
        res = {}
        for mode in ("plain", "learned", "plain", "learned"):  # the second pass is timed
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Z0 = ns.nystrom_schur_mlp_forward(m, ns.nystrom_schur_features(*A, Cd), k) if mode == "learned" else None
            h = setup(P, A, Z0, accept_tol=tau)
            x, info = h.solve(b, rtol=P.tol_outer, maxit=2000)
            torch.cuda.synchronize()
            res[mode] = dict(sec=time.perf_counter() - t1, it_pcg=info["it_pcg"], relres=info["relres_true"],
                             accepted=h.setup_info["proposal_accepted"], it_si=h.setup_info["it_inner"],
                             rho=ns.nystrom_schur_get_basis(h.handle)[1] if mode == "learned" else None)
            h.close()
        rows.append(res)
    ns.nystrom_schur_mlp_destroy(m)
    acc = [r["learned"]["accepted"] for r in rows]
    sec_l = float(np.mean([r["learned"]["sec"] for r in rows]))
    sec_p = float(np.mean([r["plain"]["sec"] for r in rows]))
    fw = stats["mlp_forward_bf16"]
    bw = stats["mlp_backward_f32"]
    ach = fw["flops"] / (fw["ms"] * 1e-3) / 1e12 if fw["ms"] > 0 else 0.0
    line = {
        "metric": METRIC,
        "value": sec_l,
        "unit": "s",
        "n_gpus": 1,
        "steps": len(rows),
        "warmup": len(rows),
        "ms_per_step": sec_l * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (inner block CG f32; network BF16 forward, FP32 backward)",
        "data": "synthetic",
        "config": {"workload": f"learned proposal on 3D 7-point lognormal sigma=1.5 ell=8, 48^3 grid, 3^3 box "
                               f"subdomains, k={k} p={held[0][0].p}; network 16-{hidden}-{hidden}-{k} trained on "
                               f"{len(data)} seeds x {args.epochs} epochs; {len(rows)} held-out seeds",
                   "n": held[0][0].n, "n_gamma": held[0][0].n_gamma},
        "plain_sec_per_problem": sec_p,
        "learned_speedup": sec_p / sec_l,
        "accepted": int(sum(acc)),
        "held_out": len(rows),
        "accept_tol": tau,
        "validation": [{"rho": r, "it_pcg_forced": f, "it_pcg_plain": q} for r, f, q in tune],
        "accepted_sec_learned_vs_plain": [float(np.mean([r[m_]["sec"] for r in rows if r["learned"]["accepted"]]))
                                          if any(acc) else None for m_ in ("learned", "plain")],
        "rejected_sec_learned_vs_plain": [float(np.mean([r[m_]["sec"] for r in rows if not r["learned"]["accepted"]]))
                                          if not all(acc) else None for m_ in ("learned", "plain")],
        "rho": {"min": min(r["learned"]["rho"] for r in rows), "max": max(r["learned"]["rho"] for r in rows)},
        "it_PCG_learned": float(np.mean([r["learned"]["it_pcg"] for r in rows])),
        "it_PCG_plain": float(np.mean([r["plain"]["it_pcg"] for r in rows])),
        "it_SI_plain": float(np.mean([r["plain"]["it_si"] for r in rows])),
        "relres_true_max": max(max(r["learned"]["relres"], r["plain"]["relres"]) for r in rows),
        "train": {"loss_per_epoch": losses, "seconds": t_train, "collect_seconds": t_collect,
                  "steps": args.epochs * len(data)},
        "roofline": {"kernel": "mlp_forward_bf16", "bound": "mfma", "achieved": ach, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": ach / 2500.0, "traffic": None,
                     "avg_launch_ms": fw["ms"] / max(fw["launches"], 1), "launches": fw["launches"]},
        "mlp_backward_tflops": bw["flops"] / (bw["ms"] * 1e-3) / 1e12 if bw["ms"] > 0 else 0.0,
    }
    print(json.dumps(line))


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


SINGLE = {
    # workload -> (generator, traffic-profile key, description)
    "c5": ("config_c5", "lognormal2d_2048",
           "2D 5-point lognormal diffusion sigma=2 ell=8, 2048^2 grid, 32^2 box subdomains (63^2 interiors), "
           "k=128 p=32, eps_SI=0.1, rtol 1e-8"),
    "c2": ("config_c2", "lognormal3d_64",
           "3D 7-point lognormal diffusion sigma=2 ell=8, 64^3 grid, 4^3 box subdomains, k=64 p=16, eps_SI=0.1, "
           "rtol 1e-8"),
}
BCG_FAMILIES = {"f64": ("local_schur_apply_f64", "interface_inverse_f64"),
                "f32": ("local_schur_apply_f32", "interface_inverse_f32"),
                "bf16": ("local_schur_apply_bf16", "interface_inverse_bf16")}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on one GPU; sharding by subdomain across GPUs is not "
                                   "implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "c3":
        bench_c3(args)
        return
    if args.workload == "c4":
        bench_c4(args)
        return
    bench_single(args)


def bench_single(args):
    """One system per step (c5 by default, or c2): setup + solve timed per step with plain FP64 inner work
    (the value) and with the FP32 inner block CG (a sidecar)."""
    import statistics

    import numpy as np
    import torch

    import paper_2101_12164_amd as ns
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    gen, traffic_key, desc = SINGLE[args.workload]
    t0 = time.perf_counter()
    P = getattr(workloads, gen)()
    print(f"generated {args.workload} (n={P.n}) in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = "cuda"

    def T(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)

    A = dict(row_ptr=T(P.row_ptr, torch.int64), col_idx=T(P.col, torch.int32), val=T(P.val, torch.float64),
             part=T(P.part, torch.int32))
    omega = T(P.omega(), torch.float64)
    b = T(P.b(), torch.float64)
    # one plain device-to-device copy of 256 MiB: the HBM counters of a profiled run are scaled by what the
    # same counters read for this copy of known size
    cal = torch.empty(2**25, dtype=torch.float64, device=dev)
    torch.empty_like(cal).copy_(cal)
    del cal
    torch.cuda.synchronize()

    tuning = {}

    def step(prec, solve=True):
        s = ns.NystromSchur(A["row_ptr"], A["col_idx"], A["val"], A["part"], k=P.k, p=P.p, omega=omega,
                            tol_inner=P.tol_inner, prec_inner=prec, trsm_cols=args.trsm_cols,
                            pcg_graph_iters=args.pcg_graph)
        info = None
        if solve:
            x, info = s.solve(b, rtol=P.tol_outer, maxit=4000)
        si = s.setup_info
        tuning[["fp64", "fp32", "bf16"][prec]] = ns.nystrom_schur_get_tuning(s.handle)
        s.close()
        return si, info

    def timed_steps(prec, n):
        out, secs = [], []
        for i in range(n):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            out.append(step(prec))
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t1)
            print(f"{['fp64', 'fp32-inner', 'bf16-inner'][prec]} step {i}: {secs[-1] * 1e3:.1f} ms",
                  file=sys.stderr, flush=True)
        return out, secs

    main_prec = {"fp64": ns.NS_FP64, "fp32": ns.NS_FP32, "bf16": ns.NS_BF16}[args.prec]
    # warmup with every kernel family timed: it names the dominant family
    ns.nystrom_schur_kernel_timing(True)
    for _ in range(max(args.warmup, 1)):
        step(main_prec)
        print("warmup step done", file=sys.stderr, flush=True)
    warm = {f: ns.nystrom_schur_kernel_stats(f) for f in ns.KERNEL_FAMILIES}
    timed = dominant_families(warm, args.timing)
    ns.nystrom_schur_kernel_timing(False)
    # the measured steps run as a user's would: no events, iterations replayed from graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs, secs = timed_steps(main_prec, args.steps)
    torch.cuda.synchronize()
    t_region = time.perf_counter() - t0
    sec = statistics.median(secs)
    si, info = runs[-1]
    # the same number of steps again with the dominant family's launches bracketed by HIP events on their stream
    # (events cannot time launches inside a replayed graph, so the loops that contain the family run as plain
    # launches there); the roofline is taken from these launches
    stats = {f: {"ms": 0.0, "launches": 0, "bytes": 0.0, "flops": 0.0} for f in ns.KERNEL_FAMILIES}
    timed_secs = []
    if timed:
        ns.nystrom_schur_kernel_timing_families(timed)
        _, timed_secs = timed_steps(main_prec, args.steps)
        stats = {f: ns.nystrom_schur_kernel_stats(f) for f in ns.KERNEL_FAMILIES}
        ns.nystrom_schur_kernel_timing(False)

    # the other inner precisions, timed the same way after the measured region; each result also reports
    # ||M^mixed r - M^fp64 r|| / ||M^fp64 r|| for four random interface vectors
    R = torch.as_tensor(np.random.default_rng(77).standard_normal((P.n_gamma, 4)), device=dev)

    def apply_of(prec):
        s = ns.NystromSchur(A["row_ptr"], A["col_idx"], A["val"], A["part"], k=P.k, p=P.p, omega=omega,
                            tol_inner=P.tol_inner, prec_inner=prec)
        z = s.apply(R)
        s.close()
        return z

    sides = {}
    if not args.no_fp64_compare:
        ref = apply_of(ns.NS_FP64)
        others = [ns.NS_FP32, ns.NS_BF16] if main_prec == ns.NS_FP64 else [ns.NS_FP64]
        for sp in others:
            step(sp)
            side_runs, side_secs = timed_steps(sp, max(1, args.steps))
            ssi, sinfo = side_runs[-1]
            name = {ns.NS_FP64: "plain_fp64", ns.NS_FP32: "fp32_inner", ns.NS_BF16: "bf16_inner"}[sp]
            sides[name] = {"sec_per_step_median": statistics.median(side_secs), "sec_per_step": side_secs,
                           "it_SI": ssi["it_inner"], "it_PCG": sinfo["it_pcg"], "relres_true": sinfo["relres_true"],
                           "t_setup_s": ssi["t_total"], "t_solve_s": sinfo["t_solve"],
                           "t_inner_s": ssi["t_inner"], "inner_bf16_schur": ssi.get("inner_bf16_schur"),
                           "apply_rel_err_vs_fp64": float(torch.linalg.norm(apply_of(sp) - ref) /
                                                          torch.linalg.norm(ref))}

    # Schur-BCG HBM GB/s: bytes the inner block CG's operator applications move (the explicit local Schur
    # blocks, the interface-level inverses and the block vectors they read and write, each once per apply)
    # over the HIP-event time of those launches, from one setup (no solve) per inner precision
    def bcg_gbs(prec):
        key = {ns.NS_FP64: "f64", ns.NS_FP32: "f32", ns.NS_BF16: "bf16"}[prec]
        ns.nystrom_schur_kernel_timing_families(list(BCG_FAMILIES[key]))
        step(prec, solve=False)
        st_ = [ns.nystrom_schur_kernel_stats(f) for f in BCG_FAMILIES[key]]
        ns.nystrom_schur_kernel_timing(False)
        by = sum(x["bytes"] for x in st_)
        ms = sum(x["ms"] for x in st_)
        return {"gbs": by / (ms * 1e-3) / 1e9 if ms else None, "bytes": by, "ms": ms,
                "launches": int(sum(x["launches"] for x in st_)), "families": list(BCG_FAMILIES[key])}

    gbs_main = bcg_gbs(main_prec)

    kern = {f: {"ms_total": v["ms"], "launches": v["launches"],
                "gbs": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] else None,
                "tflops": v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] else None}
            for f, v in stats.items() if v["launches"]}
    roof = roofline(stats, args.steps, workload=traffic_key)
    if roof is not None:
        roof["measured_in"] = (f"{args.steps} further steps with the {roof['kernel']} launches event-timed on their "
                               f"stream (plain launches in the iterations that contain them; "
                               f"{statistics.median(timed_secs) * 1e3:.1f} ms per step there)")
    prec_name = ["fp64", "fp32", "bf16"][main_prec]
    line = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "mean_ms_per_step": t_region / args.steps * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ["f64", "f64 (inner block CG f32)", "f64 (inner block CG f32, bf16 operator operands)"][main_prec],
        "data": "synthetic",
        "config": {"workload": desc, "n": P.n, "n_gamma": P.n_gamma, "inner_prec": prec_name},
        "roofline": roof,
        "kernels": kern,
        "it_SI": si["it_inner"],
        "it_PCG": info["it_pcg"],
        "relres_true": info["relres_true"],
        "relres_schur": info["relres_schur"],
        "k_eff": si["k_eff"],
        "t_setup_s": si["t_total"],
        "t_solve_s": info["t_solve"],
        "t_phases_s": {k: si[k] for k in ("t_extract", "t_factor", "t_inner", "t_nystrom")},
        "schur_bcg_gbs": gbs_main["gbs"],
        "schur_bcg": {prec_name: gbs_main},
        "tuning": {"table_entries": ns.nystrom_schur_tuning_info()[0], "applied": tuning},
    }
    for name, side in sides.items():
        sp = {"plain_fp64": ns.NS_FP64, "fp32_inner": ns.NS_FP32, "bf16_inner": ns.NS_BF16}[name]
        g_ = bcg_gbs(sp)
        side["schur_bcg_gbs"] = g_["gbs"]
        line[name] = side
        line["schur_bcg"][{"plain_fp64": "fp64", "fp32_inner": "fp32", "bf16_inner": "bf16"}[name]] = g_
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(P, si["it_inner"], info["it_pcg"])
    print(json.dumps(line))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(P, it_si, it_pcg):
    """The FP64 oracle timed on the host cores on a bounded sample of the same workload, scaled to one step.

    Timed whole: the DBBD split and the factorisation of every interior block and of A_Gamma; the Nystrom core
    and Z = A_Gamma^{-1} U; the reduction of b and the back-substitution.  Sampled: the block CG's first
    iteration (with the right-hand side W Omega and the first orthonormalisation) and one later iteration
    (S_Gamma and A_Gamma^{-1} on k+p columns, the Gram products, the block update, the orthonormalisation),
    scaled by it_SI; three outer PCG iterations, scaled by it_PCG (the iteration counts the GPU measured; the
    oracle reaches the same counts within one where it runs whole).  Interior factors are dense LAPACK
    Cholesky blocks up to 4096 unknowns per block times 64 blocks, SuperLU factors otherwise (same result to
    rounding); A_Gamma is factorised by SuperLU.
    """
    import numpy as np
    import scipy.linalg as sla

    from oracle import DBBD, Operators, bf_bpcg, nystrom_core, orth, pcg

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_info = threadpool_limits = None
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1]) if threadpool_info else 0

    t = {}
    t0 = time.perf_counter()
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    nb = np.diff(d.block_ptr)
    factor = "dense" if d.n_sub <= 64 and nb.max() <= 4096 else "sparse"
    ops = Operators(d, factor=factor, gamma_factor="sparse")
    t["extract_factor"] = time.perf_counter() - t0
    s = P.k + P.p
    Om = P.omega()
    t0 = time.perf_counter()
    F = ops.W(Om)
    first = bf_bpcg(ops.S, ops.solve_G, F, 0.0, 1, 1e-6)
    t["bcg_first_iteration"] = time.perf_counter() - t0

    def bcg_iteration():
        Pm = orth(ops.solve_G(F), 1e-6)
        Q = ops.S(Pm)
        Delta = Pm.T @ Q
        cf = sla.cho_factor(0.5 * (Delta + Delta.T), lower=True)
        alpha = sla.cho_solve(cf, Pm.T @ F)
        X = Pm @ alpha
        R = F - Q @ alpha
        Z = ops.solve_G(R)
        beta = -sla.cho_solve(cf, Q.T @ Z)
        return X, orth(Z + Pm @ beta, 1e-6)

    t0 = time.perf_counter()
    bcg_iteration()
    t["bcg_iteration"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Y = d.A_G @ first.X
    U, Sig, _ = nystrom_core(Y, Om, P.k)
    Zl = ops.solve_G(U)
    t["nystrom"] = time.perf_counter() - t0
    b = P.b()
    t0 = time.perf_counter()
    f = b[d.G] - d.A_GI @ ops.solve_I(b[d.I])
    t["reduce_rhs"] = time.perf_counter() - t0

    def M(r):
        return ops.solve_G(r) + Zl @ (Sig * (Zl.T @ r))

    t0 = time.perf_counter()
    res = pcg(ops.S, M, f, 0.0, 3)
    t["pcg_3_iterations"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    ops.solve_I(b[d.I] - d.A_IG @ res.w)
    t["back_substitution"] = time.perf_counter() - t0
    est = (t["extract_factor"] + t["bcg_first_iteration"] + max(it_si - 1, 0) * t["bcg_iteration"] + t["nystrom"]
           + t["reduce_rhs"] + it_pcg * t["pcg_3_iterations"] / 3.0 + t["back_substitution"])
    one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            bcg_iteration()
            one = time.perf_counter() - t0
    return {"value": est, "unit": "s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(), "factor": factor,
            "bcg_iteration_s": t["bcg_iteration"], "bcg_iteration_1thread_s": one,
            "sample": f"oracle on the full system: split + {factor} factorisation of all {d.n_sub} blocks and of "
                      f"A_Gamma, Nystrom core, reduction and back-substitution timed whole; block CG first "
                      f"iteration + one iteration on {s} columns (x{max(it_si - 1, 0)}), 3 PCG iterations "
                      f"(x{it_pcg}/3); seconds {json.dumps({k: round(v, 3) for k, v in t.items()})}"}


if __name__ == "__main__":
    main()
