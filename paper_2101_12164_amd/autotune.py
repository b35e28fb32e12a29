"""Autotuner of the library's automatic settings on the current device.

For each setting the library decides by itself -- columns per workgroup of the multi-column triangular sweeps
(trsm_cols), PCG iterations per replayed graph (pcg_graph_iters), block-CG iterations per replayed graph
(bcg_graph_iters), output columns per workgroup of the local Schur products for 65-80 columns (ls_gemm_cols) --
the tuner times setup + solve for every candidate value on generated problems of several sizes (candidates are
passed as explicit options, which take precedence over any table), checks that every candidate gives the same
counts and solution as the others, keeps the fastest per (kernel, precision, size class), and writes the table
tuning_<arch>.tsv that the library reads from its own directory.

    python -m paper_2101_12164_amd.autotune [--quick] [--out PATH]
"""

from __future__ import annotations

import argparse
import datetime
import json
import os
import statistics
import sys
import time

import numpy as np
import torch

from . import nystrom_schur as ns

HERE = os.path.dirname(os.path.abspath(__file__))


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _arch():
    name = torch.cuda.get_device_properties(0).gcnArchName
    return name.split(":")[0]


class Problem:
    def __init__(self, P):
        self.P = P
        self.A = (_dev(P.row_ptr, torch.int64), _dev(P.col, torch.int32), _dev(P.val, torch.float64),
                  _dev(P.part, torch.int32))
        self.om = _dev(P.omega(), torch.float64)
        self.b = _dev(P.b(), torch.float64)

    def run(self, **opt):
        P = self.P
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = ns.NystromSchur(*self.A, k=P.k, p=P.p, omega=self.om, tol_inner=P.tol_inner, **opt)
        try:
            x, info = h.solve(self.b, rtol=P.tol_outer, maxit=5000)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            return sec, h.setup_info["it_inner"], info["it_pcg"], x
        finally:
            h.close()


def time_candidates(prob, key, values, reps, base):
    """Median seconds of each candidate value of option `key` (other options from `base`), and a check that
    all candidates give the same counts and, to 1e-10, the same solution."""
    out, ref = {}, None
    for v in values:
        opt = dict(base)
        if key in OPTION_KEYS:
            opt[key] = v
        else:
            ns.nystrom_schur_tuning_override(key, v)
        try:
            prob.run(**opt)  # warm-up (workspaces, code objects)
            secs, res = [], None
            for _ in range(reps):
                sec, isi, ipc, x = prob.run(**opt)
                secs.append(sec)
                res = (isi, ipc, x)
        finally:
            if key not in OPTION_KEYS:
                ns.nystrom_schur_tuning_override(key, 0)
        if ref is None:
            ref = res
        else:
            assert res[0] == ref[0] and res[1] == ref[1], (key, v, res[:2], ref[:2])
            err = float(torch.linalg.norm(res[2] - ref[2]) / torch.linalg.norm(ref[2]))
            assert err <= 1e-10, (key, v, err)
        out[v] = statistics.median(secs)
    return out


OPTION_KEYS = ("trsm_cols", "pcg_graph_iters", "bcg_graph_iters")  # settable per handle (ns_options)

# size classes: columns of a block (sweeps, products) and interface rows (iteration graphs)
COL_CLASSES = [(1, 16), (17, 48), (49, 96), (97, 256)]
ROW_CLASSES = [(0, 1000), (1001, 10000), (10001, 60000), (60001, 10 ** 9)]


def cls_of(x, classes):
    for lo, hi in classes:
        if lo <= x <= hi:
            return lo, hi
    return classes[-1]


def tune(quick=False):
    import workloads

    problems = [workloads.config_c1(),
                workloads.make_problem((32, 32, 32), (2, 2, 2), sigma=2.0, ell=8.0, k=64, p=16,
                                       name="lognormal3d_32"),
                workloads.config_c2()]
    if not quick:
        problems.append(workloads.config_c5())
    reps = 2 if quick else 3
    rows, log = [], []
    for P in problems:
        prob = Problem(P)
        s = P.k + P.p
        for prec_name, prec in (("f64", ns.NS_FP64), ("f32", ns.NS_FP32)):
            base = dict(prec_inner=prec)
            cands = {
                "pcg_graph_iters": (1, 2, 4, 8),
                "bcg_graph_iters": (2, 4, 8),
            }
            for key, vals in cands.items():
                if key == "pcg_graph_iters" and prec != ns.NS_FP64:
                    continue  # the outer iteration is FP64 whatever the inner precision
                t = time_candidates(prob, key, vals, reps, base)
                best = min(t, key=t.get)
                lo, hi = cls_of(P.n_gamma, ROW_CLASSES)
                rows.append((key, prec_name if key != "pcg_graph_iters" else "*", lo, hi, best))
                log.append({"problem": P.name, "key": key, "prec": prec_name, "seconds": t, "best": best})
                print(f"[autotune] {P.name} {key} {prec_name}: {json.dumps(t)} -> {best}", file=sys.stderr,
                      flush=True)
            # the sweeps, where the triangular Schur operator makes them matter (systems up to 60 000 interface
            # rows: beyond, that operator is too slow to time repeatedly)
            if P.n_gamma <= 60000:
                t = time_candidates(prob, "trsm_cols", (16, 32, 64), reps,
                                    dict(base, schur_mode=ns.NS_SCHUR_TRIANGULAR))
                best = min(t, key=t.get)
                lo, hi = cls_of(s, COL_CLASSES)
                rows.append(("trsm_cols", prec_name, lo, hi, best))
                log.append({"problem": P.name, "key": "trsm_cols", "prec": prec_name, "seconds": t, "best": best})
                print(f"[autotune] {P.name} trsm_cols {prec_name}: {json.dumps(t)} -> {best}", file=sys.stderr,
                      flush=True)
            if 64 < s <= 80:
                t = time_candidates(prob, "ls_gemm_cols", (64, 80), reps, base)
                best = min(t, key=t.get)
                rows.append(("ls_gemm_cols", prec_name, 65, 80, best))
                log.append({"problem": P.name, "key": "ls_gemm_cols", "prec": prec_name, "seconds": t,
                            "best": best})
    return rows, log


def write_table(rows, path, arch):
    # one entry per (kernel, precision, class): the fastest measured (later problems of the same class win ties)
    table = {}
    for key, prec, lo, hi, v in rows:
        table[(key, prec, lo, hi)] = v
    with open(path, "w") as f:
        f.write(f"# tuned settings for {arch}, written by paper_2101_12164_amd.autotune on "
                f"{datetime.date.today().isoformat()}\n")
        f.write("# arch\tkernel\tprecision\tsize_lo\tsize_hi\tvalue\n")
        for (key, prec, lo, hi), v in sorted(table.items()):
            f.write(f"{arch}\t{key}\t{prec}\t{lo}\t{hi}\t{v}\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--log", default=None)
    a = ap.parse_args(argv)
    arch = _arch()
    rows, log = tune(a.quick)
    path = a.out or os.path.join(HERE, f"tuning_{arch}.tsv")
    write_table(rows, path, arch)
    if a.log:
        with open(a.log, "w") as f:
            json.dump(log, f)
    print(open(path).read())
    return 0


if __name__ == "__main__":
    sys.exit(main())
