"""Parameter sweeps of the numerical-experiments section on the GPU library.

Runs, on one synthetic system, the studies the paper reports on its own matrices:

* inner tolerance eps_SI (the table on the impact of the tolerance): it_SI and it_PCG of M_2 for
  eps_SI = 0.8, 0.5, 0.3, 0.1, 0.01, beside the first-level preconditioner S~_1 (k = 0);
* rank k with p = 0 (the table on the rank): it_SI and it_PCG;
* oversampling p with k fixed (the table on the oversampling);
* power iterations q (eq. power);
* the variants M_1, M_2, M_3 and their adapted-deflation forms (the table comparing the variants):
  it_SI, it_PCG and it_total = it_SI + it_PCG;
* classic against block CG for the inner system (the table comparing them, and the per-right-hand-side
  histogram): each of the k + p systems solved alone (one column of the sketch, one right-hand side) gives the
  classic iteration count; the block method's it_SI solves them together.

Every number comes from the library (setup + PCG solve through the C ABI); nothing here computes the method.

    python -m paper_2101_12164_amd.sweeps --config c1 --out sweep_c1.json
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import nystrom_schur as ns


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


class Runner:
    """One generated problem on the device; run(**options) -> setup + solve counts."""

    def __init__(self, P):
        self.P = P
        self.A = (_dev(P.row_ptr, torch.int64), _dev(P.col, torch.int32), _dev(P.val, torch.float64),
                  _dev(P.part, torch.int32))
        self.b = _dev(P.b(), torch.float64)
        self.nI = int(np.count_nonzero(P.part >= 0))

    def sketch(self, k, p, variant=ns.NS_VARIANT_M2, seed=None):
        rows = self.nI if variant == ns.NS_VARIANT_M3 else self.P.n_gamma
        rng = np.random.default_rng(self.P.seed if seed is None else seed)
        return _dev(rng.standard_normal((rows, k + p)), torch.float64)

    def run(self, k, p, tol_inner=0.1, rtol=None, maxit=5000, **kw):
        P = self.P
        rtol = P.tol_outer if rtol is None else rtol
        om = self.sketch(k, p, kw.get("variant", ns.NS_VARIANT_M2)) if k > 0 else None
        t0 = time.perf_counter()
        h = ns.NystromSchur(*self.A, k=k, p=p, omega=om, tol_inner=tol_inner, **kw)
        try:
            x, info = h.solve(self.b, rtol=rtol, maxit=maxit)
            torch.cuda.synchronize()
            si = h.setup_info
        finally:
            h.close()
        return {"k": k, "p": p, "tol_inner": tol_inner, "it_SI": si["it_inner"], "it_PCG": info["it_pcg"],
                "it_total": si["it_inner"] + info["it_pcg"], "k_eff": si["k_eff"],
                "relres_true": info["relres_true"], "sec": time.perf_counter() - t0}

    def classic_counts(self, k, p, tol_inner=0.1):
        """Iterations of PCG (preconditioned by A_Gamma^{-1}) on each of the k + p inner systems alone: one
        right-hand side per setup (a one-column sketch)."""
        om = self.sketch(k, p)
        its = []
        for j in range(k + p):
            h = ns.NystromSchur(*self.A, k=1, p=0, omega=om[:, j:j + 1].contiguous(), tol_inner=tol_inner)
            its.append(h.setup_info["it_inner"])
            h.close()
        return its


def sweep(P, k0, p0, quick=False):
    r = Runner(P)
    out = {"problem": P.name, "n": P.n, "n_gamma": P.n_gamma, "k": k0, "p": p0, "rtol": P.tol_outer}
    out["first_level"] = r.run(0, 0)
    out["eps_SI"] = [r.run(k0, p0, tol_inner=t) for t in (0.8, 0.5, 0.3, 0.1, 0.01)]
    ks = (5, 10, 20, 40, 80) if quick else (5, 10, 20, 40, 80, 160, 320)
    out["rank"] = [r.run(k, 0) for k in ks if k <= P.n_gamma]
    out["oversampling"] = [r.run(k0, p) for p in (0, 5, 10, 20, 40) if k0 + p <= P.n_gamma]
    out["power"] = [dict(r.run(k0, p0, power_iters=q), q=q) for q in (0, 1, 2)]
    var = []
    for vname, v in (("M1", ns.NS_VARIANT_M1), ("M2", ns.NS_VARIANT_M2), ("M3", ns.NS_VARIANT_M3)):
        for mname, m in (("", ns.NS_APPLY_M2), ("A-DEF", ns.NS_APPLY_ADEF2)):
            try:
                var.append(dict(r.run(k0, p0, variant=v, apply_mode=m), name=vname + mname))
            except ns.NsError as e:  # e.g. an interface too large for a variant's dense work
                var.append({"name": vname + mname, "error": str(e)})
    out["variants"] = var
    classic = r.classic_counts(k0, p0)
    block = r.run(k0, p0)
    hist, edges = np.histogram(classic, bins=10)
    out["classic_vs_block"] = {"classic_max": int(max(classic)), "classic_mean": float(np.mean(classic)),
                               "classic_counts": classic, "histogram": hist.tolist(),
                               "histogram_edges": edges.tolist(), "block_it_SI": block["it_SI"],
                               "block_it_PCG": block["it_PCG"]}
    return out


def main(argv=None):
    import workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="c1", choices=["c0", "c1", "c2"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--quick", action="store_true")
    a = ap.parse_args(argv)
    P = {"c0": workloads.config_c0, "c1": workloads.config_c1, "c2": workloads.config_c2}[a.config]()
    res = sweep(P, P.k, P.p, quick=a.quick)
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
