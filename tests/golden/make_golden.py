"""Write the stored expected values under tests/golden/ from the FP64 oracle only.

Run from the repository root:  python tests/golden/make_golden.py
Each fixture records the configuration it was computed on.  Nothing here
calls the HIP library.
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import NystromSchurOracle  # noqa: E402
from workloads import config_c1, config_c2  # noqa: E402


def c1_record(seed=0):
    P = config_c1(seed=seed)
    out = {}
    for mode in ("M2", "ADEF2"):
        o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=P.k, p=P.p, omega=P.omega(),
                               tol_inner=P.tol_inner, apply_mode=mode)
        s = o.setup()
        r = o.solve(P.b(), tol=P.tol_outer)
        out[mode] = dict(it_inner=s.it_inner, k_eff=s.k_eff, it_pcg=r.it_pcg, relres_schur=r.relres_schur,
                         relres_true=r.relres_true)
    o1 = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=0, p=0, omega=None)
    out["S1"] = dict(it_pcg=o1.solve(P.b(), tol=P.tol_outer).it_pcg)
    return dict(config="c1: 2D 5-point Laplacian 64x64, 2x2 boxes, k=20, p=10, eps_SI=0.1, tol 1e-8, seed %d" % seed,
                **out)


def c2_record():
    """The 64^3 lognormal system end to end (dense per-block factors: a few minutes on 8 cores)."""
    P = config_c2()
    o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=P.k, p=P.p, omega=P.omega(),
                           tol_inner=P.tol_inner, factor="dense")
    s = o.setup()
    r = o.solve(P.b(), tol=P.tol_outer)
    return dict(config="c2: 3D 7-point lognormal sigma=2 ell=8 on 64^3, 4x4x4 boxes, k=64, p=16, eps_SI=0.1, "
                       "tol 1e-8, seed %d" % P.seed,
                M2=dict(it_inner=s.it_inner, k_eff=s.k_eff, it_pcg=r.it_pcg, relres_schur=r.relres_schur,
                        relres_true=r.relres_true))


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c2"]
    for name, rec in (("c1", lambda: c1_record(0)), ("c2", c2_record)):
        if name not in which:
            continue
        path = os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json")
        with open(path, "w") as fh:
            json.dump(rec(), fh, indent=2)
        print("wrote", path)
