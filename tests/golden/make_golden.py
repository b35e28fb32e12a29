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
from workloads import config_c1  # noqa: E402


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


if __name__ == "__main__":
    path = os.path.join(ROOT, "tests", "golden", "c1_oracle.json")
    with open(path, "w") as fh:
        json.dump(c1_record(0), fh, indent=2)
    print("wrote", path)
