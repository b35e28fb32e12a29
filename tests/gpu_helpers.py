"""Helpers shared by the GPU tests: move a generated problem to the device and run both sides."""

import numpy as np
import torch

import paper_2101_12164_amd as ns
from oracle import NystromSchurOracle


def to_dev(P, device="cuda"):
    return dict(
        row_ptr=torch.as_tensor(P.row_ptr, dtype=torch.int64, device=device),
        col=torch.as_tensor(P.col, dtype=torch.int32, device=device),
        val=torch.as_tensor(P.val, dtype=torch.float64, device=device),
        part=torch.as_tensor(P.part, dtype=torch.int32, device=device),
    )


def gpu_setup(P, omega=None, **kw):
    d = to_dev(P)
    if omega is None and P.k > 0:
        omega = P.omega()
    om = torch.as_tensor(np.ascontiguousarray(omega), device="cuda") if omega is not None else None
    args = dict(k=P.k, p=P.p, omega=om, tol_inner=P.tol_inner)
    args.update(kw)
    return ns.NystromSchur(d["row_ptr"], d["col"], d["val"], d["part"], **args)


def oracle(P, **kw):
    args = dict(k=P.k, p=P.p, omega=P.omega() if P.k > 0 else None, tol_inner=P.tol_inner)
    args.update(kw)
    return NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, **args)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
