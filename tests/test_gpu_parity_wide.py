"""GPU: sketches of 96 to 160 columns (the width of the 2048^2 benchmark system), where the s x s Cholesky
factors of the block CG and of the Cholesky-QR no longer fit in LDS as dense matrices and the packed-tile
kernels run (lower 16 x 16 tiles in LDS, solves one 16-column chunk per wave in registers).  Against the FP64
oracle on a 2D lognormal problem small enough for it: it_SI and it_PCG within one, M r element by element,
k_eff, and the 1e-8 true residual, with FP64 and FP32 inner work; widths that are and are not multiples of 16."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup, oracle, rel  # noqa: E402
from workloads import make_problem  # noqa: E402

CASES = [(120, 40), (100, 30), (72, 24), (150, 7)]


@pytest.fixture(scope="module")
def base():
    return make_problem((128, 128), (4, 4), sigma=2.0, ell=8.0, k=8, p=2)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("k,p", CASES, ids=[f"k{k}p{p}" for k, p in CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_sketch_matches_oracle(base, k, p, prec):
    P = base
    om = np.random.default_rng(17).standard_normal((P.n_gamma, k + p))
    o = oracle(P, k=k, p=p, omega=om)
    so = o.setup()
    ro = o.solve(P.b(), tol=1e-8)
    pr = {"fp64": ns.NS_FP64, "fp32": ns.NS_FP32}[prec]
    g = gpu_setup(P, omega=om, k=k, p=p, prec_inner=pr)
    try:
        si = g.setup_info
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
        R = np.random.default_rng(4).standard_normal((P.n_gamma, 3))
        em = rel(ns.nystrom_schur_apply(g.handle, dev(R)).cpu().numpy(), o.apply(R))
        print(f"[wide] s={k + p} {prec}: it_SI {si['it_inner']} (oracle {so.it_inner}), k_eff {si['k_eff']} "
              f"(oracle {so.k_eff}), it_PCG {info['it_pcg']} (oracle {ro.it_pcg}), relres_true "
              f"{info['relres_true']:.2e}, M r error {em:.2e}", flush=True)
        assert abs(si["it_inner"] - so.it_inner) <= 1
        assert si["k_eff"] == so.k_eff
        assert abs(info["it_pcg"] - ro.it_pcg) <= 1
        assert info["relres_true"] <= 1e-8
        assert em < (1e-7 if prec == "fp64" else 2e-2)
    finally:
        g.close()


def test_wide_sketch_adapted_deflation(base):
    """The A-DEF2 form also solves E = Z^T S Z (k x k, past the dense LDS limit) with the packed kernels."""
    P = base
    k, p = 120, 40
    om = np.random.default_rng(17).standard_normal((P.n_gamma, k + p))
    o = oracle(P, k=k, p=p, omega=om, apply_mode="ADEF2")
    o.setup()
    ro = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, omega=om, k=k, p=p, apply_mode=ns.NS_APPLY_ADEF2)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
        R = np.random.default_rng(4).standard_normal((P.n_gamma, 2))
        em = rel(ns.nystrom_schur_apply(g.handle, dev(R)).cpu().numpy(), o.apply(R))
        print(f"[wide] A-DEF2 s=160: it_PCG {info['it_pcg']} (oracle {ro.it_pcg}), M r error {em:.2e}", flush=True)
        assert abs(info["it_pcg"] - ro.it_pcg) <= 1 and info["relres_true"] <= 1e-8 and em < 1e-7
    finally:
        g.close()
