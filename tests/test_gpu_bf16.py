"""GPU: BF16 operands in the inner block CG (NS_BF16) against the FP64 oracle.

The local Schur blocks and the interface-level inverses are rounded to BF16 (8-bit significand, relative
rounding 2^-9) and multiplied on 16x16x32 BF16 MFMA with FP32 accumulation; the block vectors stay FP32.  The
operators therefore carry a relative error of a few 1e-3 of the products they form; the loose inner tolerance
(eps_SI = 0.1) absorbs it: the counts stay within one of the FP64 oracle and the FP64 outer PCG reaches 1e-8.
Each result reports ||M^bf16 r - M^fp64 r|| / ||M^fp64 r|| against the oracle's M_2."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup, oracle, rel  # noqa: E402
from workloads import config_c1, make_problem  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


PROBS = {
    "c1": lambda: config_c1(),
    "fd2d_60": lambda: make_problem((60, 60), (3, 3), sigma=2.0, ell=6.0, k=10, p=5),
    "lognormal2d_128": lambda: make_problem((128, 128), (4, 4), sigma=2.0, ell=8.0, k=32, p=8),
    "lognormal3d_32": lambda: make_problem((32, 32, 32), (2, 2, 2), sigma=2.0, ell=8.0, k=64, p=16),
}


@pytest.mark.parametrize("name", sorted(PROBS))
def test_bf16_operators_error(name):
    """The BF16 Schur and interface operators against the oracle's FP64 ones: relative error of the BF16
    rounding of the operands (bounded by 1e-2 of the product the rounding acts on)."""
    P = PROBS[name]()
    o = oracle(P)
    g = gpu_setup(P, prec_inner=ns.NS_BF16)
    try:
        for ncols in (1, 33, P.k + P.p):
            X = np.random.default_rng(ncols).standard_normal((o.dbbd.n_gamma, ncols))
            Y = ns.nystrom_schur_schur_apply(g.handle, dev(X), prec=ns.NS_BF16).cpu().numpy()
            err = np.linalg.norm(Y - o.ops.S(X)) / np.linalg.norm(o.ops.W(X))
            Z = ns.nystrom_schur_interface_solve(g.handle, dev(X), prec=ns.NS_BF16).cpu().numpy()
            zref = o.ops.solve_G(X)
            zerr = rel(Z, zref)
            print(f"[bf16] {name} ncols={ncols}: S X error {err:.2e} (of ||W X||), A_G^-1 X error {zerr:.2e}",
                  flush=True)
            assert err <= 1e-2 and zerr <= 1e-2
            assert err >= 1e-6  # the BF16 path really ran (FP32 or FP64 would be far below)
    finally:
        g.close()


@pytest.mark.parametrize("name", sorted(PROBS))
def test_bf16_inner_solve_matches_fp64_oracle(name):
    P = PROBS[name]()
    o = oracle(P)
    r = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, prec_inner=ns.NS_BF16)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=2000)
        R = np.random.default_rng(5).standard_normal((o.dbbd.n_gamma, 3))
        Mr = ns.nystrom_schur_apply(g.handle, dev(R)).cpu().numpy()
        merr = rel(Mr, o.apply(R))
        print(f"[bf16] {name}: it_SI {g.setup_info['it_inner']} (oracle {o.setup_result.it_inner}), it_PCG "
              f"{info['it_pcg']} (oracle {r.it_pcg}), relres_true {info['relres_true']:.2e}, "
              f"||M r - M_fp64 r|| / ||M_fp64 r|| {merr:.2e}", flush=True)
        assert abs(g.setup_info["it_inner"] - o.setup_result.it_inner) <= 1
        assert abs(info["it_pcg"] - r.it_pcg) <= 1
        assert info["relres_true"] <= 1e-8
        assert merr < 0.5
    finally:
        g.close()


def test_bf16_requires_bf16_handle():
    P = config_c1()
    g = gpu_setup(P, prec_inner=ns.NS_FP32)
    try:
        with pytest.raises(ns.NsError):
            ns.nystrom_schur_schur_apply(g.handle, dev(np.ones((P.n_gamma, 2))), prec=ns.NS_BF16)
    finally:
        g.close()
