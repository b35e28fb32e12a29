"""GPU parity on a mid-size problem that runs the benchmark's kernel paths, element by element against the FP64
oracle: 3D lognormal diffusion (sigma 2, correlation 8 cells) on 32^3 with 2^3 box subdomains (interiors of
16^3 down to 15^3 nodes: half-bandwidths of 225-256 rows, so the four-tile register sweeps of the local Schur
formation), k = 64, p = 16 (the 80-column applies of the inner block CG and the 65-column ragged case).

Tolerances: FP64 operators 1e-11 relative to the largest entry of the result (the rounding of the block solves),
FP32 operators 1e-4 (FP32 arithmetic on these conditioning levels), counts within +-1, relative residual 1e-8."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup, oracle, rel  # noqa: E402
from workloads import make_problem  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def problem():
    return make_problem((32, 32, 32), (2, 2, 2), sigma=2.0, ell=8.0, k=64, p=16, name="lognormal3d_32")


@pytest.fixture(scope="module")
def mid():
    P = problem()
    print(f"[mid] n={P.n} n_gamma={P.n_gamma} k={P.k} p={P.p}", flush=True)
    o = oracle(P)
    r = o.solve(P.b(), tol=1e-8)
    g64 = gpu_setup(P, prec_inner=ns.NS_FP64)
    g32 = gpu_setup(P, prec_inner=ns.NS_FP32)
    yield P, o, r, g64, g32
    g64.close()
    g32.close()


def elementwise(Y, ref, tol):
    return float(np.max(np.abs(Y - ref))) <= tol * float(np.max(np.abs(ref)))


def test_band_and_sizes(mid):
    P, o, r, g64, g32 = mid
    sizes = np.diff(o.dbbd.block_ptr)
    assert sizes.min() == 15 ** 3 and sizes.max() == 16 ** 3
    assert g64.sizes()["n_gamma"] == o.dbbd.n_gamma


def test_factor_blocks(mid):
    P, o, r, g64, g32 = mid
    bp = o.dbbd.block_ptr
    for j in (0, o.dbbd.n_sub - 1):
        L = ns.nystrom_schur_export_factor(g64.handle, j, int(bp[j + 1] - bp[j])).cpu().numpy()
        assert rel(L, o.ops.block_factor(j)) < 1e-12


@pytest.mark.parametrize("ncols", [1, 65, 80])
def test_schur_apply_fp64_and_fp32(mid, ncols):
    P, o, r, g64, g32 = mid
    X = np.random.default_rng(ncols).standard_normal((o.dbbd.n_gamma, ncols))
    ref = o.ops.S(X)
    Y = ns.nystrom_schur_schur_apply(g64.handle, dev(X)).cpu().numpy()
    assert rel(Y, ref) < 1e-11 and elementwise(Y, ref, 1e-11)
    Y32 = ns.nystrom_schur_schur_apply(g32.handle, dev(X), prec=ns.NS_FP32).cpu().numpy()
    assert rel(Y32, ref) < 1e-4 and elementwise(Y32, ref, 1e-4)


@pytest.mark.parametrize("ncols", [65, 80])
def test_interface_solve_fp64_and_fp32(mid, ncols):
    P, o, r, g64, g32 = mid
    X = np.random.default_rng(7 + ncols).standard_normal((o.dbbd.n_gamma, ncols))
    ref = o.ops.solve_G(X)
    Y = ns.nystrom_schur_interface_solve(g64.handle, dev(X)).cpu().numpy()
    assert rel(Y, ref) < 1e-11 and elementwise(Y, ref, 1e-11)
    Y32 = ns.nystrom_schur_interface_solve(g32.handle, dev(X), prec=ns.NS_FP32).cpu().numpy()
    assert rel(Y32, ref) < 1e-4 and elementwise(Y32, ref, 1e-4)


def test_interior_solve_80(mid):
    P, o, r, g64, g32 = mid
    X = np.random.default_rng(3).standard_normal((o.dbbd.I.size, 80))
    Y = ns.nystrom_schur_interior_solve(g64.handle, dev(X)).cpu().numpy()
    ref = o.ops.solve_I(X)
    assert rel(Y, ref) < 1e-11 and elementwise(Y, ref, 1e-11)


def test_counts_apply_and_solve(mid):
    P, o, r, g64, g32 = mid
    for g in (g64, g32):
        si = g.setup_info
        print(f"[mid] it_SI gpu {si['it_inner']} oracle {o.setup_result.it_inner}", flush=True)
        assert abs(si["it_inner"] - o.setup_result.it_inner) <= 1
        assert si["k_eff"] == o.setup_result.k_eff
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=1000)
        print(f"[mid] it_PCG gpu {info['it_pcg']} oracle {r.it_pcg} relres_true {info['relres_true']:.2e}",
              flush=True)
        assert abs(info["it_pcg"] - r.it_pcg) <= 1
        assert info["relres_true"] <= 1e-8
        assert rel(x.cpu().numpy(), r.x) < 1e-6
    if g64.setup_info["it_inner"] == o.setup_result.it_inner:
        R = np.random.default_rng(5).standard_normal((o.dbbd.n_gamma, 3))
        Z = ns.nystrom_schur_apply(g64.handle, dev(R)).cpu().numpy()
        assert rel(Z, o.apply(R)) < 1e-7
