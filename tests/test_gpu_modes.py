"""GPU: precision and preconditioner variants, edge cases and error paths, against the FP64 oracle."""

import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2101_12164_amd as ns  # noqa: E402
from gpu_helpers import gpu_setup, oracle, rel, to_dev  # noqa: E402
from workloads import config_c1, make_problem, random_dbbd  # noqa: E402


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


PROBS = {
    "c1": lambda: config_c1(),
    "fd3d_16": lambda: make_problem((16, 16, 16), (2, 2, 2), sigma=2.0, ell=4.0, k=12, p=6),
    "fd2d_60": lambda: make_problem((60, 60), (3, 3), sigma=2.0, ell=6.0, k=10, p=5),
}


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("mode", [ns.NS_SCHUR_TRIANGULAR, ns.NS_SCHUR_LOCAL])
def test_fp32_inner_matches_fp64_oracle(name, mode):
    """FP32 factors / block vectors in the inner block CG (eps_SI = 0.1): counts within +-1 of
    the FP64 oracle and the outer FP64 PCG still reaches 1e-8."""
    P = PROBS[name]()
    o = oracle(P)
    r = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, prec_inner=ns.NS_FP32, schur_mode=mode)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8)
        assert abs(g.setup_info["it_inner"] - o.setup_result.it_inner) <= 1
        assert abs(info["it_pcg"] - r.it_pcg) <= 1
        assert info["relres_true"] <= 1e-8
        assert rel(x.cpu().numpy(), r.x) < 1e-6
        # FP32 operators against the FP64 oracle: error of FP32 arithmetic
        X = np.random.default_rng(0).standard_normal((o.dbbd.n_gamma, 8))
        Y32 = ns.nystrom_schur_schur_apply(g.handle, dev(X), prec=ns.NS_FP32).cpu().numpy()
        assert rel(Y32, o.ops.S(X)) < 1e-4
        Z32 = ns.nystrom_schur_interface_solve(g.handle, dev(X), prec=ns.NS_FP32).cpu().numpy()
        assert rel(Z32, o.ops.solve_G(X)) < 1e-4
    finally:
        g.close()


@pytest.mark.parametrize("name", sorted(PROBS))
def test_adef2_matches_oracle(name):
    P = PROBS[name]()
    o = oracle(P, apply_mode="ADEF2")
    r = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, apply_mode=ns.NS_APPLY_ADEF2)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8)
        assert abs(info["it_pcg"] - r.it_pcg) <= 1, (info["it_pcg"], r.it_pcg)
        assert info["relres_true"] <= 1e-8
        R = np.random.default_rng(3).standard_normal((o.dbbd.n_gamma, 2))
        if g.setup_info["it_inner"] == o.setup_result.it_inner:
            assert rel(ns.nystrom_schur_apply(g.handle, dev(R)).cpu().numpy(), o.apply(R)) < 1e-6
    finally:
        g.close()


def test_k0_is_first_level():
    P = config_c1()
    o = oracle(P, k=0, p=0, omega=None)
    r = o.solve(P.b(), tol=1e-8)
    d = to_dev(P)
    s = ns.NystromSchur(d["row_ptr"], d["col"], d["val"], d["part"], k=0, p=0)
    try:
        x, info = s.solve(dev(P.b()), rtol=1e-8)
        assert abs(info["it_pcg"] - r.it_pcg) <= 1
        R = np.random.default_rng(1).standard_normal((o.dbbd.n_gamma, 3))
        assert rel(ns.nystrom_schur_apply(s.handle, dev(R)).cpu().numpy(), o.ops.solve_G(R)) < 1e-12
    finally:
        s.close()


def test_full_rank_sketch_one_iteration():
    """k = n_Gamma, tight inner tolerance: M_2 = S^{-1} and PCG converges in one iteration."""
    P = make_problem((12, 12), (2, 2), sigma=1.0, ell=3.0, k=4, p=0)
    ng = P.n_gamma
    Om = np.random.default_rng(5).standard_normal((ng, ng))
    g = gpu_setup(P, omega=Om, k=ng, p=0, tol_inner=1e-13, eig_thresh_rel=1e-14)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8)
        assert info["it_pcg"] <= 2
    finally:
        g.close()


def test_duplicate_sketch_columns():
    P = config_c1()
    Om = P.omega()
    Om[:, 7] = Om[:, 3]
    o = oracle(P, omega=Om)
    r = o.solve(P.b(), tol=1e-8)
    g = gpu_setup(P, omega=Om)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8)
        assert abs(g.setup_info["it_inner"] - o.setup_result.it_inner) <= 1
        assert abs(info["it_pcg"] - r.it_pcg) <= 1
    finally:
        g.close()


def test_zero_rhs():
    P = config_c1()
    g = gpu_setup(P)
    try:
        x, info = g.solve(dev(np.zeros(P.n)), rtol=1e-8)
        assert info["it_pcg"] == 0 and float(x.abs().max()) == 0.0
    finally:
        g.close()


def test_not_converged_writes_iterate():
    P = config_c1()
    g = gpu_setup(P)
    try:
        x, info = g.solve(dev(P.b()), rtol=1e-8, maxit=3, raise_on_not_converged=False)
        assert info["status"] == ns.nystrom_schur.NS_ERR_NOT_CONVERGED
        assert info["it_pcg"] == 3 and info["converged"] == 0
        assert np.isfinite(x.cpu().numpy()).all() and info["relres_true"] < 1.0
    finally:
        g.close()


def test_nan_rhs_rejected():
    P = config_c1()
    g = gpu_setup(P)
    try:
        b = P.b()
        b[17] = np.nan
        with pytest.raises(ns.NsError) as e:
            g.solve(dev(b))
        assert e.value.status == ns.nystrom_schur.NS_ERR_INVALID_ARG
    finally:
        g.close()


def test_not_spd_block_reported():
    P = config_c1()
    A = P.csr().tolil()
    i = int(np.nonzero(P.part == 2)[0][10])
    A[i, i] = -4.0
    A = A.tocsr()
    P.row_ptr, P.col, P.val = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    with pytest.raises(ns.NsError) as e:
        gpu_setup(P)
    assert e.value.status == ns.nystrom_schur.NS_ERR_NOT_SPD
    assert e.value.info["bad_block"] == 2


def test_dbbd_violation_rejected():
    P = random_dbbd(4, sizes=(20, 30), n_gamma=8)
    A = P.csr().tolil()
    i = int(np.nonzero(P.part == 0)[0][0])
    j = int(np.nonzero(P.part == 1)[0][0])
    A[i, j] = A[j, i] = -0.05
    A = A.tocsr()
    P.row_ptr, P.col, P.val = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    with pytest.raises(ns.NsError) as e:
        gpu_setup(P)
    assert e.value.status == ns.nystrom_schur.NS_ERR_INVALID_ARG


def test_asymmetric_rejected():
    P = random_dbbd(6, sizes=(20, 30), n_gamma=8)
    A = P.csr().tolil()
    A[3, 3] += 0.0
    r = int(np.nonzero(P.part == 0)[0][0])
    cols = A.rows[r]
    c = [x for x in cols if x != r][0]
    A[r, c] = A[r, c] * 1.5
    A = A.tocsr()
    P.row_ptr, P.col, P.val = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    with pytest.raises(ns.NsError) as e:
        gpu_setup(P)
    assert e.value.status == ns.nystrom_schur.NS_ERR_INVALID_ARG


def test_too_large_sketch_rejected():
    P = config_c1()
    with pytest.raises(ns.NsError) as e:
        gpu_setup(P, omega=np.zeros((P.n_gamma, 128)), k=100, p=28)
    assert e.value.status == ns.nystrom_schur.NS_ERR_INVALID_ARG
