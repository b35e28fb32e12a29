"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test ties one oracle routine to a closed form, an identity from the
paper, an invariant, a textbook / library routine, or brute force on a tiny
input, so that a dropped term, a wrong sign, a wrong index or a transposed
operand in the oracle fails at least one of them.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import (DBBD, NystromSchurOracle, Operators, bf_bpcg, dense_schur, full_system_pcg, ideal_s2,
                    nystrom_core, orth, pcg)
from workloads import config_c1, laplacian, make_problem, partition_boxes, random_dbbd


def tiny2d(N=16, nb=2, sigma=0.0, k=4, p=3, seed=0):
    return make_problem((N, N), (nb, nb), sigma=sigma, ell=3.0, k=k, p=p, seed=seed)


def oracle_for(P, **kw):
    args = dict(k=P.k, p=P.p, omega=P.omega(), tol_inner=P.tol_inner)
    args.update(kw)
    return NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, **args)


# ---------------------------------------------------------------------------
# generators (closed forms)


def test_c1_spectrum_closed_form():
    """5-point Dirichlet Laplacian on 64^2: eigenvalues 4 - 2cos(i pi/65) - 2cos(j pi/65)."""
    A = laplacian((64, 64)).toarray()
    ev = np.sort(np.linalg.eigvalsh(A))
    i = np.arange(1, 65)
    lam = (2 - 2 * np.cos(i * np.pi / 65))[:, None] + (2 - 2 * np.cos(i * np.pi / 65))[None, :]
    assert np.allclose(ev, np.sort(lam.ravel()), atol=1e-11)


def test_c1_partition_sizes():
    P = config_c1()
    assert P.n_gamma == 127
    counts = sorted(np.bincount(P.part[P.part >= 0]).tolist())
    assert counts == [961, 992, 992, 1024]
    # separators are row 32 and column 32 (0-based)
    lab = partition_boxes((64, 64), (2, 2)).reshape(64, 64)
    assert np.all(lab[32, :] == -1) and np.all(lab[:, 32] == -1)


# ---------------------------------------------------------------------------
# DBBD split (eq. perm_A)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dbbd_blocks_reassemble(seed):
    P = random_dbbd(seed)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    A = P.csr().toarray()
    perm = np.concatenate([d.I, d.G])
    Ap = A[np.ix_(perm, perm)]
    nI = d.I.size
    assert np.array_equal(Ap[:nI, :nI], d.A_I.toarray())
    assert np.array_equal(Ap[:nI, nI:], d.A_IG.toarray())
    assert np.array_equal(Ap[nI:, :nI], d.A_GI.toarray())
    assert np.array_equal(Ap[nI:, nI:], d.A_G.toarray())
    # A_I block diagonal with blocks in subdomain order
    AI = d.A_I.toarray()
    bp = d.block_ptr
    mask = np.zeros_like(AI, dtype=bool)
    for j in range(d.n_sub):
        mask[bp[j]:bp[j + 1], bp[j]:bp[j + 1]] = True
    assert np.all(AI[~mask] == 0)
    assert np.all(np.diff(d.G) > 0)


def test_dbbd_rejects_cross_coupling_and_asymmetry():
    P = random_dbbd(3)
    A = P.csr().toarray()
    i = np.nonzero(P.part == 0)[0][0]
    j = np.nonzero(P.part == 1)[0][0]
    B = A.copy()
    B[i, j] = B[j, i] = -0.1
    Bs = sp.csr_matrix(B)
    with pytest.raises(ValueError):
        DBBD(P.n, Bs.indptr, Bs.indices, Bs.data, P.part)
    C = A.copy()
    C[i, i + 1 if i + 1 < P.n else i - 1] += 0.5
    Cs = sp.csr_matrix(C)
    with pytest.raises(ValueError):
        DBBD(P.n, Cs.indptr, Cs.indices, Cs.data, P.part)


# ---------------------------------------------------------------------------
# exact solves and the Schur operator (eq. schur_complement, eq. S-1, eq. SI)


@pytest.mark.parametrize("seed", [0, 4])
def test_solves_are_inverses(seed):
    P = random_dbbd(seed, sizes=(12, 9, 15, 4), n_gamma=10)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    for factor in ("dense", "sparse"):
        ops = Operators(d, factor=factor, gamma_factor=factor)
        X = np.random.default_rng(1).standard_normal((d.I.size, 3))
        assert np.allclose(d.A_I @ ops.solve_I(X), X, atol=1e-12)
        Y = np.random.default_rng(2).standard_normal((d.n_gamma, 3))
        assert np.allclose(d.A_G @ ops.solve_G(Y), Y, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 5, 6])
def test_schur_equals_inverse_of_inverse_block(seed):
    """S_Gamma = ((A^{-1})_{Gamma Gamma})^{-1}: an independent route to the Schur complement."""
    P = random_dbbd(seed, sizes=(8, 6, 11), n_gamma=7)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ops = Operators(d)
    Ainv = np.linalg.inv(P.csr().toarray())
    S_ref = np.linalg.inv(Ainv[np.ix_(d.G, d.G)])
    S_op = ops.S(np.eye(d.n_gamma))
    assert np.allclose(S_op, S_ref, rtol=1e-10, atol=1e-10)
    assert np.allclose(ops.W(np.eye(d.n_gamma)), d.A_G.toarray() - S_ref, atol=1e-10)
    # S_I likewise is the inverse of the interior block of A^{-1}
    SI_ref = np.linalg.inv(Ainv[np.ix_(d.I, d.I)])
    assert np.allclose(ops.S_I(np.eye(d.I.size)), SI_ref, rtol=1e-10, atol=1e-10)


def test_schur_spd_and_first_level_spectrum_in_unit_interval():
    """S_Gamma is SPD and Lambda(A_Gamma^{-1} S_Gamma) lies in (0, 1] (section on eq. GEVP)."""
    P = config_c1()
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    S = dense_schur(d)
    assert np.allclose(S, S.T, atol=1e-12)
    lam = sla.eigh(S, d.A_G.toarray(), eigvals_only=True)
    assert lam.min() > 0 and lam.max() <= 1 + 1e-12
    assert 0.02 < lam.min() < 0.05  # c1: about 0.032


def test_smw_identity():
    """eq. S-1: S^{-1} = A_G^{-1} + A_G^{-1} A_GI S_I^{-1} A_IG A_G^{-1}."""
    P = random_dbbd(7, sizes=(9, 10, 6), n_gamma=8)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ops = Operators(d)
    S = ops.S(np.eye(d.n_gamma))
    SI = ops.S_I(np.eye(d.I.size))
    AGi = np.linalg.inv(d.A_G.toarray())
    rhs = AGi + AGi @ d.A_GI.toarray() @ np.linalg.solve(SI, d.A_IG.toarray()) @ AGi
    assert np.allclose(np.linalg.inv(S), rhs, rtol=1e-9, atol=1e-11)


def test_eigen_mapping_of_reformulation():
    """If (lam, u) is an eigenpair of R^-T S R^-1 then 1/lam - 1 is an eigenvalue of
    R^-T A_GI S_I^{-1} A_IG R^-1 (the reformulation section)."""
    P = tiny2d(N=12, sigma=1.0)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ops = Operators(d)
    S = dense_schur(d)
    R = np.linalg.cholesky(d.A_G.toarray()).T  # A_G = R^T R
    Ri = np.linalg.inv(R)
    lam = np.linalg.eigvalsh(Ri.T @ S @ Ri)
    B = d.A_GI.toarray() @ np.linalg.solve(ops.S_I(np.eye(d.I.size)), d.A_IG.toarray())
    mu = np.linalg.eigvalsh(Ri.T @ B @ Ri)
    assert np.allclose(np.sort(1.0 / lam - 1.0), np.sort(mu), rtol=1e-8, atol=1e-9)


# ---------------------------------------------------------------------------
# block PCG


def test_orth_known_singular_values():
    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((50, 6)))
    V, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    s = np.array([1.0, 0.5, 1e-3, 1e-7, 1e-10, 0.0])
    A = U @ np.diag(s) @ V.T
    Q = orth(A, 1e-8)
    assert Q.shape[1] == 4
    assert np.allclose(Q.T @ Q, np.eye(4), atol=1e-12)
    # spans the leading 4 left singular vectors
    assert np.allclose(Q @ (Q.T @ U[:, :4]), U[:, :4], atol=1e-8)


def test_block_pcg_single_column_is_textbook_pcg():
    """With one right-hand side the block method is PCG: compare iterates with SciPy's cg."""
    P = tiny2d(N=14, sigma=1.5)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ops = Operators(d)
    S = ops.S(np.eye(d.n_gamma))
    AGi = np.linalg.inv(d.A_G.toarray())
    f = np.random.default_rng(3).standard_normal((d.n_gamma, 1))
    for m in (1, 2, 4, 7):
        res = bf_bpcg(ops.S, ops.solve_G, f, 0.0, m, 1e-8)
        x_ref, _ = spla.cg(S, f[:, 0], M=AGi, maxiter=m, rtol=1e-300, atol=0.0)
        assert res.iters == m
        assert np.allclose(res.X[:, 0], x_ref, rtol=1e-9, atol=1e-11)


def test_block_pcg_converges_and_terminates():
    P = config_c1()
    o = oracle_for(P)
    d, ops = o.dbbd, o.ops
    F = ops.W(P.omega())
    res = bf_bpcg(ops.S, ops.solve_G, F, 1e-12, 60, 1e-8)
    assert res.converged
    # finite termination: at most ceil(n_gamma / s) + a few iterations in practice
    assert res.iters <= math.ceil(d.n_gamma / F.shape[1]) + 4
    assert np.linalg.norm(ops.S(res.X) - F) / np.linalg.norm(F) < 1e-10
    assert all(w <= F.shape[1] for w in res.widths)


def test_block_pcg_rank_deficient_block_drops_directions():
    P = config_c1()
    o = oracle_for(P)
    ops = o.ops
    Om = P.omega()
    Om[:, 5] = Om[:, 2]  # duplicated sketch column
    F = ops.W(Om)
    res = bf_bpcg(ops.S, ops.solve_G, F, 1e-10, 60, 1e-8)
    assert res.converged
    assert res.widths[0] == F.shape[1] - 1
    assert np.allclose(res.X[:, 5], res.X[:, 2], atol=1e-10)


def test_shifted_inner_solve_equals_paper_form_and_dense_target():
    """At tight inner tolerance: A_G D (shifted form) = A_GI X (Algorithm alg:prec1 step 3-4)
    = A_GI S_I^{-1} A_IG Omega computed densely (eq. S-1)."""
    P = tiny2d(N=16, sigma=1.0, k=4, p=3)
    Om = P.omega()
    a = oracle_for(P, tol_inner=1e-13)
    b = oracle_for(P, tol_inner=1e-13, inner="formA")
    ya = a.setup().Y
    yb = b.setup().Y
    d, ops = a.dbbd, a.ops
    B = d.A_GI.toarray() @ np.linalg.solve(ops.S_I(np.eye(d.I.size)), d.A_IG.toarray())
    ref = B @ Om
    scale = np.linalg.norm(ref)
    assert np.linalg.norm(ya - ref) / scale < 1e-11
    assert np.linalg.norm(yb - ref) / scale < 1e-11


# ---------------------------------------------------------------------------
# Nystrom core (Algorithm alg:nystrom)


def test_nystrom_closed_form():
    """With k >= r: U Sigma U^T = Y C_eps^+ Y^T, C_eps^+ the thresholded pseudo-inverse."""
    rng = np.random.default_rng(0)
    n, s = 40, 8
    Vb, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 10.0 ** -np.arange(n, dtype=float) * 5.0
    B = Vb @ np.diag(lam) @ Vb.T
    Om = rng.standard_normal((n, s))
    Y = B @ Om
    U, Sig, r = nystrom_core(Y, Om, s, 1e-10)
    C = Om.T @ Y
    C = 0.5 * (C + C.T)
    d, V = np.linalg.eigh(C)
    keep = d >= 1e-10 * d.max()
    Cp = V[:, keep] @ np.diag(1.0 / d[keep]) @ V[:, keep].T
    ref = Y @ Cp @ Y.T
    assert np.allclose(U @ np.diag(Sig) @ U.T, ref, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    assert np.all(np.diff(Sig) <= 0)
    assert r == keep.sum()


def test_nystrom_exact_for_low_rank():
    """Nystrom of an SPSD matrix of rank <= s is exact: B G (G^T B G)^+ (BG)^T = B."""
    rng = np.random.default_rng(1)
    n, rk, s = 30, 5, 8
    X = rng.standard_normal((n, rk))
    B = X @ X.T
    Om = rng.standard_normal((n, s))
    U, Sig, r = nystrom_core(B @ Om, Om, 10, 1e-10)
    assert r == rk and U.shape[1] == rk
    assert np.allclose(U @ np.diag(Sig) @ U.T, B, atol=1e-9 * np.abs(B).max())
    # eigenvalues match the exact top eigenvalues of B
    assert np.allclose(Sig, np.sort(np.linalg.eigvalsh(B))[::-1][:rk], rtol=1e-9)


def test_nystrom_truncation_takes_leading_pairs():
    rng = np.random.default_rng(2)
    n, s, k = 60, 14, 4
    Vb, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([[100.0, 50.0, 20.0, 10.0], 1e-3 * rng.random(n - 4)])
    B = Vb @ np.diag(lam) @ Vb.T
    Om = rng.standard_normal((n, s))
    U, Sig, _ = nystrom_core(B @ Om, Om, k, 1e-10)
    assert U.shape == (n, k)
    assert np.allclose(Sig, lam[:4], rtol=1e-3)
    # principal angles to the exact leading eigenvectors are small
    sv = np.linalg.svd(U.T @ Vb[:, :4], compute_uv=False)
    assert sv.min() > 1 - 1e-4


# ---------------------------------------------------------------------------
# the preconditioner and the outer PCG


def test_outer_pcg_is_textbook_pcg():
    P = tiny2d(N=14, sigma=1.0)
    o = oracle_for(P)
    o.setup()
    d = o.dbbd
    S = o.ops.S(np.eye(d.n_gamma))
    M = o.apply(np.eye(d.n_gamma))
    f = np.random.default_rng(9).standard_normal(d.n_gamma)
    for m in (1, 3, 5):
        res = pcg(o.ops.S, o.apply, f, 0.0, m)
        x_ref, _ = spla.cg(S, f, M=M, maxiter=m, rtol=1e-300, atol=0.0)
        assert np.allclose(res.w, x_ref, rtol=1e-9, atol=1e-12)


def test_m2_symmetric_and_k0_is_first_level():
    P = config_c1()
    o = oracle_for(P)
    o.setup()
    rng = np.random.default_rng(0)
    z1, z2 = rng.standard_normal((2, o.dbbd.n_gamma))
    assert abs(z1 @ o.apply(z2) - z2 @ o.apply(z1)) < 1e-12 * np.linalg.norm(z1) * np.linalg.norm(z2) * 10
    o0 = oracle_for(P, k=0, p=0, omega=None)
    o0.setup()
    assert np.allclose(o0.apply(z1), o.ops.solve_G(z1), atol=1e-14)
    # the k=0 iteration count equals SciPy's cg with M = A_Gamma^{-1}
    f = o0.reduce_rhs(P.b())
    it0 = o0.solve(P.b()).it_pcg
    S = dense_schur(o0.dbbd)
    counter = []
    spla.cg(S, f, M=np.linalg.inv(o0.dbbd.A_G.toarray()), rtol=1e-8, atol=0.0, maxiter=500,
            callback=lambda xk: counter.append(1))
    assert abs(it0 - len(counter)) <= 1


def test_full_nystrom_is_exact_inverse_one_iteration():
    """s = n_Gamma and an exact inner solve: Nystrom is exact, M_2 = S^{-1}, PCG takes one step."""
    P = tiny2d(N=12, sigma=1.0)
    ng = P.n_gamma
    Om = np.random.default_rng(5).standard_normal((ng, ng))
    o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=ng, p=0, omega=Om, tol_inner=1e-14,
                           eps_rel=1e-14)
    o.setup()
    S = dense_schur(o.dbbd)
    M = o.apply(np.eye(ng))
    assert np.allclose(M @ S, np.eye(ng), atol=1e-8)
    assert o.solve(P.b()).it_pcg == 1


def test_iteration_ordering_and_parity_c1():
    """S~_2 <= M_2 <= S~_1 in PCG iterations; relative residual reached; true full-system residual small."""
    P = config_c1()
    o = oracle_for(P)
    s = o.setup()
    r = o.solve(P.b(), tol=1e-8)
    assert s.inner_converged and r.converged
    assert r.relres_schur <= 1e-8
    assert r.relres_schur_true <= 2e-8
    assert r.relres_true <= 1e-8
    it1 = oracle_for(P, k=0, p=0, omega=None).solve(P.b()).it_pcg
    s2_apply, _ = ideal_s2(o.dbbd, P.k)
    f = o.reduce_rhs(P.b())
    it2 = pcg(o.ops.S, s2_apply, f, 1e-8, 500).iters
    assert it2 <= r.it_pcg <= it1
    assert it1 >= 1.5 * r.it_pcg


def test_ideal_s2_spectrum():
    """Lambda(S~_2^{-1} S) = {lambda_{k+1}, ..., lambda_n} u {1} (eq. S2)."""
    P = tiny2d(N=14, sigma=1.5)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    k = 5
    app, lam = ideal_s2(d, k)
    S = dense_schur(d)
    M = app(np.eye(d.n_gamma))
    ev = np.sort(np.linalg.eigvals(M @ S).real)
    ref = np.sort(np.concatenate([lam[k:], np.ones(k)]))
    assert np.allclose(ev, ref, rtol=1e-8, atol=1e-10)


def test_adef2_with_exact_eigenbasis_has_ideal_spectrum():
    """A-DEF2 built on exact GEVP eigenvectors: eigenvalues {1 (x k)} u {lambda_{k+1}, ...}."""
    P = tiny2d(N=14, sigma=1.5)
    o = oracle_for(P, apply_mode="ADEF2")
    d = o.dbbd
    k = 5
    S = dense_schur(d)
    lam, Zf = sla.eigh(S, d.A_G.toarray())
    o.Z = Zf[:, :k]
    o.Sigma = np.zeros(k)
    o._post_setup()
    o.setup_result = object()
    M = o.apply(np.eye(d.n_gamma))
    ev = np.sort(np.linalg.eigvals(M @ S).real)
    ref = np.sort(np.concatenate([lam[k:], np.ones(k)]))
    assert np.allclose(ev, ref, rtol=1e-7, atol=1e-9)


def test_cg_error_bound_every_iterate():
    """eq. k-th_error_cg with kappa = kappa(M_2 S), A-norm error of every PCG iterate."""
    P = tiny2d(N=16, sigma=2.0, k=4, p=3)
    o = oracle_for(P)
    o.setup()
    d = o.dbbd
    S = dense_schur(d)
    M = o.apply(np.eye(d.n_gamma))
    ev = np.linalg.eigvals(M @ S).real
    kappa = ev.max() / ev.min()
    f = o.reduce_rhs(P.b())
    wstar = np.linalg.solve(S, f)
    iters = []
    pcg(o.ops.S, o.apply, f, 1e-12, 200, callback=lambda w: iters.append(w.copy()))
    e0 = math.sqrt(wstar @ S @ wstar)
    q = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    for j, w in enumerate(iters, start=1):
        e = w - wstar
        assert math.sqrt(max(e @ S @ e, 0.0)) <= 2 * e0 * q ** j * (1 + 1e-8) + 1e-12


def test_full_system_block_preconditioner_spectrum():
    """Lambda(M^{-1} A) = Lambda(S~^{-1} S_Gamma) u {1} for the approximate block factorisation."""
    P = tiny2d(N=12, sigma=1.0)
    o = oracle_for(P)
    o.setup()
    d, ops = o.dbbd, o.ops
    perm = np.concatenate([d.I, d.G])
    A = P.csr().toarray()[np.ix_(perm, perm)]
    nI = d.I.size
    n = A.shape[0]
    Minv = np.zeros((n, n))
    E = np.eye(n)
    for c in range(n):
        r = E[:, c]
        uI = ops.solve_I(r[:nI])
        yG = o.apply(r[nI:] - d.A_GI @ uI)
        Minv[:nI, c] = uI - ops.solve_I(d.A_IG @ yG)
        Minv[nI:, c] = yG
    ev = np.sort(np.linalg.eigvals(Minv @ A).real)
    S = dense_schur(d)
    evS = np.linalg.eigvals(o.apply(np.eye(d.n_gamma)) @ S).real
    ref = np.sort(np.concatenate([evS, np.ones(nI)]))
    assert np.allclose(ev, ref, rtol=1e-7, atol=1e-9)
    res = full_system_pcg(o, P.b(), tol=1e-10)
    assert res.converged


def test_sparse_and_dense_factors_agree():
    P = tiny2d(N=20, sigma=2.0, k=5, p=4)
    a = oracle_for(P)
    b = oracle_for(P, factor="sparse", gamma_factor="sparse")
    ra, rb = a.solve(P.b()), b.solve(P.b())
    assert a.setup_result.it_inner == b.setup_result.it_inner
    assert abs(ra.it_pcg - rb.it_pcg) <= 1
    assert np.linalg.norm(ra.x - rb.x) / np.linalg.norm(ra.x) < 1e-7
