"""Pins of the oracle's method variants (M_1, M_3 and the adapted-deflation forms of the variants section)
and of the power-iteration sketch (eq. power), against facts that do not come from the oracle itself:
dense factorisations, the exact truncated eigendecomposition, the Sherman-Morrison-Woodbury identities and the
closed form of the Nystrom approximation."""

import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import DBBD, GammaFactor, NystromSchurOracle, dense_schur, ideal_s2, level2_order, nystrom_core
from workloads import config_c1, make_problem, random_dbbd


def tiny2d(N=14, nb=2, sigma=1.5, ell=3.0, k=4, p=3, seed=0):
    return make_problem((N, N), (nb, nb), sigma=sigma, ell=ell, k=k, p=p, seed=seed)


def make(P, **kw):
    args = dict(k=P.k, p=P.p, omega=P.omega(), tol_inner=P.tol_inner)
    args.update(kw)
    return NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, **args)


def dense_target(P):
    """B = A_G (A^{-1})_GG A_G - A_G (= A_GI S_I^{-1} A_IG by eq. S-1) and S_I^{-1} = (A^{-1})_II, from the
    dense inverse of A."""
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    Ainv = np.linalg.inv(P.csr().toarray())
    AG = d.A_G.toarray()
    B = AG @ Ainv[np.ix_(d.G, d.G)] @ AG - AG
    return d, 0.5 * (B + B.T), Ainv[np.ix_(d.I, d.I)]


# ---------------------------------------------------------------------------
# the factor R_Gamma


@pytest.mark.parametrize("level2", [True, False])
def test_gamma_factor(level2):
    """R^T R = A_Gamma; R is upper triangular with rows and columns in the level-2 order; the three solves
    invert it."""
    P = make_problem((20, 20), (2, 2), sigma=1.0, ell=4.0, k=4, p=3, level2=level2)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    R = GammaFactor(d)
    ng = d.n_gamma
    I = np.eye(ng)
    Rm = R.mult(I)
    AG = d.A_G.toarray()
    assert np.allclose(Rm.T @ Rm, AG, atol=1e-12 * np.abs(AG).max())
    perm = level2_order(d)
    assert np.allclose(np.tril(Rm[np.ix_(perm, perm)], -1), 0.0)
    assert not np.allclose(np.tril(Rm, -1), 0.0) or not level2
    X = np.random.default_rng(0).standard_normal((ng, 3))
    assert np.allclose(R.solve(R.mult(X)), X, atol=1e-12)
    assert np.allclose(Rm.T @ R.solve_t(X), X, atol=1e-12)
    # the level-2 order puts the separator blocks first and the junction last
    pg = d.part[d.G][perm]
    if level2:
        nj = int(np.count_nonzero(pg == -1))
        assert np.all(pg[ng - nj:] == -1) and np.all(np.diff(-2 - pg[: ng - nj]) >= 0)
    else:
        assert np.array_equal(perm, np.arange(ng))


# ---------------------------------------------------------------------------
# M_1 with the exact truncated EVD is the ideal adapted preconditioner


def exact_sketch(ng, seed=5):
    return np.random.default_rng(seed).standard_normal((ng, ng))


def test_m1_with_exact_truncated_evd_is_ideal_adapted():
    """A square sketch and an exact inner solve make Nystrom exact, so its rank-k truncation is the truncated EVD
    of R^{-T} B R^{-1}.  Then M_1 S has the spectrum {1 (k times)} u {lambda_{k+1}, ..., lambda_n} of the ideal
    S~_2 (the adapted-deflation form derived for the truncated EVD), and so has M_1A-DEF.  M_2 built on the same
    exact Nystrom of B is not the ideal form."""
    P = tiny2d(N=12, sigma=1.5)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ng, k = d.n_gamma, 5
    S = dense_schur(d)
    _, lam = ideal_s2(d, k)
    ref = np.sort(np.concatenate([np.ones(k), lam[k:]]))
    Om = exact_sketch(ng)
    for mode in ("M2", "ADEF2"):
        o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=k, p=ng - k, omega=Om, tol_inner=1e-15,
                               eps_rel=1e-14, variant="M1", apply_mode=mode)
        o.setup()
        ev = np.sort(np.linalg.eigvals(o.apply(np.eye(ng)) @ S).real)
        assert np.allclose(ev, ref, rtol=1e-7, atol=1e-9), mode
    o2 = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=k, p=ng - k, omega=Om, tol_inner=1e-15,
                            eps_rel=1e-14, variant="M2")
    o2.setup()
    ev2 = np.sort(np.linalg.eigvals(o2.apply(np.eye(ng)) @ S).real)
    assert not np.allclose(ev2, ref, rtol=1e-3)


def test_m1_nystrom_eigenvalues_map_to_schur_spectrum():
    """The eigenvalues Nystrom finds for R^{-T} B R^{-1} with an exact square sketch are 1/lambda - 1 for the
    eigenvalues lambda of R^{-T} S R^{-1} (the reformulation section), largest first."""
    P = tiny2d(N=12, sigma=1.0)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ng, k = d.n_gamma, 6
    lam = sla.eigh(dense_schur(d), d.A_G.toarray(), eigvals_only=True)
    o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=k, p=ng - k, omega=exact_sketch(ng),
                           tol_inner=1e-15, eps_rel=1e-14, variant="M1")
    s = o.setup()
    assert np.allclose(s.Sigma, (1.0 / lam - 1.0)[:k], rtol=1e-8)


@pytest.mark.parametrize("variant", ["M1", "M3"])
def test_full_rank_variant_is_exact_inverse(variant):
    """Nystrom of the whole space with an exact inner solve: M_1 = A_G^{-1} + R^{-1} (R^{-T} B R^{-1}) R^{-T}
    and M_3 = A_G^{-1} + A_G^{-1} A_GI S_I^{-1} A_IG A_G^{-1} both equal S^{-1} (eq. S-1), so PCG takes one
    step."""
    P = random_dbbd(4, sizes=(6, 5, 7), n_gamma=6)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    dim = d.n_gamma if variant == "M1" else d.I.size
    Om = np.random.default_rng(2).standard_normal((dim, dim))
    o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=dim, p=0, omega=Om, tol_inner=1e-15,
                           eps_rel=1e-14, variant=variant)
    o.setup()
    S = dense_schur(d)
    assert np.allclose(o.apply(np.eye(d.n_gamma)) @ S, np.eye(d.n_gamma), atol=1e-8)
    assert o.solve(P.b()).it_pcg == 1


# ---------------------------------------------------------------------------
# M_3: Nystrom of S_I^{-1} on the interior space


def test_m3_inner_forms_agree_with_dense_inverse():
    """At tight tolerance both inner forms return S_I^{-1} G = (A^{-1})_II G (shifted: through S_Gamma and
    the SMW identity with the roles of I and Gamma exchanged)."""
    P = tiny2d(N=12, sigma=1.0)
    d, B, SIinv = dense_target(P)
    G = np.random.default_rng(3).standard_normal((d.I.size, 5))
    for inner in ("shifted", "formA"):
        o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=3, p=2, omega=G, tol_inner=1e-14,
                               variant="M3", inner=inner)
        X, its, conv = o.apply_target(G)
        assert conv
        assert np.linalg.norm(X - SIinv @ G) <= 1e-10 * np.linalg.norm(SIinv @ G), inner


def test_m3_lowrank_term_and_loewner_order():
    """M_3's Z = A_G^{-1} A_GI V with V Sigma V^T the Nystrom approximation of S_I^{-1} (below S_I^{-1} in the
    Loewner order); the M_3 apply is symmetric and lies between A_G^{-1} and S^{-1}."""
    P = tiny2d(N=12, sigma=1.5)
    d, B, SIinv = dense_target(P)
    nI = d.I.size
    G = np.random.default_rng(4).standard_normal((nI, 9))
    o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=6, p=3, omega=G, tol_inner=1e-14,
                           variant="M3")
    s = o.setup()
    ev = np.sort(np.linalg.eigvalsh(SIinv))[::-1]
    assert np.all(s.Sigma <= ev[:6] * (1 + 1e-9))
    AG = d.A_G.toarray()
    assert np.allclose(s.Z, np.linalg.solve(AG, d.A_GI.toarray() @ s.U), atol=1e-12)
    M = o.apply(np.eye(d.n_gamma))
    assert np.allclose(M, M.T, atol=1e-12 * np.abs(M).max())
    S = dense_schur(d)
    lo = np.linalg.eigvalsh(M - np.linalg.inv(AG)).min()
    hi = np.linalg.eigvalsh(np.linalg.inv(S) - M).min()
    assert lo >= -1e-12 and hi >= -1e-10


@pytest.mark.parametrize("variant", ["M1", "M2", "M3"])
@pytest.mark.parametrize("mode", ["M2", "ADEF2"])
def test_variants_converge_and_beat_first_level(variant, mode):
    P = config_c1()
    om = P.omega() if variant != "M3" else np.random.default_rng(0).standard_normal(
        (int(np.count_nonzero(P.part >= 0)), P.k + P.p))
    o = make(P, variant=variant, apply_mode=mode, omega=om)
    r = o.solve(P.b(), tol=1e-8)
    assert r.converged and r.relres_true <= 1e-8
    it1 = make(P, k=0, p=0, omega=None).solve(P.b()).it_pcg
    assert r.it_pcg < it1


# ---------------------------------------------------------------------------
# power iterations (eq. power)


def test_power_iteration_closed_form():
    """q = 1 with an exact inner solve: U Sigma U^T = (B G)(G^T B G)^+ (B G)^T with G = orth(B Omega)
    (eq. NystromApprox with the sketch of eq. power), B formed densely."""
    P = tiny2d(N=14, sigma=1.5, k=4, p=3)
    d, B, _ = dense_target(P)
    Om = P.omega()
    o = make(P, tol_inner=1e-14, power=1, eps_rel=1e-14)
    s = o.setup()
    G = np.linalg.qr(B @ Om)[0]
    BG = B @ G
    C = G.T @ BG
    C = 0.5 * (C + C.T)
    ev, V = np.linalg.eigh(C)
    Cp = V @ np.diag(1.0 / ev) @ V.T
    ref = BG @ Cp @ BG.T
    Uall, Sall, r = nystrom_core(s.Y, G, P.k + P.p, 1e-14)
    assert r == P.k + P.p
    assert np.allclose(Uall @ np.diag(Sall) @ Uall.T, ref, atol=1e-9 * np.abs(ref).max())
    # the rank-k result is the leading part of it
    assert np.allclose(s.Sigma, Sall[: P.k], rtol=1e-10)


def test_power_iteration_sharpens_angles():
    """The mean over sketches of sin angle(u_j, range) falls from q = 0 to q = 1 and stays within
    gamma_{j,k}^{q+1} E(c) (eqs. bound_theta_k, constant)."""
    P = tiny2d(N=16, sigma=2.0, k=4, p=3)
    d, B, _ = dense_target(P)
    ng = d.n_gamma
    sig, V = np.linalg.eigh(B)
    sig, V = sig[::-1], V[:, ::-1]
    k, p = 4, 3
    Ec = math.sqrt(k / (p - 1)) + math.e * math.sqrt((k + p) * (ng - k)) / p
    mean = {}
    for q in (0, 1):
        sins = []
        for seed in range(20):
            Om = np.random.default_rng(50 + seed).standard_normal((ng, k + p))
            o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=k, p=p, omega=Om, tol_inner=1e-14,
                                   power=q)
            s = o.setup()
            Q = np.linalg.qr(s.Y)[0]
            sins.append(np.linalg.norm(V[:, :k] - Q @ (Q.T @ V[:, :k]), axis=0))
        mean[q] = np.mean(sins, axis=0)
        assert np.all(mean[q] <= (sig[k] / sig[:k]) ** (q + 1) * Ec)
    assert np.all(mean[1] < mean[0])


def test_power_iteration_counts_every_inner_solve():
    P = config_c1()
    s0 = make(P).setup()
    s1 = make(P, power=1).setup()
    assert s1.it_inner > s0.it_inner
    r1 = make(P, power=1).solve(P.b())
    assert r1.converged and r1.relres_true <= 1e-8
