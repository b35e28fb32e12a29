"""Pins of the learned-proposal reference (oracle/learned.py) against facts
that do not come from the code itself: finite differences, invariances and
closed forms, exact eigenvectors of the pencil, and hand-computed features."""

import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import NystromSchurOracle, dense_schur
from oracle import learned as L
from workloads import config_c1, make_problem


def orthonormal(rng, n, k):
    return np.linalg.qr(rng.standard_normal((n, k)))[0]


def test_loss_closed_forms():
    rng = np.random.default_rng(0)
    U = orthonormal(rng, 40, 5)
    R = rng.standard_normal((5, 5)) + 3 * np.eye(5)
    assert L.subspace_loss(U @ R, U) == pytest.approx(0.0, abs=1e-12)  # same span
    V = rng.standard_normal((40, 5))
    V -= U @ (U.T @ V)  # orthogonal complement
    assert L.subspace_loss(V, U) == pytest.approx(1.0, abs=1e-12)
    Z = rng.standard_normal((40, 5))
    l0 = L.subspace_loss(Z, U)
    assert 0.0 <= l0 <= 1.0
    assert L.subspace_loss(Z @ R, U) == pytest.approx(l0, rel=1e-10)  # depends on span(Z0) only
    # half of the subspace captured: L = 1/2 for Z0 = [u1 u2 v v] style construction
    Zh = np.hstack([U[:, :2], V[:, :3]])
    Uh = U[:, :4]
    assert L.subspace_loss(Zh, Uh) == pytest.approx(1.0 - 2.0 / 4.0, abs=1e-12)


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    U = orthonormal(rng, 30, 4)
    Z = rng.standard_normal((30, 4))
    g = L.subspace_loss_grad(Z, U)
    h = 1e-6
    num = np.zeros_like(Z)
    for i in range(Z.shape[0]):
        for j in range(Z.shape[1]):
            E = np.zeros_like(Z)
            E[i, j] = h
            num[i, j] = (L.subspace_loss(Z + E, U) - L.subspace_loss(Z - E, U)) / (2 * h)
    assert np.max(np.abs(num - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))
    # a gradient step lowers the loss
    assert L.subspace_loss(Z - 0.1 * g / np.linalg.norm(g), U) < L.subspace_loss(Z, U)


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = L.mlp_init(6, 9, 3, seed=3)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((11, 6))
    C = rng.standard_normal((11, 3))
    f = lambda q: float(np.sum(L.mlp_forward(q, X)[0] * C))  # noqa: E731
    Z0, cache = L.mlp_forward(p, X)
    g = L.mlp_backward(p, cache, C)
    h = 1e-6
    for name in L.PARAM_ORDER:
        num = np.zeros_like(p[name])
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += h
            fp = f(q)
            q[name][idx] -= 2 * h
            fm = f(q)
            num[idx] = (fp - fm) / (2 * h)
        assert np.max(np.abs(num - g[name])) <= 1e-6 * max(1.0, np.max(np.abs(num))), name


def test_flatten_roundtrip():
    p = L.mlp_init(4, 5, 2, seed=0)
    v = L.flatten(p)
    assert v.size == 4 * 5 + 5 + 25 + 5 + 5 * 2 + 2
    q = L.unflatten(v, 4, 5, 2)
    for k in L.PARAM_ORDER:
        assert np.array_equal(p[k], q[k])


def _pencil(P):
    orc = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=0, p=0, omega=None)
    d = orc.dbbd
    S = dense_schur(d)
    AG = d.A_G.toarray()
    return orc, d, S, AG


def test_rayleigh_ritz_on_exact_eigenvectors():
    P = config_c1()
    orc, d, S, AG = _pencil(P)
    lam, V = sla.eigh(S, AG)  # ascending, lambda in (0, 1]
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-10
    k = 6
    R = np.random.default_rng(4).standard_normal((k, k)) + 2 * np.eye(k)
    Z = V[:, :k] @ R  # any basis of the exact invariant subspace
    lr, Y, rho = L.rayleigh_ritz(lambda X: S @ X, lambda X: AG @ X, Z)
    assert np.allclose(lr, lam[:k], rtol=1e-10, atol=1e-13)
    assert np.max(rho) <= 1e-9
    assert np.allclose(Y.T @ AG @ Y, np.eye(k), atol=1e-9)  # A_Gamma-orthonormal Ritz vectors
    assert L.accept(rho, k, 0.2)
    # a random subspace is rejected
    Zr = np.random.default_rng(5).standard_normal((d.n_gamma, k))
    _, _, rho_r = L.rayleigh_ritz(lambda X: S @ X, lambda X: AG @ X, Zr)
    assert not L.accept(rho_r, k, 0.2)


def test_oracle_accepted_proposal_is_exact_deflation():
    """An accepted proposal spanning A_Gamma times the exact smallest eigenvectors deflates them: PCG with
    the adapted deflation converges in no more iterations than the first-level preconditioner, and the
    proposal path skips the inner solve."""
    P = config_c1()
    orc, d, S, AG = _pencil(P)
    lam, V = sla.eigh(S, AG)
    k = 10
    Z0 = AG @ V[:, :k]  # so that A_Gamma^{-1} Z0 spans the eigenvectors
    b = P.b()
    o1 = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=k, p=2, omega=P.omega()[:, :k + 2],
                            proposal=Z0)
    r1 = o1.setup()
    assert r1.proposal_accepted and r1.it_inner == 0
    s1 = o1.solve(b)
    s0 = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=0, p=0, omega=None).solve(b)
    assert s1.converged and s1.relres_true <= 1e-7
    assert s1.it_pcg < s0.it_pcg


def test_oracle_rejected_proposal_falls_back_to_plain():
    P = config_c1()
    Z0 = np.random.default_rng(6).standard_normal((127, P.k))
    o1 = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=P.k, p=P.p, omega=P.omega(), proposal=Z0)
    o0 = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=P.k, p=P.p, omega=P.omega())
    r1, r0 = o1.setup(), o0.setup()
    assert not r1.proposal_accepted
    assert r1.it_inner == r0.it_inner
    assert np.array_equal(r1.Z, r0.Z) and np.array_equal(r1.Sigma, r0.Sigma)


def test_features_hand_computed():
    """A 4-node path 0-1-2-3 with node 0 in subdomain 0, nodes 1, 2 interface (1 a junction), 3 in
    subdomain 1; the features follow from the definitions by hand."""
    rows = [0, 0, 1, 1, 1, 2, 2, 2, 3, 3]
    cols = [0, 1, 0, 1, 2, 1, 2, 3, 2, 3]
    vals = [4.0, -1.0, -1.0, 5.0, -2.0, -2.0, 6.0, -3.0, -3.0, 7.0]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(4, 4))
    part = np.array([0, -1, -2, 1], dtype=np.int32)
    coords = np.arange(12, dtype=float).reshape(4, 3)
    F = L.interface_features(4, A.indptr, A.indices, A.data, part, coords)
    assert F.shape == (2, 16)
    f1 = F[0]  # node 1: neighbours 0 (interior, |a|=1) and 2 (interface, |a|=2)
    assert np.allclose(f1[0:3], coords[1])
    assert f1[3] == pytest.approx(math.log(5.0))
    assert f1[4] == pytest.approx((math.log(1.0) + math.log(2.0)) / 2)
    assert f1[5] == pytest.approx(0.0) and f1[6] == pytest.approx(math.log(2.0))
    assert f1[7] == pytest.approx(math.log(1.0 + 1e-30)) and f1[8] == pytest.approx(math.log(2.0))
    assert f1[9] == 1.0 and f1[10] == 0.25 and f1[14] == 0.125 and f1[15] == 1.0
    f2 = F[1]  # node 2: neighbours 1 (interface, 2) and 3 (interior of subdomain 1, 3)
    assert f2[9] == 0.0 and f2[10] == 0.25
    s1 = [(math.log(5) + math.log(6)) / 2] * 2  # each has one interface neighbour
    assert F[0, 11] == pytest.approx(s1[0]) and F[1, 11] == pytest.approx(s1[1])
    assert F[0, 13] == pytest.approx(s1[0])  # constant after the first averaging


def test_features_of_grid_problem_are_finite():
    P = make_problem((20, 20), (2, 2), sigma=1.0, ell=4.0, k=4, p=2)
    F = L.interface_features(P.n, P.row_ptr, P.col, P.val, P.part)
    assert F.shape == (P.n_gamma, L.D_IN) and np.all(np.isfinite(F))
