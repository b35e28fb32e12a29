"""Plant plausible mistakes in a copy of the oracle and check that the pins catch them.

Each mutation edits the oracle's source text (a sign, a dropped term, a
transposed operand, a wrong index) and loads it as a fresh module on the CPU;
the pin checks below must then fail.  The unmodified source must pass them.
"""

import importlib.util
import os
import sys
import types

import numpy as np
import pytest
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nystrom_schur_oracle.py")

from workloads import make_problem, random_dbbd  # noqa: E402


def load_variant(old, new):
    text = open(SRC).read()
    if old is not None:
        assert text.count(old) >= 1, old
        text = text.replace(old, new, 1)
    mod = types.ModuleType("oracle_variant")
    mod.__dict__["__name__"] = "oracle_variant"
    sys.modules["oracle_variant"] = mod
    exec(compile(text, "oracle_variant", "exec"), mod.__dict__)
    return mod


def pins_pass(m):
    """A compact subset of the oracle pins, run against module ``m``."""
    ok = []
    # 1. Schur operator vs ((A^{-1})_GG)^{-1}
    P = random_dbbd(5, sizes=(8, 6, 11), n_gamma=7)
    d = m.DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    ops = m.Operators(d)
    Ainv = np.linalg.inv(P.csr().toarray())
    S_ref = np.linalg.inv(Ainv[np.ix_(d.G, d.G)])
    ok.append(np.allclose(ops.S(np.eye(d.n_gamma)), S_ref, rtol=1e-10, atol=1e-10))
    # 2. block PCG with one column is textbook PCG
    Q = make_problem((14, 14), (2, 2), sigma=1.5, ell=3.0, k=4, p=3)
    d2 = m.DBBD(Q.n, Q.row_ptr, Q.col, Q.val, Q.part)
    ops2 = m.Operators(d2)
    S = ops2.S(np.eye(d2.n_gamma))
    AGi = np.linalg.inv(d2.A_G.toarray())
    f = np.random.default_rng(3).standard_normal((d2.n_gamma, 1))
    res = m.bf_bpcg(ops2.S, ops2.solve_G, f, 0.0, 4, 1e-8)
    x_ref, _ = spla.cg(S, f[:, 0], M=AGi, maxiter=4, rtol=1e-300, atol=0.0)
    ok.append(np.allclose(res.X[:, 0], x_ref, rtol=1e-9, atol=1e-11))
    # 3. Nystrom closed form / exactness for low rank
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 5))
    B = X @ X.T
    Om = rng.standard_normal((30, 8))
    U, Sig, r = m.nystrom_core(B @ Om, Om, 10, 1e-10)
    ok.append(U.shape[1] == 5 and np.allclose(U @ np.diag(Sig) @ U.T, B, atol=1e-9 * np.abs(B).max()))
    # 4. outer PCG vs textbook, with M_2
    o = m.NystromSchurOracle(Q.n, Q.row_ptr, Q.col, Q.val, Q.part, k=4, p=3, omega=Q.omega())
    o.setup()
    M = o.apply(np.eye(d2.n_gamma))
    g = np.random.default_rng(9).standard_normal(d2.n_gamma)
    pr = m.pcg(o.ops.S, o.apply, g, 0.0, 3)
    x2, _ = spla.cg(S, g, M=M, maxiter=3, rtol=1e-300, atol=0.0)
    ok.append(np.allclose(pr.w, x2, rtol=1e-9, atol=1e-12))
    # 5. exact inverse in one iteration (Nystrom of the whole space)
    ng = d2.n_gamma
    Om2 = np.random.default_rng(5).standard_normal((ng, ng))
    o2 = m.NystromSchurOracle(Q.n, Q.row_ptr, Q.col, Q.val, Q.part, k=ng, p=0, omega=Om2, tol_inner=1e-14,
                              eps_rel=1e-14)
    o2.setup()
    ok.append(np.allclose(o2.apply(np.eye(ng)) @ S, np.eye(ng), atol=1e-8))
    # 6. full solve reaches the true residual
    sr = o.solve(Q.b(), tol=1e-8)
    ok.append(sr.relres_true <= 1e-8 and sr.relres_schur_true <= 2e-8)
    # 7. adapted deflation: the start leaves a residual orthogonal to span(Z), and M S has the eigenvalue 1
    #    k times plus the nonzero spectrum of the deflated operator in A_Gamma = R^T R coordinates
    oa = m.NystromSchurOracle(Q.n, Q.row_ptr, Q.col, Q.val, Q.part, k=4, p=3, omega=Q.omega(), apply_mode="ADEF2")
    oa.setup()
    fa = oa.reduce_rhs(Q.b())
    w0 = oa.initial_guess(fa)
    ok.append(w0 is not None and np.linalg.norm(oa.Z.T @ (fa - oa.ops.S(w0))) <= 1e-11 * np.linalg.norm(oa.Z.T @ fa))
    Rg = np.linalg.cholesky(d2.A_G.toarray()).T
    Ah = np.linalg.inv(Rg).T @ S @ np.linalg.inv(Rg)
    Zh = Rg @ oa.Z
    PD = np.eye(ng) - Ah @ Zh @ np.linalg.solve(Zh.T @ Ah @ Zh, Zh.T)
    mu = np.sort(np.linalg.eigvals(PD @ Ah).real)[4:]
    ev = np.sort(np.linalg.eigvals(oa.apply(np.eye(ng)) @ S).real)
    ok.append(np.allclose(ev, np.sort(np.concatenate([np.ones(4), mu])), rtol=1e-7, atol=1e-9))
    # 8. Nystrom eigenvalues never exceed the exact eigenvalues of B = A_G (A^{-1})_GG A_G - A_G
    Ainv2 = np.linalg.inv(Q.csr().toarray())
    AG2 = d2.A_G.toarray()
    Bx = AG2 @ Ainv2[np.ix_(d2.G, d2.G)] @ AG2 - AG2
    sig = np.sort(np.linalg.eigvalsh(0.5 * (Bx + Bx.T)))[::-1]
    ox = m.NystromSchurOracle(Q.n, Q.row_ptr, Q.col, Q.val, Q.part, k=4, p=3, omega=Q.omega(), tol_inner=1e-14)
    sx = ox.setup()
    ok.append(sx.Sigma.size == 4 and bool(np.all(sx.Sigma <= sig[:4] * (1 + 1e-9)))
              and bool(np.all(sx.Sigma >= 0.5 * sig[:4])))
    # 9. M_1 with an exact square sketch: the truncated EVD gives the ideal adapted spectrum
    T = make_problem((12, 12), (2, 2), sigma=1.5, ell=3.0, k=4, p=3)
    dT = m.DBBD(T.n, T.row_ptr, T.col, T.val, T.part)
    ngT = dT.n_gamma
    ST = m.dense_schur(dT)
    _, lamT = m.ideal_s2(dT, 5)
    o1 = m.NystromSchurOracle(T.n, T.row_ptr, T.col, T.val, T.part, k=5, p=ngT - 5,
                              omega=np.random.default_rng(5).standard_normal((ngT, ngT)), tol_inner=1e-15,
                              eps_rel=1e-14, variant="M1")
    o1.setup()
    ev1 = np.sort(np.linalg.eigvals(o1.apply(np.eye(ngT)) @ ST).real)
    ok.append(np.allclose(ev1, np.sort(np.concatenate([np.ones(5), lamT[5:]])), rtol=1e-7, atol=1e-9))
    # 10. M_3 of the whole interior space with an exact inner solve is S^{-1}
    Rd = random_dbbd(4, sizes=(6, 5, 7), n_gamma=6)
    dR = m.DBBD(Rd.n, Rd.row_ptr, Rd.col, Rd.val, Rd.part)
    nIR = dR.I.size
    o3 = m.NystromSchurOracle(Rd.n, Rd.row_ptr, Rd.col, Rd.val, Rd.part, k=nIR, p=0,
                              omega=np.random.default_rng(2).standard_normal((nIR, nIR)), tol_inner=1e-15,
                              eps_rel=1e-14, variant="M3")
    o3.setup()
    ok.append(np.allclose(o3.apply(np.eye(dR.n_gamma)) @ m.dense_schur(dR), np.eye(dR.n_gamma), atol=1e-8))
    # 11. one power iteration: the Nystrom approximation with the sketch orth(B Omega), B formed densely
    oq = m.NystromSchurOracle(T.n, T.row_ptr, T.col, T.val, T.part, k=4, p=3, omega=T.omega(), tol_inner=1e-14,
                              eps_rel=1e-14, power=1)
    sq = oq.setup()
    AinvT = np.linalg.inv(T.csr().toarray())
    AGT = dT.A_G.toarray()
    BT = AGT @ AinvT[np.ix_(dT.G, dT.G)] @ AGT - AGT
    BT = 0.5 * (BT + BT.T)
    Gq = np.linalg.qr(BT @ T.omega())[0]
    BGq = BT @ Gq
    ref = BGq @ np.linalg.pinv(0.5 * (Gq.T @ BGq + BGq.T @ Gq)) @ BGq.T
    Uq, Sq, _ = m.nystrom_core(sq.Y, Gq, 7, 1e-14)
    ok.append(np.allclose(Uq @ np.diag(Sq) @ Uq.T, ref, atol=1e-9 * np.abs(ref).max()))
    # 12. recursive level: a full-rank level-2 sketch gives the exact A_Gamma^{-1}; a low-rank one keeps the block
    #     LDL^T spectrum identity Lambda(A~^{-1} A_Gamma) = Lambda(M_J S_J) u {1}
    V = make_problem((8, 8, 8), (2, 2, 2), sigma=1.5, ell=3.0, k=4, p=2)
    dV = m.DBBD(V.n, V.row_ptr, V.col, V.val, V.part)
    nJ = int(np.count_nonzero(m.level2_part(dV) == -1))
    AGV = dV.A_G.toarray()
    rf = m.RecursiveGamma(dV, k=nJ, p=0, omega=np.random.default_rng(3).standard_normal((nJ, nJ)), tol_inner=1e-14,
                          eps_rel=1e-14)
    XV = np.random.default_rng(1).standard_normal((dV.n_gamma, 2))
    ok.append(np.allclose(rf.solve(XV), np.linalg.solve(AGV, XV), rtol=1e-9, atol=1e-11))
    rl = m.RecursiveGamma(dV, k=5, p=2, omega=np.random.default_rng(4).standard_normal((nJ, 7)))
    Mt = rl.solve(np.eye(dV.n_gamma))
    Lc = np.linalg.cholesky(0.5 * (Mt + Mt.T))
    ev = np.sort(np.linalg.eigvalsh(Lc.T @ AGV @ Lc))
    MJ = rl.inner.apply(np.eye(nJ))
    LJ = np.linalg.cholesky(0.5 * (MJ + MJ.T))
    evJ = np.sort(np.linalg.eigvalsh(LJ.T @ m.dense_schur(rl.inner.dbbd) @ LJ))
    ok.append(np.allclose(Mt, Mt.T, atol=1e-13 * np.abs(Mt).max())
              and np.allclose(ev, np.sort(np.concatenate([evJ, np.ones(dV.n_gamma - nJ)])), atol=1e-10))
    return all(ok), ok


MUTATIONS = {
    "schur_sign": ("return d.A_G @ X - d.A_GI @ self.solve_I(d.A_IG @ X)",
                   "return d.A_G @ X + d.A_GI @ self.solve_I(d.A_IG @ X)"),
    "schur_drop_AG": ("return d.A_G @ X - d.A_GI @ self.solve_I(d.A_IG @ X)",
                      "return - d.A_GI @ self.solve_I(d.A_IG @ X)"),
    "bcg_beta_sign": ("beta = -sla.cho_solve(cf, Q.T @ Z)", "beta = sla.cho_solve(cf, Q.T @ Z)"),
    "bcg_alpha_transposed": ("alpha = sla.cho_solve(cf, P.T @ R)", "alpha = sla.cho_solve(cf, Q.T @ R)"),
    "bcg_residual_update": ("R -= Q @ alpha", "R -= P @ alpha"),
    "nystrom_U_from_Y": ("U = Q @ Wm[:, order[:kk]]", "U = Y @ Wm[:, order[:kk]]"),
    "nystrom_T_no_inverse": ("T = (RV1 / D1) @ RV1.T", "T = (RV1 * D1) @ RV1.T"),
    "nystrom_ascending": ("order = np.argsort(-e, kind=\"stable\")", "order = np.argsort(e, kind=\"stable\")"),
    "nystrom_C_uses_Q": ("C = Omega.T @ Y", "C = Omega.T @ Q"),
    "pcg_beta": ("beta = rho_new / rho", "beta = rho / rho_new"),
    "pcg_alpha": ("alpha = rho / float(p @ q)", "alpha = rho / float(q @ q)"),
    "m2_drop_sigma": ("c = (self.Sigma * c.T).T if c.ndim == 2 else self.Sigma * c", "pass"),
    "reduce_sign": ("return b[d.G] - d.A_GI @ self.ops.solve_I(b[d.I])",
                    "return b[d.G] + d.A_GI @ self.ops.solve_I(b[d.I])"),
    "backsub_drop": ("xI = ops.solve_I(b[d.I] - d.A_IG @ w)", "xI = ops.solve_I(b[d.I])"),
    "interior_order": ("order = np.lexsort((interior, part[interior]))", "order = np.lexsort((part[interior], interior))"),
    "adef2_start_zero": ("return self.Z @ sla.cho_solve(self.E_cf, self.Z.T @ f)", "return None"),
    "adef2_coarse_sign": ("Z.T @ r - self.SZ.T @ t", "Z.T @ r + self.SZ.T @ t"),
    "adef2_E_without_S": ("E = self.Z.T @ self.SZ", "E = self.Z.T @ self.Z"),
    "shifted_rhs_uses_AG": ("res = bf_bpcg(ops.S, ops.solve_G, ops.W(X),", "res = bf_bpcg(ops.S, ops.solve_G, d.A_G @ X,"),
    "m1_Z_with_transpose": ("self.Z = self.Rg.solve(U)", "self.Z = self.Rg.solve_t(U)"),
    "m1_target_without_Rt": ("BX = self.Rg.solve_t(BX)", "BX = BX"),
    "m3_Z_without_coupling": ("self.Z = ops.solve_G(d.A_GI @ U)", "self.Z = d.A_GI @ U"),
    "m3_shifted_drops_interior_term": ("return ops.solve_I(G + d.A_IG @ res.X), res.iters",
                                       "return ops.solve_I(d.A_IG @ res.X), res.iters"),
    "power_keeps_first_sketch": ("            G = np.linalg.qr(Y)[0]\n", "            pass\n"),
    "Y_without_AG": ("BX = d.A_G @ res.X", "BX = res.X"),
    "rec_drops_coupling": ("yG = sub.apply(R[sd.G] - sd.A_GI @ uI)", "yG = sub.apply(R[sd.G])"),
    "rec_backsub_sign": ("zI = so.solve_I(R[sd.I] - sd.A_IG @ yG)", "zI = so.solve_I(R[sd.I] + sd.A_IG @ yG)"),
    "rec_without_low_rank": ("yG = sub.apply(R[sd.G] - sd.A_GI @ uI)", "yG = so.solve_G(R[sd.G] - sd.A_GI @ uI)"),
    "rec_backsub_from_first_solve": ("zI = so.solve_I(R[sd.I] - sd.A_IG @ yG)", "zI = uI"),
}


def test_unmodified_oracle_passes_pins():
    m = load_variant(None, None)
    passed, detail = pins_pass(m)
    assert passed, detail


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    old, new = MUTATIONS[name]
    m = load_variant(old, new)
    try:
        passed, detail = pins_pass(m)
    except Exception:
        passed = False
    assert not passed, f"mutation {name} was not detected"
