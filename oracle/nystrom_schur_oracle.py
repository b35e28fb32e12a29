"""FP64 CPU oracle: DBBD split, Schur operator, block PCG, Nystrom, M_2, PCG.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every routine is the
plain definition or the paper's algorithm step by step, in float64, with
NumPy / SciPy dense and sparse primitives as the only building blocks.  There
is no blocking, fusion or reordering beyond what the definitions state.

Readings taken where the paper is silent (each is repeated in the design
notes of the repository):

* inner solve: block PCG on the shifted system S_Gamma D = W Omega with
  W = A_GammaI A_I^{-1} A_IGamma, preconditioned by A_Gamma^{-1}; then
  Y = A_Gamma D.  By eq. (S-1) this Y equals A_GammaI S_I^{-1} A_IGamma Omega,
  the product of Algorithm alg:prec1 steps 2-4 (``inner='formA'`` runs
  those steps literally).
* block stopping rule: max over columns of ||R_j|| / ||F_j|| <= eps_SI.
* breakdown-free orthonormalisation: thin SVD, keep sigma_i > delta*sigma_max
  with delta = 1e-6 (the drop tolerance of Ji & Li's method is not given).
* Nystrom threshold: eigenvalues of sym(Omega^T Y) >= eps_rel * max eigenvalue.
* Algorithm alg:prec1 step 10 reads U = Q W(:, 1:k) (Q from the QR of Y, as in
  Algorithm alg:nystrom); eigenvalues of T sorted descending; k' = min(k, r).
* outer PCG: recurrence residual ||r_j|| / ||f|| <= tol, w_0 = 0 for M_2 and
  w_0 = Z E^{-1} Z^T f for the adapted-deflation form.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ----------------------------------------------------------------------------
# doubly bordered block diagonal split  (eq. perm_A)


class DBBD:
    """Index sets and blocks of P^T A P = [[A_I, A_IG], [A_GI, A_G]] (eq. perm_A).

    Interior nodes (part >= 0) are ordered by (subdomain, original index);
    interface nodes (part < 0) by original index.  A_I must be block diagonal
    (no coupling between distinct subdomains) and A symmetric.
    """

    def __init__(self, n, row_ptr, col, val, part):
        A = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))
        part = np.asarray(part).astype(np.int64)
        if part.shape != (n,):
            raise ValueError("part must have length n")
        asym = A - A.T
        if asym.nnz and np.max(np.abs(asym.data)) != 0.0:
            raise ValueError("A is not symmetric")
        interior = np.nonzero(part >= 0)[0]
        order = np.lexsort((interior, part[interior]))
        self.I = interior[order]
        self.G = np.nonzero(part < 0)[0]
        coo = A.tocoo()
        pi, pj = part[coo.row], part[coo.col]
        cross = (pi >= 0) & (pj >= 0) & (pi != pj) & (coo.data != 0)
        if np.any(cross):
            raise ValueError("A couples interior nodes of different subdomains: not DBBD")
        self.A = A.tocsr()
        self.part = part
        nsub = int(part.max()) + 1 if interior.size else 0
        counts = np.bincount(part[interior], minlength=nsub) if nsub else np.zeros(0, dtype=np.int64)
        self.block_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        AI = self.A[self.I]
        AG = self.A[self.G]
        self.A_I = AI[:, self.I].tocsr()
        self.A_IG = AI[:, self.G].tocsr()
        self.A_GI = AG[:, self.I].tocsr()
        self.A_G = AG[:, self.G].tocsr()

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def n_gamma(self):
        return self.G.size

    @property
    def n_sub(self):
        return self.block_ptr.size - 1

    def block(self, j):
        a, b = self.block_ptr[j], self.block_ptr[j + 1]
        return self.A_I[a:b, a:b]


# ----------------------------------------------------------------------------
# exact solves with A_I (block diagonal) and A_Gamma


class Operators:
    """A_I^{-1}, A_Gamma^{-1}, the Schur operator S_Gamma and W.

    A_I^{-1}: one Cholesky factor per diagonal block (the blocks are independent
    of each other, so each is factorised on its own).  A_Gamma^{-1}:
    exact, assumed available by eq. (S1).  ``factor='dense'`` uses LAPACK
    Cholesky on dense blocks; ``'sparse'`` uses SuperLU (same result up to
    rounding, for sizes where dense copies do not fit in host memory).
    """

    def __init__(self, dbbd: DBBD, factor: str = "dense", gamma_factor: Optional[str] = None,
                 gamma_solve: Optional[Callable] = None):
        self.d = dbbd
        self.factor = factor
        self._gamma_solve = gamma_solve  # an approximate A_Gamma^{-1} (the recursive level), else exact
        self._blk = []
        for j in range(dbbd.n_sub):
            Aj = dbbd.block(j)
            if factor == "dense":
                L = sla.cholesky(Aj.toarray(), lower=True)
                self._blk.append(("dense", L))
            else:
                self._blk.append(("sparse", spla.splu(Aj.tocsc())))
        gf = gamma_factor or ("dense" if dbbd.n_gamma <= 6000 else "sparse")
        if gamma_solve is not None:
            self._g = ("given", None)
        elif dbbd.n_gamma == 0:
            self._g = ("none", None)
        elif gf == "dense":
            self._g = ("dense", sla.cholesky(dbbd.A_G.toarray(), lower=True))
        else:
            self._g = ("sparse", spla.splu(dbbd.A_G.tocsc()))

    def block_factor(self, j):
        kind, F = self._blk[j]
        if kind != "dense":
            raise ValueError("dense factor not available")
        return F

    def solve_I(self, X):
        """A_I^{-1} X, block by block."""
        X = np.asarray(X, dtype=np.float64)
        out = np.empty_like(X)
        bp = self.d.block_ptr
        for j, (kind, F) in enumerate(self._blk):
            a, b = bp[j], bp[j + 1]
            if kind == "dense":
                out[a:b] = sla.cho_solve((F, True), X[a:b])
            else:
                out[a:b] = F.solve(np.ascontiguousarray(X[a:b]))
        return out

    def solve_G(self, X):
        """A_Gamma^{-1} X (the first-level preconditioner of eq. S1)."""
        X = np.asarray(X, dtype=np.float64)
        kind, F = self._g
        if kind == "given":
            return self._gamma_solve(X)
        if kind == "none":
            return X.copy()
        if kind == "dense":
            return sla.cho_solve((F, True), X)
        return F.solve(np.ascontiguousarray(X))

    def S(self, X):
        """S_Gamma X = A_Gamma X - A_GammaI A_I^{-1} A_IGamma X  (eq. schur_complement)."""
        d = self.d
        return d.A_G @ X - d.A_GI @ self.solve_I(d.A_IG @ X)

    def W(self, X):
        """W X = A_GammaI A_I^{-1} A_IGamma X = (A_Gamma - S_Gamma) X."""
        d = self.d
        return d.A_GI @ self.solve_I(d.A_IG @ X)

    def S_I(self, X):
        """S_I X = A_I X - A_IGamma A_Gamma^{-1} A_GammaI X  (eq. SI)."""
        d = self.d
        return d.A_I @ X - d.A_IG @ self.solve_G(d.A_GI @ X)


# ----------------------------------------------------------------------------
# a factor R_Gamma with A_Gamma = R_Gamma^T R_Gamma  (eq. cholesky), for the variant M_1


def level2_order(d: DBBD):
    """Interface positions in the order of the level-2 split of A_Gamma: the nodes of each separator block
    (label -2 - b for block b; blocks in label order, nodes by interface index), then the junction nodes
    (label -1) by interface index.  Without level-2 labels this is the interface order itself."""
    pg = d.part[d.G]
    blk = np.where(pg <= -2, -2 - pg, np.iinfo(np.int64).max)
    return np.lexsort((np.arange(d.n_gamma), blk))


class GammaFactor:
    """R_Gamma = P^T L^T P: L the Cholesky factor of A_Gamma with rows and columns in the level-2 order
    ((P x) = x[perm]), so that A_Gamma = R^T R with the rows of R labelled, like its columns and like the
    sketch, by interface index.  Any R with R^T R = A_Gamma serves the derivation of M_1 (eq. cholesky); this
    one is the factor the level-2 block LDL^T of A_Gamma defines.  Dense (small interfaces only)."""

    def __init__(self, d: DBBD, max_dense: int = 8000):
        if d.n_gamma > max_dense:
            raise ValueError("GammaFactor: interface too large for a dense factor")
        self.perm = level2_order(d)
        AG = d.A_G.toarray()
        self.L = sla.cholesky(AG[np.ix_(self.perm, self.perm)], lower=True)

    def _unperm(self, u):
        out = np.empty_like(u)
        out[self.perm] = u
        return out

    def mult(self, X):
        """R X = P^T L^T (P X)."""
        return self._unperm(self.L.T @ np.asarray(X)[self.perm])

    def solve(self, Y):
        """R^{-1} Y = P^T L^{-T} (P Y)."""
        return self._unperm(sla.solve_triangular(self.L, np.asarray(Y)[self.perm], lower=True, trans="T"))

    def solve_t(self, Y):
        """R^{-T} Y = P^T L^{-1} (P Y)."""
        return self._unperm(sla.solve_triangular(self.L, np.asarray(Y)[self.perm], lower=True))


# ----------------------------------------------------------------------------
# the recursive (multilevel) construction: A_Gamma^{-1} replaced by a Nystrom-Schur preconditioner one level down


def level2_part(d: DBBD):
    """Labels that make A_Gamma a DBBD matrix of its own: separator block b (label -2 - b) -> subdomain b, junction
    node (label -1) -> interface.  Rows and columns of A_Gamma keep the interface order."""
    pg = d.part[d.G]
    return np.where(pg <= -2, -2 - pg, -1).astype(np.int32)


class RecursiveGamma:
    """Approximate A_Gamma^{-1} of the recursive construction the conclusions name as future work (with the
    reading of the design notes): A_Gamma, split by the level-2 labels (separator blocks = its interior s,
    junction nodes = its interface J), is preconditioned exactly as A is -- the block LDL^T solve of eq. A_LDLT
    with the inverse of its Schur complement S_J = A_J - A_Js A_s^{-1} A_sJ replaced by the Nystrom-Schur
    preconditioner M_J of S_J (eq. left_prec_mat one level down: sketch ``omega`` of n_J x (k + p), inner
    block solve preconditioned by A_J^{-1}):

        u_s = A_s^{-1} r_s,   y_J = M_J (r_J - A_Js u_s),   z_s = A_s^{-1} (r_s - A_sJ y_J),   z_J = y_J,

    the preconditioner M^{-1} of the Schur-complement section applied to A_Gamma.  Only the separator blocks and
    A_J are factorised.  ``k = 0`` gives M_J = A_J^{-1}."""

    def __init__(self, d: DBBD, *, k, p, omega, tol_inner=0.1, eps_rel=1e-10, delta=1e-6, maxit_inner=500,
                 factor="dense"):
        part2 = level2_part(d)
        if not np.any(part2 == -1):
            raise ValueError("RecursiveGamma: the level-2 split has no junction nodes")
        if not np.any(part2 >= 0):
            raise ValueError("RecursiveGamma: the level-2 split has no separator blocks")
        AG = sp.csr_matrix(d.A_G)
        AG.sort_indices()
        self.inner = NystromSchurOracle(d.n_gamma, AG.indptr, AG.indices, AG.data, part2, k=k, p=p, omega=omega,
                                        tol_inner=tol_inner, eps_rel=eps_rel, delta=delta, maxit_inner=maxit_inner,
                                        factor=factor)
        self.setup_result = self.inner.setup()

    def solve(self, R):
        """Approximate A_Gamma^{-1} R (interface order, one vector or a block of columns)."""
        sub = self.inner
        sd, so = sub.dbbd, sub.ops
        R = np.asarray(R, dtype=np.float64)
        uI = so.solve_I(R[sd.I])
        yG = sub.apply(R[sd.G] - sd.A_GI @ uI)
        zI = so.solve_I(R[sd.I] - sd.A_IG @ yG)
        out = np.empty_like(R)
        out[sd.I] = zI
        out[sd.G] = yG
        return out


# ----------------------------------------------------------------------------
# breakdown-free block PCG  (block CG of O'Leary with the rank-revealing
# orthonormalisation of Ji & Li, the inner solver of the numerical section)


def orth(V, delta):
    """Orthonormal basis of range(V): thin SVD, keep sigma_i > delta * sigma_1."""
    V = np.asarray(V, dtype=np.float64)
    if V.shape[1] == 0:
        return V.copy()
    U, s, _ = np.linalg.svd(V, full_matrices=False)
    if s.size == 0 or not s[0] > 0.0:
        return V[:, :0].copy()
    r = int(np.count_nonzero(s > delta * s[0]))
    return U[:, :r]


@dataclasses.dataclass
class BCGResult:
    X: np.ndarray
    iters: int
    converged: bool
    relres: float
    widths: list


def _col_relres(R, nF):
    nr = np.linalg.norm(R, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(nF > 0, nr / np.where(nF > 0, nF, 1.0), 0.0)
    return float(rel.max()) if rel.size else 0.0


def bf_bpcg(Sop: Callable, Mop: Callable, F, tol: float, maxit: int, delta: float = 1e-6) -> BCGResult:
    """Block PCG for S X = F with preconditioner M, from X_0 = 0.

    P_0 = orth(M R_0); per iteration Q = S P, Delta = P^T Q,
    alpha = Delta^{-1} P^T R, X += P alpha, R -= Q alpha, stop when the largest
    column relative residual is <= tol, then Z = M R,
    beta = -Delta^{-1} Q^T Z, P = orth(Z + P beta).
    """
    F = np.asarray(F, dtype=np.float64)
    X = np.zeros_like(F)
    R = F.copy()
    nF = np.linalg.norm(F, axis=0)
    rel = _col_relres(R, nF)
    widths = []
    if rel <= tol:
        return BCGResult(X, 0, True, rel, widths)
    P = orth(Mop(R), delta)
    for it in range(1, maxit + 1):
        widths.append(P.shape[1])
        if P.shape[1] == 0:
            return BCGResult(X, it - 1, False, rel, widths)
        Q = Sop(P)
        Delta = P.T @ Q
        Delta = 0.5 * (Delta + Delta.T)
        cf = sla.cho_factor(Delta, lower=True)
        alpha = sla.cho_solve(cf, P.T @ R)
        X += P @ alpha
        R -= Q @ alpha
        rel = _col_relres(R, nF)
        if rel <= tol:
            return BCGResult(X, it, True, rel, widths)
        Z = Mop(R)
        beta = -sla.cho_solve(cf, Q.T @ Z)
        P = orth(Z + P @ beta, delta)
    return BCGResult(X, maxit, False, rel, widths)


# ----------------------------------------------------------------------------
# Nystrom core: Algorithm alg:nystrom steps 3-8 / Algorithm alg:prec1 steps 5-10


def nystrom_core(Y, Omega, k, eps_rel=1e-10):
    """Rank-k' Nystrom factors (U, Sigma) of B from Y = B Omega.

    QR of Y; C = Omega^T Y (symmetrised); EVD of C, keep eigenvalues
    >= eps_rel * max (V_1, D_1, rank r); T = (R V_1) D_1^{-1} (R V_1)^T; EVD of
    T sorted descending; U = Q W(:, 1:k'), Sigma = E(1:k'), k' = min(k, r).
    """
    Y = np.asarray(Y, dtype=np.float64)
    Q, R = np.linalg.qr(Y)
    C = Omega.T @ Y
    C = 0.5 * (C + C.T)
    d, V = np.linalg.eigh(C)
    if d.size == 0 or not d.max() > 0.0:
        return Q[:, :0], np.zeros(0), 0
    keep = d >= eps_rel * d.max()
    V1, D1 = V[:, keep], d[keep]
    r = int(D1.size)
    RV1 = R @ V1
    T = (RV1 / D1) @ RV1.T
    T = 0.5 * (T + T.T)
    e, Wm = np.linalg.eigh(T)
    order = np.argsort(-e, kind="stable")
    kk = min(int(k), r)
    U = Q @ Wm[:, order[:kk]]
    return U, e[order[:kk]], r


# ----------------------------------------------------------------------------
# PCG on S_Gamma w = f  (eq. Sx=b)


@dataclasses.dataclass
class PCGResult:
    w: np.ndarray
    iters: int
    converged: bool
    hist: list


def pcg(Sop: Callable, Mop: Callable, f, tol: float, maxit: int, w0=None, callback=None) -> PCGResult:
    """Preconditioned CG (Hestenes-Stiefel); stops on ||r_j|| / ||f|| <= tol.

    ``iters`` counts applications of S inside the loop; ``callback(w)`` sees
    every iterate.
    """
    f = np.asarray(f, dtype=np.float64)
    nf = float(np.linalg.norm(f))
    if w0 is None:
        w = np.zeros_like(f)
        r = f.copy()
    else:
        w = np.array(w0, dtype=np.float64)
        r = f - Sop(w)
    if nf == 0.0:
        return PCGResult(np.zeros_like(f), 0, True, [0.0])
    hist = [float(np.linalg.norm(r)) / nf]
    if hist[0] <= tol:
        return PCGResult(w, 0, True, hist)
    z = Mop(r)
    p = z.copy()
    rho = float(r @ z)
    for it in range(1, maxit + 1):
        q = Sop(p)
        alpha = rho / float(p @ q)
        w = w + alpha * p
        r = r - alpha * q
        if callback is not None:
            callback(w)
        hist.append(float(np.linalg.norm(r)) / nf)
        if hist[-1] <= tol:
            return PCGResult(w, it, True, hist)
        z = Mop(r)
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return PCGResult(w, maxit, False, hist)


# ----------------------------------------------------------------------------
# the whole method


@dataclasses.dataclass
class SetupResult:
    it_inner: int
    inner_converged: bool
    k_eff: int
    rank_C: int
    U: np.ndarray
    Sigma: np.ndarray
    Z: np.ndarray
    Y: np.ndarray
    proposal_accepted: bool = False
    ritz_rho: Optional[np.ndarray] = None


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    w: np.ndarray
    it_pcg: int
    converged: bool
    relres_schur: float
    relres_schur_true: float
    relres_true: float
    hist: list


class NystromSchurOracle:
    """Algorithm alg:prec1 plus the block LDL^T solve of eq. A_LDLT.

    ``variant`` picks the matrix Nystrom approximates and how Z is formed:
      'M2': B = A_GammaI S_I^{-1} A_IGamma (eq. internal_term_lr_approximation_1),
            Z = A_Gamma^{-1} U (eq. left_prec_mat, the preconditioner of the experiments);
      'M1': R_Gamma^{-T} B R_Gamma^{-1} (eq. lr_approximation_S-1_A-I), Z = R_Gamma^{-1} U (eq. prec1S);
      'M3': S_I^{-1} on the interior space (eq. internal_term_lr_approximation_2; the sketch ``omega`` is
            then n_I x (k+p) in interior order), Z = A_Gamma^{-1} A_GammaI U (eq. left_prec_mat2).
    ``apply_mode``: 'M2' -- the additive low-rank form A_Gamma^{-1} + Z Sigma Z^T of the variant (M_1, M_2
    or M_3) -- or 'ADEF2' -- the adapted deflation built from the variant's Z (eqs. adapted_deflation_prec,
    deflation_comp_from_low_rank, our_two_level_preconditioner: M_1A-DEF, M_2A-DEF, M_3A-DEF).
    ``inner``: 'shifted' (systems with S_Gamma, preconditioned by A_Gamma^{-1}) or 'formA' (S_I X = F,
    preconditioned by A_I^{-1}, the literal step 3).
    ``power``: q of eq. power -- the sketch is B^q Omega, orthonormalised (QR) after every product with B.
    ``k = 0`` gives the first-level preconditioner S_1.
    ``level2``: None -- A_Gamma^{-1} exact (eq. S1) -- or dict(k=, p=, omega=, tol_inner=) -- every solve with
    A_Gamma uses the recursive approximation of ``RecursiveGamma`` built with those parameters (its tolerance
    defaults to ``tol_inner``); not with 'M1', which needs an exact factor of A_Gamma.
    """

    def __init__(self, n, row_ptr, col, val, part, *, k, p, omega, tol_inner=0.1, eps_rel=1e-10, delta=1e-6,
                 maxit_inner=500, factor="dense", apply_mode="M2", inner="shifted", gamma_factor=None,
                 proposal=None, accept_tol=0.2, variant="M2", power=0, level2=None):
        self.dbbd = DBBD(n, row_ptr, col, val, part)
        self.level2 = None
        if level2 is not None:
            if variant == "M1":
                raise ValueError("variant M1 needs an exact factor of A_Gamma (no recursive level)")
            l2 = dict(level2)
            l2.setdefault("tol_inner", tol_inner)
            self.level2 = RecursiveGamma(self.dbbd, factor=factor, eps_rel=eps_rel, delta=delta, **l2)
        self.ops = Operators(self.dbbd, factor=factor, gamma_factor=gamma_factor,
                             gamma_solve=self.level2.solve if self.level2 is not None else None)
        self.k, self.p = int(k), int(p)
        self.omega = np.asarray(omega, dtype=np.float64) if omega is not None else None
        self.tol_inner = tol_inner
        self.eps_rel = eps_rel
        self.delta = delta
        self.maxit_inner = maxit_inner
        self.apply_mode = apply_mode
        self.inner = inner
        self.proposal = np.asarray(proposal, dtype=np.float64) if proposal is not None else None
        self.accept_tol = accept_tol
        if variant not in ("M1", "M2", "M3"):
            raise ValueError(variant)
        if inner not in ("shifted", "formA"):
            raise ValueError(inner)
        self.variant = variant
        self.power = int(power)
        self.setup_result: Optional[SetupResult] = None
        self.Rg = GammaFactor(self.dbbd) if variant == "M1" and self.k > 0 else None

    # -- Algorithm alg:prec1 ------------------------------------------------
    def setup(self) -> SetupResult:
        ops, d = self.ops, self.dbbd
        if self.k == 0:
            ng = d.n_gamma
            self.Z = np.zeros((ng, 0))
            self.Sigma = np.zeros(0)
            self.setup_result = SetupResult(0, True, 0, 0, np.zeros((ng, 0)), self.Sigma, self.Z, np.zeros((ng, 0)))
            self._post_setup()
            return self.setup_result
        rho = None
        if self.proposal is not None:
            # learned starting subspace: Z = A_Gamma^{-1} Z0, judged by Rayleigh-Ritz on (S_Gamma, A_Gamma);
            # accepted -> adapted deflation with the Ritz vectors (eqs. adapted_deflation_prec,
            # deflation_comp_from_low_rank), rejected -> plain Nystrom below
            from .learned import accept, rayleigh_ritz

            Zp = ops.solve_G(self.proposal)
            lam, Yr, rho = rayleigh_ritz(ops.S, lambda X: d.A_G @ X, Zp)
            if accept(rho, self.k, self.accept_tol):
                self.apply_mode = "ADEF2"
                self.Z = Yr
                self.Sigma = np.zeros(Yr.shape[1])
                ng = d.n_gamma
                self.setup_result = SetupResult(0, True, Yr.shape[1], 0, np.zeros((ng, 0)), self.Sigma, self.Z,
                                                np.zeros((ng, 0)), True, rho)
                self._post_setup()
                return self.setup_result
        # sketch G = B^q Omega (eq. power), orthonormalised after every product, then Y = B G
        G = self.omega
        Y, its, conv = self.apply_target(G)
        for _ in range(self.power):
            G = np.linalg.qr(Y)[0]
            Y, it2, c2 = self.apply_target(G)
            its += it2
            conv = conv and c2
        U, Sig, r = nystrom_core(Y, G, self.k, self.eps_rel)
        if self.variant == "M2":
            self.Z = ops.solve_G(U)
        elif self.variant == "M1":
            self.Z = self.Rg.solve(U)
        else:
            self.Z = ops.solve_G(d.A_GI @ U)
        self.Sigma = Sig
        self.setup_result = SetupResult(its, conv, U.shape[1], r, U, Sig, self.Z, Y, False, rho)
        self._post_setup()
        return self.setup_result

    def apply_target(self, G):
        """B G for the variant's Nystrom target B, through the inner block solve (Algorithm alg:prec1
        steps 2-4); returns (B G, inner iterations, converged)."""
        ops, d = self.ops, self.dbbd
        if self.variant == "M3":
            # S_I^{-1} G.  formA: S_I X = G, preconditioned by A_I^{-1}.  shifted: by SMW,
            # S_I^{-1} = A_I^{-1} + A_I^{-1} A_IGamma S_Gamma^{-1} A_GammaI A_I^{-1}, so
            # X = A_I^{-1} (G + A_IGamma D) with S_Gamma D = A_GammaI A_I^{-1} G.
            if self.inner == "formA":
                res = bf_bpcg(ops.S_I, ops.solve_I, G, self.tol_inner, self.maxit_inner, self.delta)
                return res.X, res.iters, res.converged
            F = d.A_GI @ ops.solve_I(G)
            res = bf_bpcg(ops.S, ops.solve_G, F, self.tol_inner, self.maxit_inner, self.delta)
            return ops.solve_I(G + d.A_IG @ res.X), res.iters, res.converged
        X = self.Rg.solve(G) if self.variant == "M1" else G
        if self.inner == "shifted":
            # S_Gamma D = W X preconditioned by A_Gamma^{-1}; B X = A_Gamma D (eq. S-1)
            res = bf_bpcg(ops.S, ops.solve_G, ops.W(X), self.tol_inner, self.maxit_inner, self.delta)
            BX = d.A_G @ res.X
        else:
            res = bf_bpcg(ops.S_I, ops.solve_I, d.A_IG @ X, self.tol_inner, self.maxit_inner, self.delta)
            BX = d.A_GI @ res.X
        if self.variant == "M1":
            BX = self.Rg.solve_t(BX)
        return BX, res.iters, res.converged

    def _post_setup(self):
        if self.apply_mode == "ADEF2" and self.Z.shape[1] > 0:
            self.SZ = self.ops.S(self.Z)
            E = self.Z.T @ self.SZ
            self.E_cf = sla.cho_factor(0.5 * (E + E.T), lower=True)

    # -- preconditioner application (Algorithm alg:prec1 step 12) ------------
    def apply(self, r):
        """z = M r for one vector or a block of columns."""
        ops = self.ops
        t = ops.solve_G(r)
        Z = self.Z
        if Z.shape[1] == 0:
            return t
        if self.apply_mode == "M2":
            c = Z.T @ r
            c = (self.Sigma * c.T).T if c.ndim == 2 else self.Sigma * c
            return t + Z @ c
        # adapted deflation: t + Z E^{-1} (Z^T r - (S Z)^T t)
        return t + Z @ sla.cho_solve(self.E_cf, Z.T @ r - self.SZ.T @ t)

    def initial_guess(self, f):
        if self.apply_mode == "ADEF2" and self.Z.shape[1] > 0:
            return self.Z @ sla.cho_solve(self.E_cf, self.Z.T @ f)
        return None

    # -- block LDL^T solve of A x = b (eq. A_LDLT, eq. Sx=b) -----------------
    def reduce_rhs(self, b):
        """f = b_Gamma - A_GammaI A_I^{-1} b_I."""
        d = self.dbbd
        return b[d.G] - d.A_GI @ self.ops.solve_I(b[d.I])

    def solve(self, b, tol=1e-8, maxit=1000) -> SolveResult:
        if self.setup_result is None:
            self.setup()
        d, ops = self.dbbd, self.ops
        b = np.asarray(b, dtype=np.float64)
        f = self.reduce_rhs(b)
        res = pcg(ops.S, self.apply, f, tol, maxit, w0=self.initial_guess(f))
        w = res.w
        xI = ops.solve_I(b[d.I] - d.A_IG @ w)
        x = np.empty(d.n)
        x[d.I] = xI
        x[d.G] = w
        nb = float(np.linalg.norm(b))
        nf = float(np.linalg.norm(f))
        rt = float(np.linalg.norm(b - d.A @ x)) / nb if nb > 0 else 0.0
        rs = float(np.linalg.norm(f - ops.S(w))) / nf if nf > 0 else 0.0
        return SolveResult(x, w, res.iters, res.converged, res.hist[-1], rs, rt, res.hist)


# ----------------------------------------------------------------------------
# dense references for tiny inputs


def dense_schur(d: DBBD):
    """Explicit S_Gamma = A_Gamma - A_GammaI A_I^{-1} A_IGamma (dense)."""
    AI = d.A_I.toarray()
    return d.A_G.toarray() - d.A_GI.toarray() @ np.linalg.solve(AI, d.A_IG.toarray())


def ideal_s2(d: DBBD, k: int):
    """Ideal second-level preconditioner of eq. S2 from the exact GEVP S z = lambda A_Gamma z.

    Returns (apply, lam) with apply(r) = A_Gamma^{-1} r + Z_k (Lambda_k^{-1} - I) Z_k^T r,
    Z_k the A_Gamma-orthonormal eigenvectors of the k smallest eigenvalues.
    """
    S = dense_schur(d)
    AG = d.A_G.toarray()
    lam, Zf = sla.eigh(S, AG)
    Zk, lk = Zf[:, :k], lam[:k]
    cf = sla.cho_factor(AG, lower=True)

    def apply(r):
        c = Zk.T @ r
        c = ((1.0 / lk - 1.0) * c.T).T if c.ndim == 2 else (1.0 / lk - 1.0) * c
        return sla.cho_solve(cf, r) + Zk @ c

    return apply, lam


def full_system_pcg(orc: NystromSchurOracle, b, tol=1e-8, maxit=1000) -> PCGResult:
    """PCG on A x = b (DBBD order) with the block LDL^T preconditioner built
    from S~^{-1} = the oracle's apply (the approximate block factorisation
    M^{-1} of the Schur-complement section; spectrum Lambda(S~^{-1} S) u {1})."""
    d, ops = orc.dbbd, orc.ops
    nI = d.I.size
    Aperm = d.A[np.concatenate([d.I, d.G])][:, np.concatenate([d.I, d.G])].tocsr()

    def Minv(r):
        rI, rG = r[:nI], r[nI:]
        uI = ops.solve_I(rI)
        yG = orc.apply(rG - d.A_GI @ uI)
        yI = uI - ops.solve_I(d.A_IG @ yG)
        return np.concatenate([yI, yG])

    bp = np.asarray(b)[np.concatenate([d.I, d.G])]
    return pcg(lambda v: Aperm @ v, Minv, bp, tol, maxit)
