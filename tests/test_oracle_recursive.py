"""Pins of the oracle's recursive construction (A_Gamma^{-1} replaced by a Nystrom-Schur preconditioner of A_Gamma
one level down), each against something other than the oracle itself:

* exactness: with a full-rank level-2 sketch (k_2 = n_J) and a tight level-2 inner solve the Nystrom
  approximation of A_Js S_s^{-1} A_sJ is exact, so M_J = S_J^{-1} and the recursive solve equals the exact
  A_Gamma^{-1} (a dense LAPACK solve here), and the level-1 counts equal the exact oracle's;
* the block LDL^T identity of the Schur-complement section one level down: Lambda(A~^{-1} A_Gamma) =
  Lambda(M_J S_J) u {1}^{n_s}, with S_J formed densely from its definition;
* symmetry and positive definiteness of A~^{-1};
* with k_2 = 0, M_J = A_J^{-1} and Lambda(A_J^{-1} S_J) lies in (0, 1] (eq. schur_complement one level down);
  with an exact level-2 sketch product the low-rank term lies between 0 and A_J^{-1} B_J A_J^{-1} (Nystrom never
  overestimates), so the spectrum stays in (0, 1] and rises monotonically above the k_2 = 0 spectrum.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import DBBD, NystromSchurOracle, RecursiveGamma, dense_schur, level2_part
from workloads import make_problem


@pytest.fixture(scope="module")
def prob():
    P = make_problem((10, 10, 10), (2, 2, 2), sigma=1.5, ell=3.0, k=6, p=3)
    d = DBBD(P.n, P.row_ptr, P.col, P.val, P.part)
    nJ = int(np.count_nonzero(level2_part(d) == -1))
    return P, d, nJ


def spd_spectrum(M, A):
    """Eigenvalues of M A for SPD M and symmetric A (through the Cholesky factor of M)."""
    L = np.linalg.cholesky(0.5 * (M + M.T))
    return np.sort(np.linalg.eigvalsh(L.T @ A @ L))


def test_level2_labels_split_interface(prob):
    P, d, nJ = prob
    part2 = level2_part(d)
    pg = d.part[d.G]
    assert np.array_equal(part2 == -1, pg == -1)
    assert np.array_equal(part2[pg <= -2], -2 - pg[pg <= -2])
    assert 0 < nJ < d.n_gamma


def test_full_rank_level2_is_the_exact_solve(prob):
    P, d, nJ = prob
    om2 = np.random.default_rng(3).standard_normal((nJ, nJ))
    rg = RecursiveGamma(d, k=nJ, p=0, omega=om2, tol_inner=1e-14, eps_rel=1e-14)
    X = np.random.default_rng(1).standard_normal((d.n_gamma, 3))
    ref = sla.solve(d.A_G.toarray(), X, assume_a="pos")
    assert np.linalg.norm(rg.solve(X) - ref) <= 1e-10 * np.linalg.norm(ref)
    o_ex = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=6, p=3, omega=P.omega())
    o_rec = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=6, p=3, omega=P.omega(),
                               level2=dict(k=nJ, p=0, omega=om2, tol_inner=1e-14), eps_rel=1e-10)
    s1, s2 = o_ex.setup(), o_rec.setup()
    r1, r2 = o_ex.solve(P.b(), tol=1e-8), o_rec.solve(P.b(), tol=1e-8)
    assert s1.it_inner == s2.it_inner and r1.it_pcg == r2.it_pcg
    assert np.linalg.norm(r1.x - r2.x) <= 1e-8 * np.linalg.norm(r1.x)


@pytest.mark.parametrize("k2,p2,tol2", [(6, 3, 0.1), (10, 0, 0.1), (4, 4, 1e-3)])
def test_block_ldlt_spectrum_identity(prob, k2, p2, tol2):
    P, d, nJ = prob
    rg = RecursiveGamma(d, k=k2, p=p2, omega=np.random.default_rng(k2).standard_normal((nJ, k2 + p2)),
                        tol_inner=tol2)
    Mt = rg.solve(np.eye(d.n_gamma))
    assert np.linalg.norm(Mt - Mt.T) <= 1e-13 * np.linalg.norm(Mt)
    assert np.linalg.eigvalsh(0.5 * (Mt + Mt.T)).min() > 0
    ev = spd_spectrum(Mt, d.A_G.toarray())
    sub = rg.inner
    evJ = spd_spectrum(sub.apply(np.eye(nJ)), dense_schur(sub.dbbd))
    ref = np.sort(np.concatenate([evJ, np.ones(d.n_gamma - nJ)]))
    assert np.abs(ev - ref).max() <= 1e-10


def test_first_level_and_monotone_low_rank(prob):
    P, d, nJ = prob
    AG = d.A_G.toarray()
    r0 = RecursiveGamma(d, k=0, p=0, omega=None)
    ev0 = spd_spectrum(r0.solve(np.eye(d.n_gamma)), AG)
    assert ev0.min() > 0 and ev0.max() <= 1 + 1e-12
    # dense A_J^{-1} S_J from the definitions, plus the unit eigenvalues of the separator blocks
    sd = r0.inner.dbbd
    evJ = spd_spectrum(np.linalg.inv(sd.A_G.toarray()), dense_schur(sd))
    assert np.abs(ev0 - np.sort(np.concatenate([evJ, np.ones(d.n_gamma - nJ)]))).max() <= 1e-10
    prev = ev0
    for k2 in (4, 8, 16):
        rk = RecursiveGamma(d, k=k2, p=4, omega=np.random.default_rng(k2).standard_normal((nJ, k2 + 4)),
                            tol_inner=1e-13)
        ev = spd_spectrum(rk.solve(np.eye(d.n_gamma)), AG)
        assert ev.max() <= 1 + 1e-9
        assert np.all(ev >= ev0 - 1e-10)
        assert ev.min() >= prev.min() - 1e-10
        prev = ev


def test_recursive_outer_solve_converges(prob):
    P, d, nJ = prob
    o = NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=6, p=3, omega=P.omega(),
                           level2=dict(k=6, p=3, omega=np.random.default_rng(4).standard_normal((nJ, 9))))
    o.setup()
    r = o.solve(P.b(), tol=1e-8)
    assert r.converged and r.relres_true <= 1e-8 and r.relres_schur_true <= 2e-8


def test_recursive_rejects_m1_and_missing_junctions(prob):
    P, d, nJ = prob
    with pytest.raises(ValueError):
        NystromSchurOracle(P.n, P.row_ptr, P.col, P.val, P.part, k=6, p=3, omega=P.omega(), variant="M1",
                           level2=dict(k=2, p=0, omega=np.ones((nJ, 2))))
    Q = make_problem((12, 12), (1, 2), sigma=0.0, ell=3.0, k=2, p=1)  # one straight separator: no junctions
    dq = DBBD(Q.n, Q.row_ptr, Q.col, Q.val, Q.part)
    if not np.any(level2_part(dq) == -1):
        with pytest.raises(ValueError):
            RecursiveGamma(dq, k=0, p=0, omega=None)
