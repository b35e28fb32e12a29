"""Grid PDE matrices, box partitions and seeded random inputs.

Conventions shared by every consumer:

* Grid nodes are the unknowns; the homogeneous Dirichlet boundary lies outside
  the grid.  Nodes are numbered x fastest, then y, then z.
* Separators: along an axis with N nodes split into nb boxes, the N-(nb-1)
  non-separator nodes are cut into near-equal boxes, larger boxes first, with a
  one-node separator line/plane between consecutive boxes.
* Partition labels (int32, one per node):
    part >= 0   interior node of subdomain `part`
    part == -1  interface node that is a level-2 junction
    part <= -2  interface node in level-2 block (-2 - part)
  With ``level2=False`` every interface node is labelled -1.
* Sketch: ``numpy.random.default_rng(seed).standard_normal((n_gamma, k+p))``,
  row-major, rows in ascending original node index of the interface.
* Right-hand side: ``numpy.random.default_rng(1000 + seed).standard_normal(n)``.
* Coefficient fields: g = sigma * standardize(h) with h i.i.d. N(0,1) node
  noise smoothed by a periodic separable Gaussian filter of standard deviation
  ell/sqrt(2) cells (covariance ~ exp(-r^2/(2 ell^2))); kappa = exp(g).  A face
  between two nodes carries the harmonic mean of their kappa; a face to the
  Dirichlet boundary carries the node's kappa.  A_ii = sum of its faces,
  A_ij = -kappa_face.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import scipy.sparse as sp
from scipy import ndimage


@dataclasses.dataclass
class GridProblem:
    """One synthetic SPD system in CSR form plus its DBBD partition labels."""

    name: str
    shape: tuple
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]
    part: np.ndarray  # int32 [n]
    k: int
    p: int
    tol_inner: float = 0.1
    tol_outer: float = 1e-8
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])

    @property
    def n_gamma(self) -> int:
        return int(np.count_nonzero(self.part < 0))

    @property
    def n_sub(self) -> int:
        return int(self.part.max()) + 1 if np.any(self.part >= 0) else 0

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def omega(self) -> np.ndarray:
        return sketch(self.n_gamma, self.k + self.p, self.seed)

    def b(self) -> np.ndarray:
        return rhs(self.n, self.seed)


# ----------------------------------------------------------------------------
# partitions


def box_ids_1d(N: int, nb: int) -> np.ndarray:
    """Box index of every node along one axis (-1 on separator nodes)."""
    if nb < 1 or N - (nb - 1) < nb:
        raise ValueError(f"cannot split {N} nodes into {nb} boxes")
    m = N - (nb - 1)
    base, extra = divmod(m, nb)
    sizes = [base + 1 if b < extra else base for b in range(nb)]
    ids = np.empty(N, dtype=np.int64)
    pos = 0
    for b, s in enumerate(sizes):
        ids[pos : pos + s] = b
        pos += s
        if b < nb - 1:
            ids[pos] = -1
            pos += 1
    assert pos == N
    return ids


def partition_boxes(shape: Sequence[int], nboxes: Sequence[int]) -> np.ndarray:
    """Level-1 labels: box id for interior nodes, -1 for separator nodes.

    ``shape`` is (Nx,), (Nx, Ny) or (Nx, Ny, Nz); box ids are numbered x fastest.
    """
    ids = [box_ids_1d(N, nb) for N, nb in zip(shape, nboxes)]
    grids = np.meshgrid(*ids, indexing="ij")  # axis order x, y, z
    sep = np.zeros(grids[0].shape, dtype=bool)
    lin = np.zeros(grids[0].shape, dtype=np.int64)
    stride = 1
    for g, nb in zip(grids, nboxes):
        sep |= g < 0
        lin += np.maximum(g, 0) * stride
        stride *= nb
    lab = np.where(sep, -1, lin)
    # flatten x fastest: transpose (x,y,z) -> (z,y,x) C-order
    return np.ascontiguousarray(lab.transpose(tuple(reversed(range(len(shape)))))).ravel().astype(np.int32)


def level2_labels(A: sp.csr_matrix, part1: np.ndarray) -> np.ndarray:
    """Split the interface into level-2 blocks and junctions.

    An interface node is a junction when its interior neighbours do not lie in
    exactly two subdomains, or when it is coupled to another interface node
    whose pair of adjacent subdomains differs from its own.  The remaining
    interface nodes are grouped by their pair of adjacent subdomains; groups are
    numbered by their smallest node index.  Distinct groups are then never
    coupled, so A_Gamma is itself in doubly bordered block diagonal form.
    """
    A = A.tocsr()
    n = A.shape[0]
    part1 = np.asarray(part1)
    is_if = part1 < 0
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    keep = (rows != cols) & (A.data != 0)
    rows, cols = rows[keep], cols[keep]
    # interface rows, interior columns: which subdomains touch each interface node
    m = is_if[rows] & ~is_if[cols]
    ri, pj = rows[m], part1[cols[m]].astype(np.int64)
    nsub = int(part1.max()) + 1 if np.any(~is_if) else 1
    key = np.unique(ri.astype(np.int64) * nsub + pj)
    ui, up = key // nsub, key % nsub
    cnt = np.bincount(ui, minlength=n)
    lo = np.full(n, np.iinfo(np.int64).max)
    hi = np.full(n, -1, dtype=np.int64)
    np.minimum.at(lo, ui, up)
    np.maximum.at(hi, ui, up)
    junction = is_if & (cnt != 2)
    pair = np.where(junction | ~is_if, -1, lo * nsub + hi)
    # second rule: coupled interface nodes with different pairs
    m2 = is_if[rows] & is_if[cols] & ~junction[rows] & ~junction[cols]
    bad = m2 & (pair[rows] != pair[cols])
    junction[rows[bad]] = True
    junction[cols[bad]] = True
    out = part1.astype(np.int32).copy()
    out[junction] = -1
    seg = is_if & ~junction
    if np.any(seg):
        idx = np.nonzero(seg)[0]
        pk = pair[idx]
        uniq, first = np.unique(pk, return_index=True)
        order = np.argsort(idx[first], kind="stable")
        gid = np.empty(uniq.shape[0], dtype=np.int64)
        gid[order] = np.arange(uniq.shape[0])
        g = gid[np.searchsorted(uniq, pk)]
        out[idx] = (-2 - g).astype(np.int32)
    return out


# ----------------------------------------------------------------------------
# coefficient fields and matrices


def lognormal_field(shape: Sequence[int], sigma: float, ell: float, seed: int) -> np.ndarray:
    """kappa = exp(sigma * standardize(gaussian_filter(noise, ell/sqrt(2), wrap))).

    Returned with the x axis first (array index [x, y, z]).
    """
    rng = np.random.default_rng(seed)
    h = rng.standard_normal(tuple(shape))
    h = ndimage.gaussian_filter(h, sigma=ell / math.sqrt(2.0), mode="wrap")
    h = (h - h.mean()) / h.std()
    return np.exp(sigma * h)


def _flat_index(coords, shape):
    idx = np.zeros_like(coords[0])
    stride = 1
    for c, N in zip(coords, shape):
        idx = idx + c * stride
        stride *= N
    return idx


def diffusion_fd(kappa: np.ndarray) -> sp.csr_matrix:
    """Cell-centred finite-difference diffusion (5-point in 2D, 7-point in 3D).

    ``kappa`` is indexed [x, y(, z)].  Face coefficient = harmonic mean of the
    two nodes; Dirichlet faces use the node coefficient.
    """
    shape = kappa.shape
    d = len(shape)
    n = int(np.prod(shape))
    coords = np.meshgrid(*[np.arange(N) for N in shape], indexing="ij")
    diag = np.zeros(shape)
    rows, cols, vals = [], [], []
    for ax in range(d):
        N = shape[ax]
        sl_lo = [slice(None)] * d
        sl_hi = [slice(None)] * d
        sl_lo[ax] = slice(0, N - 1)
        sl_hi[ax] = slice(1, N)
        k0 = kappa[tuple(sl_lo)]
        k1 = kappa[tuple(sl_hi)]
        face = 2.0 * k0 * k1 / (k0 + k1)
        diag[tuple(sl_lo)] += face
        diag[tuple(sl_hi)] += face
        # boundary faces
        first = [slice(None)] * d
        last = [slice(None)] * d
        first[ax] = slice(0, 1)
        last[ax] = slice(N - 1, N)
        diag[tuple(first)] += kappa[tuple(first)]
        diag[tuple(last)] += kappa[tuple(last)]
        i0 = _flat_index([c[tuple(sl_lo)] for c in coords], shape).ravel()
        i1 = _flat_index([c[tuple(sl_hi)] for c in coords], shape).ravel()
        f = face.ravel()
        rows += [i0, i1]
        cols += [i1, i0]
        vals += [-f, -f]
    ii = _flat_index(coords, shape).ravel()
    rows.append(ii)
    cols.append(ii)
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A = A.tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def laplacian(shape: Sequence[int]) -> sp.csr_matrix:
    """Unscaled Dirichlet Laplacian (diagonal 2*dim, off-diagonals -1)."""
    return diffusion_fd(np.ones(tuple(shape)))


def q1_element_stiffness(K: np.ndarray) -> np.ndarray:
    """4x4 bilinear element stiffness of div(K grad u) on the unit square.

    Local node order: (0,0), (1,0), (1,1), (0,1).  2x2 Gauss quadrature is
    exact for this integrand.
    """
    g = 0.5 / math.sqrt(3.0)
    pts = [0.5 - g, 0.5 + g]
    corners = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=float)
    Ke = np.zeros((4, 4))
    for xq in pts:
        for yq in pts:
            grads = np.empty((4, 2))
            for a, (cx, cy) in enumerate(corners):
                sx = 1.0 if cx else -1.0
                sy = 1.0 if cy else -1.0
                fx = xq if cx else 1.0 - xq
                fy = yq if cy else 1.0 - yq
                grads[a] = (sx * fy, sy * fx)
            Ke += 0.25 * grads @ K @ grads.T
    return Ke


def anisotropic_q1(L: int, eps: float, theta: float) -> sp.csr_matrix:
    """9-point Q1 finite-element matrix of -div(K grad u) on an L x L node grid.

    K = R(theta) diag(1, eps) R(theta)^T, unit elements, homogeneous Dirichlet
    nodes surrounding the grid.
    """
    c, s = math.cos(theta), math.sin(theta)
    R = np.array([[c, -s], [s, c]])
    K = R @ np.diag([1.0, eps]) @ R.T
    Ke = q1_element_stiffness(K)
    offs = np.array([[0, 0], [1, 0], [1, 1], [0, 1]])
    ex, ey = np.meshgrid(np.arange(-1, L), np.arange(-1, L), indexing="ij")
    ex, ey = ex.ravel(), ey.ravel()
    rows, cols, vals = [], [], []
    for a in range(4):
        xa, ya = ex + offs[a, 0], ey + offs[a, 1]
        ma = (xa >= 0) & (xa < L) & (ya >= 0) & (ya < L)
        for b in range(4):
            xb, yb = ex + offs[b, 0], ey + offs[b, 1]
            m = ma & (xb >= 0) & (xb < L) & (yb >= 0) & (yb < L)
            rows.append(xa[m] + L * ya[m])
            cols.append(xb[m] + L * yb[m])
            vals.append(np.full(int(m.sum()), Ke[a, b]))
    n = L * L
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    # exact symmetry (rounding in the element sum is identical for (i,j),(j,i))
    A = ((A + A.T) * 0.5).tocsr()
    A.sort_indices()
    return A


# ----------------------------------------------------------------------------
# random inputs


def sketch(n_gamma: int, s: int, seed: int) -> np.ndarray:
    """Gaussian sketch Omega: n_gamma x s, row-major, from default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal((n_gamma, s))


def rhs(n: int, seed: int) -> np.ndarray:
    """Right-hand side b ~ N(0,1) from default_rng(1000 + seed)."""
    return np.random.default_rng(1000 + seed).standard_normal(n)


# ----------------------------------------------------------------------------
# problem builders


def _to_problem(name, shape, A, part, k, p, tol_inner, tol_outer, seed) -> GridProblem:
    A = A.tocsr()
    A.sort_indices()
    return GridProblem(
        name=name,
        shape=tuple(shape),
        row_ptr=A.indptr.astype(np.int64),
        col=A.indices.astype(np.int32),
        val=A.data.astype(np.float64),
        part=np.ascontiguousarray(part, dtype=np.int32),
        k=k,
        p=p,
        tol_inner=tol_inner,
        tol_outer=tol_outer,
        seed=seed,
    )


def make_problem(
    shape: Sequence[int],
    nboxes: Sequence[int],
    *,
    sigma: float = 0.0,
    ell: float = 8.0,
    field_seed: int = 0,
    k: int = 20,
    p: int = 10,
    tol_inner: float = 0.1,
    tol_outer: float = 1e-8,
    seed: int = 0,
    level2: bool = True,
    name: Optional[str] = None,
) -> GridProblem:
    """Finite-difference diffusion on a box grid; sigma=0 gives the Laplacian."""
    shape = tuple(int(s) for s in shape)
    if sigma == 0.0:
        A = laplacian(shape)
    else:
        A = diffusion_fd(lognormal_field(shape, sigma, ell, field_seed))
    part = partition_boxes(shape, nboxes)
    if level2:
        part = level2_labels(A, part)
    return _to_problem(name or f"fd{len(shape)}d_{'x'.join(map(str, shape))}", shape, A, part, k, p, tol_inner,
                       tol_outer, seed)


def config_c0(level2: bool = True) -> GridProblem:
    """Paper-protocol shape: 2D lognormal (sigma 2, ell 8) 200^2, 8x8 boxes, k=20, p=0, tol 1e-6."""
    return make_problem((200, 200), (8, 8), sigma=2.0, ell=8.0, field_seed=0, k=20, p=0, tol_outer=1e-6,
                        level2=level2, name="c0_lognormal2d_200")


def config_c1(level2: bool = True, seed: int = 0) -> GridProblem:
    """2D 5-point Laplacian 64x64, 2x2 boxes (separators row/col 32), k=20, p=10."""
    return make_problem((64, 64), (2, 2), k=20, p=10, seed=seed, level2=level2, name="c1_laplace2d_64")


def config_c2(level2: bool = True, N: int = 64, nb: int = 4) -> GridProblem:
    """3D 7-point lognormal (sigma 2, ell 8) 64^3, 4x4x4 boxes, k=64, p=16."""
    return make_problem((N, N, N), (nb, nb, nb), sigma=2.0, ell=8.0, field_seed=0, k=64, p=16, level2=level2,
                        name=f"c2_lognormal3d_{N}")


def aniso_problem(L: int, theta: float, *, eps: float = 1e-3, nboxes=(4, 4), k: int = 32, p: int = 8,
                  seed: int = 0, level2: bool = True, name: Optional[str] = None) -> GridProblem:
    """2D anisotropic Q1 problem on an L x L grid split into box subdomains."""
    A = anisotropic_q1(L, eps, theta)
    part = partition_boxes((L, L), nboxes)
    if level2:
        part = level2_labels(A, part)
    return _to_problem(name or f"aniso_q1_L{L}", (L, L), A, part, k, p, 0.1, 1e-8, seed)


def config_c3_problem(i: int, level2: bool = True, L_range=(128, 512)) -> GridProblem:
    """Problem i of the batched set: 2D anisotropic Q1, L ~ U{128..512}, eps=1e-3,
    random rotation, 4x4 boxes, k=32, p=8; everything drawn from default_rng(7000+i)."""
    rng = np.random.default_rng(7000 + i)
    L = int(rng.integers(L_range[0], L_range[1] + 1))
    theta = float(rng.uniform(0.0, math.pi))
    return aniso_problem(L, theta, k=32, p=8, seed=i, level2=level2, name=f"c3_aniso_q1_{i}_L{L}")


def config_c4(seed: int = 0, level2: bool = True, N: int = 48) -> GridProblem:
    """3D 7-point lognormal (sigma 1.5, ell 8) 48^3, 3x3x3 boxes, k=48, p=12.

    ``seed`` selects the coefficient field (the learned-proposal family) and
    the sketch / right-hand side.
    """
    return make_problem((N, N, N), (3, 3, 3), sigma=1.5, ell=8.0, field_seed=seed, k=48, p=12, seed=seed,
                        level2=level2, name=f"c4_lognormal3d_{N}_s{seed}")


def config_c5(level2: bool = True, N: int = 2048, nb: int = 32) -> GridProblem:
    """2D 5-point lognormal (sigma 2, ell 8) 2048^2, 32x32 boxes, k=128, p=32."""
    return make_problem((N, N), (nb, nb), sigma=2.0, ell=8.0, field_seed=0, k=128, p=32, level2=level2,
                        name=f"c5_lognormal2d_{N}")


CONFIGS = {
    "c0": config_c0,
    "c1": config_c1,
    "c2": config_c2,
    "c4": config_c4,
    "c5": config_c5,
}


def random_dbbd(seed: int, sizes=(7, 5, 9), n_gamma: int = 6, density: float = 0.4,
                level2: bool = False) -> GridProblem:
    """Small random SPD matrix already in DBBD structure (for property tests).

    Interior blocks of the given sizes, ``n_gamma`` interface nodes, random
    sparse symmetric couplings and a strictly dominant diagonal.  Nodes are
    shuffled so the ordering is not the DBBD one.
    """
    rng = np.random.default_rng(seed)
    nI = int(sum(sizes))
    n = nI + n_gamma
    lab = np.concatenate([np.repeat(np.arange(len(sizes)), sizes), -np.ones(n_gamma, dtype=np.int64)])
    M = np.zeros((n, n))
    for i in range(n):
        for j in range(i):
            a, b = lab[i], lab[j]
            if a >= 0 and b >= 0 and a != b:
                continue
            if rng.random() < density:
                v = rng.uniform(-1.0, 1.0)
                M[i, j] = M[j, i] = v
    M += np.diag(np.abs(M).sum(axis=1) + rng.uniform(0.1, 1.0, n))
    perm = rng.permutation(n)
    Mp = M[np.ix_(perm, perm)]
    part = lab[perm].astype(np.int32)
    A = sp.csr_matrix(Mp)
    A.sort_indices()
    return _to_problem(f"random_dbbd_{seed}", (n,), A, part, 2, 1, 0.1, 1e-8, seed)
