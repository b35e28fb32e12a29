// One-workgroup dense kernels on the s x s matrices of the method (s = k + p):
// Cholesky and solves for block CG, the eigen-decomposition based
// orthonormalisation of a block, shifted Cholesky-QR, and the Nystrom core of
// Algorithm alg:nystrom (EVD of C, threshold, T, EVD of T).  Symmetric
// eigen-decompositions use the cyclic two-sided Jacobi method with a
// round-robin ordering, so all rotations of a round are independent.
// Matrices staged in LDS use a row stride of n + 1 doubles so that column
// accesses spread over the LDS banks.
#include "ns_vec.h"

namespace ns {
namespace {

constexpr int NT = 1024;                  // threads per workgroup
constexpr size_t LDS_LIMIT = 136 * 1024;  // dynamic LDS used when the matrices fit
constexpr int SMAX = 256;                 // largest s supported by the small kernels
constexpr int NB = 16;                    // block size of the blocked factorisations and solves
constexpr int NBL = NB + 1;               // row stride of a diagonal-block inverse

// Workspace (doubles) of the blocked Cholesky kernels, dimensions padded to whole 16-wide tiles
// (rp = ceil16(r), cp = ceil16(c)): factor L (rp x (rp+1)), right-hand sides / inverse X (rp x (cp+1)),
// diagonal-block inverses, panel buffer (rp x NBL) and block-row buffer (NB x (cp+1)).
__host__ __device__ inline int pad16(int n) { return (n + 15) & ~15; }
__host__ __device__ inline size_t chol_ws(int r, int c) {
  const size_t rp = size_t(pad16(r)), cp = size_t(pad16(c));
  return rp * (rp + 1) + rp * (cp + 1) + (rp / NB) * NB * NBL + rp * NBL + size_t(NB) * (cp + 1);
}
__host__ __device__ inline size_t evd_elems(int n) { return size_t(2) * n * (n + 1); }

// 1 / sqrt(d) for d > 0: the hardware estimate refined by two Newton steps y <- y (3 - d y^2) / 2.
__device__ __forceinline__ double rcp_nr(double x) {  // 1 / x: estimate and one Newton step
  const double y = __builtin_amdgcn_rcp(x);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d * y, y, 1.5);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Cyclic Jacobi: A (n x n, row stride ld, symmetric) is diagonalised in place;
// V (stride ld) receives the eigenvectors in its columns.  cs: 2n doubles,
// pr: n+2 ints.  Each round applies the n/2 disjoint rotations J of a
// round-robin ordering at once: A <- J^T A J block by block (2 x 2 blocks of
// two rotation pairs) and V <- V J (columns p, q of every row).
__device__ __forceinline__ void jacobi(double* A, double* V, int n, int ld, double* cs, int* pr, double* red) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    V[i * ld + j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  if (n < 2) return;
  const int m = n + (n & 1);
  const int half = m / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += NT) {
      const int i = e / n, j = e % n;
      const double v = A[i * ld + j] * A[i * ld + j];
      tot += v;
      if (i != j) off += v;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    // stop at the rounding floor: off-diagonal Frobenius norm <= 2 n eps ||A||_F
    if (!(off > 2e-31 * double(n) * double(n) * tot)) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < half) {
        auto pos = [&](int x) { return x == 0 ? 0 : 1 + (x - 1 + round) % (m - 1); };
        int p = pos(tid), q = pos(m - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * ld + q];
          const double app = A[p * ld + p], aqq = A[q * ld + q];
          if (apq * apq > 1e-36 * fabs(app * aqq) && fabs(apq) > 1e-300) {
            // the angle from hardware reciprocal / square-root estimates with one Newton step each; c and s
            // from t keep the rotation orthogonal to rounding whatever the angle's accuracy
            const double tau = (aqq - app) * rcp_nr(2.0 * apq);
            const double at = fabs(tau);
            double tf;
            if (at > 1e15) {
              tf = 0.5 * rcp_nr(at);
            } else {
              const double u = 1.0 + at * at;
              tf = rcp_nr(at + u * rsqrt_nr(u));
            }
            const double t = tau >= 0.0 ? tf : -tf;
            c = rsqrt_nr(1.0 + t * t);
            s = t * c;
          }
        }
        pr[2 * tid] = p;
        pr[2 * tid + 1] = q;  // q == n marks the dummy partner of an odd n
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
      }
      __syncthreads();
      // A <- J^T A J, one thread per 2 x 2 block (rows of pair P, columns of pair Q): the columns are
      // rotated first, then the rows, with the arithmetic of the two separate passes, but with no barrier
      // between them since the blocks are disjoint
      for (int t = tid; t < half * half; t += NT) {
        const int P = t / half, Q = t - P * half;
        const int p = pr[2 * P], q = pr[2 * P + 1], p2 = pr[2 * Q], q2 = pr[2 * Q + 1];
        const bool hq = q < n, hq2 = q2 < n;  // q == n: the dummy partner of an odd n
        const double c1 = cs[2 * P], s1 = cs[2 * P + 1], c2 = cs[2 * Q], s2 = cs[2 * Q + 1];
        const double a = A[p * ld + p2], b = hq2 ? A[p * ld + q2] : 0.0;
        const double c = hq ? A[q * ld + p2] : 0.0, d = (hq && hq2) ? A[q * ld + q2] : 0.0;
        const double a1 = c2 * a - s2 * b, b1 = s2 * a + c2 * b;
        const double c3 = c2 * c - s2 * d, d1 = s2 * c + c2 * d;
        A[p * ld + p2] = c1 * a1 - s1 * c3;
        if (hq2) A[p * ld + q2] = c1 * b1 - s1 * d1;
        if (hq) {
          A[q * ld + p2] = s1 * a1 + c1 * c3;
          if (hq2) A[q * ld + q2] = s1 * b1 + c1 * d1;
        }
      }
      for (int t = tid; t < n * half; t += NT) {  // V <- V J
        const int P = t / n, i = t - P * n;
        const int p = pr[2 * P], q = pr[2 * P + 1];
        if (q >= n) continue;
        const double c = cs[2 * P], s = cs[2 * P + 1];
        const double vp = V[i * ld + p], vq = V[i * ld + q];
        V[i * ld + p] = c * vp - s * vq;
        V[i * ld + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
}

// order[i] = index of the i-th largest of d[0..n) (ties by index).
__device__ __forceinline__ void sort_desc(const double* d, int n, int* order) {
  for (int i = threadIdx.x; i < n; i += NT) {
    int rk = 0;
    const double di = d[i];
    for (int j = 0; j < n; ++j) rk += (d[j] > di) || (d[j] == di && j < i);
    order[rk] = i;
  }
  __syncthreads();
}

// In-place lower Cholesky of A (n x n, stride lda), right-looking: every
// thread reads the pivot, the column below it is scaled, then the trailing
// lower triangle is updated by a 32 x 32 thread grid.  Returns 0 or the
// 1-based index of the first non-positive pivot (the pivot is then taken as 1).
__device__ __forceinline__ int chol_dev(double* A, int n, int lda, int* sinfo) {
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  if (threadIdx.x == 0) *sinfo = 0;
  __syncthreads();
  for (int c = 0; c < n; ++c) {
    double d = A[c * lda + c];
    const bool bad = !(d > 0.0);
    if (bad) d = 1.0;
    const double sq = sqrt(d), inv = 1.0 / sq;
    for (int r = c + 1 + threadIdx.x; r < n; r += NT) A[r * lda + c] *= inv;
    __syncthreads();
    if (threadIdx.x == 0) {
      A[c * lda + c] = sq;
      if (bad && *sinfo == 0) *sinfo = c + 1;
    }
    for (int q = c + 1 + ty; q < n; q += 32) {
      const double aq = A[q * lda + c];
      for (int r = q + tx; r < n; r += 32) A[r * lda + q] -= A[r * lda + c] * aq;
    }
    __syncthreads();
  }
  const int info = *sinfo;
  __syncthreads();
  return info;
}

// X (r x s, stride ldx) <- (L L^T)^{-1} X: forward then backward row sweeps,
// each step's rows (32 thread rows) and columns (32 thread columns) in parallel.
__device__ __forceinline__ void chol_solve_inplace(const double* L, int r, int ldl, double* X, int ldx, int s) {
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int m = 0; m < r; ++m) {  // forward: L y = x
    const double inv = 1.0 / L[m * ldl + m];
    for (int j = threadIdx.x; j < s; j += NT) X[m * ldx + j] *= inv;
    __syncthreads();
    for (int i = m + 1 + ty; i < r; i += 32) {
      const double l = L[i * ldl + m];
      for (int j = tx; j < s; j += 32) X[i * ldx + j] -= l * X[m * ldx + j];
    }
    __syncthreads();
  }
  for (int m = r - 1; m >= 0; --m) {  // backward: L^T x = y
    const double inv = 1.0 / L[m * ldl + m];
    for (int j = threadIdx.x; j < s; j += NT) X[m * ldx + j] *= inv;
    __syncthreads();
    for (int i = ty; i < m; i += 32) {
      const double l = L[m * ldl + i];
      for (int j = tx; j < s; j += 32) X[i * ldx + j] -= l * X[m * ldx + j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- blocked Cholesky toolkit
// Right-looking Cholesky in NB-wide block columns: one wave factors the diagonal block in registers (lane i
// holds row i, pivots and columns broadcast with readlane, no workgroup barrier) and inverts it; the panel
// below is L21 = A21 L11^{-T} through that inverse; the trailing lower triangle is updated by every thread.
// Three workgroup barriers per block column instead of two per column.

__device__ __forceinline__ double lane_of(double v, int lane) {  // v of `lane` (lane uniform)
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Wave-level: factor the jb x jb block at A[j0][j0] (stride ld) in place (lower) and write its inverse to
// Di (NB x NB, stride NBL; lower, zero above).  Returns 0 or the 1-based column of the first pivot <= 0
// (taken as 1).  Called by all 64 lanes of one wave.

__device__ __forceinline__ int diag_factor_wave(double* A, int ld, int j0, int jb, double* Di) {
  const int lane = threadIdx.x & 63;
  double r[NB], invd[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    r[t] = (lane < jb && t <= lane) ? A[(j0 + lane) * ld + j0 + t] : 0.0;
    invd[t] = 1.0;
  }
  int bad = 0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < jb) {
      double d = lane_of(r[c], c);
      if (!(d > 0.0)) {
        if (!bad) bad = c + 1;
        d = 1.0;
      }
      const double inv = rsqrt_nr(d);
      invd[c] = inv;
      r[c] = lane == c ? d * inv : (lane > c ? r[c] * inv : 0.0);
#pragma unroll
      for (int q = c + 1; q < NB; ++q) {
        const double lqc = lane_of(r[c], q);  // L[q][c]
        if (q < jb && lane >= q) r[q] -= r[c] * lqc;
      }
    }
  }
  // column `lane` of L^{-1} by forward substitution (lanes >= jb compute nothing useful)
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double acc = (i == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < i; ++t) acc -= lane_of(r[t], i) * x[t];
    x[i] = (i < jb) ? acc * invd[i] : 0.0;
  }
  if (lane < jb) {
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t <= lane) A[(j0 + lane) * ld + j0 + t] = r[t];
  }
  if (lane < NB) {
#pragma unroll
    for (int i = 0; i < NB; ++i) Di[i * NBL + lane] = (lane < jb && i < jb) ? x[i] : 0.0;
  }
  return bad;
}

// 16x16 tile product on FP64 MFMA: acc += A (16 x K) B (K x 16) with A(i, k) = pa[i sai + k sak] and
// B(k, j) = pb[k sbk + j sbj], K a multiple of 4.  Lane l feeds A(l%16, k + l/16) and B(k + l/16, l%16) and
// holds the output elements (4v + l/16, l%16), v = 0..3.  Called by all lanes of a wave.
typedef double sv4d __attribute__((ext_vector_type(4)));
__device__ __forceinline__ sv4d mma16(sv4d acc, const double* pa, int sai, int sak, const double* pb, int sbk,
                                      int sbj, int K) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  pa += li * sai + lk * sak;
  pb += lk * sbk + li * sbj;
#pragma unroll 4
  for (int k = 0; k < K; k += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[k * sak], pb[k * sbk], acc, 0, 0, 0);
  return acc;
}
__device__ __forceinline__ int tile_row(int v) { return 4 * v + ((threadIdx.x & 63) >> 4); }
__device__ __forceinline__ int tile_col() { return threadIdx.x & 15; }
constexpr int NW = NT / 64;  // waves per workgroup

// In-place lower Cholesky of A (np x np, np a multiple of NB, stride ld; rows and columns past the problem's
// dimension hold the identity).  Dinv: np/NB diagonal-block inverses (NB x NBL each), Pn: np x NBL panel
// scratch.  Panels and trailing updates are 16x16 MFMA tiles.  Returns 0 or the 1-based index of the first
// pivot <= 0.
__device__ __forceinline__ int chol_blocked(double* A, int np, int ld, double* Dinv, double* Pn, int* sinfo) {
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) *sinfo = 0;
  __syncthreads();
  for (int j0 = 0; j0 < np; j0 += NB) {
    double* Di = Dinv + (j0 / NB) * (NB * NBL);
    if (wave == 0) {
      const int bad = diag_factor_wave(A, ld, j0, NB, Di);
      if (bad && (threadIdx.x & 63) == 0 && *sinfo == 0) *sinfo = j0 + bad;
    }
    __syncthreads();
    const int j1 = j0 + NB, mt = (np - j1) / NB;
    for (int t = wave; t < mt; t += NW) {  // Pn = A21 L11^{-T}
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, A + (j1 + NB * t) * ld + j0, ld, 1, Di, 1, NBL, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) Pn[(NB * t + tile_row(v)) * NBL + tile_col()] = acc[v];
    }
    __syncthreads();
    const int ntri = mt * (mt + 1) / 2;
    for (int u = wave; u < ntri; u += NW) {  // A22 -= L21 L21^T on the lower tiles
      int ti = 0;
      while ((ti + 1) * (ti + 2) / 2 <= u) ++ti;
      const int tq = u - ti * (ti + 1) / 2;
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, Pn + NB * ti * NBL, NBL, 1, Pn + NB * tq * NBL, 1, NBL, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(j1 + NB * ti + tile_row(v)) * ld + j1 + NB * tq + tile_col()] -= acc[v];
    }
    for (int e = threadIdx.x; e < (np - j1) * NB; e += NT) {
      const int i = e / NB, c = e - i * NB;
      A[(j1 + i) * ld + j0 + c] = Pn[i * NBL + c];
    }
    __syncthreads();
  }
  const int info = *sinfo;
  __syncthreads();
  return info;
}

// Diagonal-block inverses of an existing factor L (np x np, stride ld): one wave per block.
__device__ __forceinline__ void diag_inverses(const double* L, int np, int ld, double* Dinv) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int bk = wave; bk < np / NB; bk += NW) {
    const int j0 = bk * NB;
    double x[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double acc = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < i; ++t) acc -= L[(j0 + i) * ld + j0 + t] * x[t];
      x[i] = acc / L[(j0 + i) * ld + j0 + i];
    }
    if (lane < NB) {
#pragma unroll
      for (int i = 0; i < NB; ++i) Dinv[bk * (NB * NBL) + i * NBL + lane] = x[i];
    }
  }
  __syncthreads();
}

// X (rp x cp, stride lx; rp, cp multiples of NB) <- (L L^T)^{-1} X by block rows: forward L Y = X, then
// backward L^T X = Y.  Tb: NB x (cp + 1) scratch.
__device__ __forceinline__ void chol_solve_blocked(const double* L, int rp, int ld, const double* Dinv, double* X, int lx, int cp,
                                   double* Tb) {
  const int wave = threadIdx.x >> 6, nbk = rp / NB, ct = cp / NB, lt = cp + 1;
  for (int bk = 0; bk < nbk; ++bk) {
    const int i0 = bk * NB;
    const double* Di = Dinv + bk * (NB * NBL);
    for (int jt = wave; jt < ct; jt += NW) {  // Tb = X_i - L_{i,<i} Y_{<i}
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, L + i0 * ld, ld, 1, X + NB * jt, lx, 1, i0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = tile_row(v), j = NB * jt + tile_col();
        Tb[a * lt + j] = X[(i0 + a) * lx + j] - acc[v];
      }
    }
    __syncthreads();
    for (int jt = wave; jt < ct; jt += NW) {  // Y_i = L_ii^{-1} Tb
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, Di, NBL, 1, Tb + NB * jt, lt, 1, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(i0 + tile_row(v)) * lx + NB * jt + tile_col()] = acc[v];
    }
    __syncthreads();
  }
  for (int bk = nbk - 1; bk >= 0; --bk) {
    const int i0 = bk * NB, i1 = i0 + NB;
    const double* Di = Dinv + bk * (NB * NBL);
    for (int jt = wave; jt < ct; jt += NW) {  // Tb = Y_i - L_{>i,i}^T X_{>i}
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, L + i1 * ld + i0, 1, ld, X + i1 * lx + NB * jt, lx, 1, rp - i1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = tile_row(v), j = NB * jt + tile_col();
        Tb[a * lt + j] = X[(i0 + a) * lx + j] - acc[v];
      }
    }
    __syncthreads();
    for (int jt = wave; jt < ct; jt += NW) {  // X_i = L_ii^{-T} Tb
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, Di, 1, NBL, Tb + NB * jt, lt, 1, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(i0 + tile_row(v)) * lx + NB * jt + tile_col()] = acc[v];
    }
    __syncthreads();
  }
}

// X = L^{-1} (np x np, stride ld, zero above the diagonal) from the factor and its diagonal-block inverses,
// by block rows: X_ij = -L_ii^{-1} sum_{j <= t < i} L_it X_tj.  Tb: NB x (np + 1) scratch.
__device__ __forceinline__ void tri_inverse_blocked(const double* L, int np, int ld, const double* Dinv, double* X, double* Tb) {
  const int wave = threadIdx.x >> 6, lt = np + 1;
  for (int e = threadIdx.x; e < np * np; e += NT) {
    const int i = e / np, j = e - i * np;
    const int bi = i / NB, bj = j / NB;
    X[i * ld + j] = (bi == bj && j <= i) ? Dinv[bi * (NB * NBL) + (i - bi * NB) * NBL + (j - bj * NB)] : 0.0;
  }
  __syncthreads();
  for (int bk = 1; bk < np / NB; ++bk) {
    const int i0 = bk * NB;
    const double* Di = Dinv + bk * (NB * NBL);
    for (int jt = wave; jt < bk; jt += NW) {  // Tb_j = L_{i, j..i-1} X_{j..i-1, j}
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, L + i0 * ld + NB * jt, ld, 1, X + NB * jt * ld + NB * jt, ld, 1, i0 - NB * jt);
#pragma unroll
      for (int v = 0; v < 4; ++v) Tb[tile_row(v) * lt + NB * jt + tile_col()] = acc[v];
    }
    __syncthreads();
    for (int jt = wave; jt < bk; jt += NW) {  // X_ij = -L_ii^{-1} Tb_j
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, Di, NBL, 1, Tb + NB * jt, lt, 1, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(i0 + tile_row(v)) * ld + NB * jt + tile_col()] = -acc[v];
    }
    __syncthreads();
  }
}

// Carve of a chol_ws(r, c) workspace (padded dimensions rp, cp).
struct CholWs {
  double *L, *X, *Dinv, *Pn, *Tb;
  int rp, cp, ldl, ldx;
};
__device__ __forceinline__ CholWs chol_carve(double* base, int r, int c) {
  CholWs w;
  w.rp = pad16(r);
  w.cp = pad16(c);
  w.ldl = w.rp + 1;
  w.ldx = w.cp + 1;
  w.L = base;
  w.X = w.L + size_t(w.rp) * w.ldl;
  w.Dinv = w.X + size_t(w.rp) * w.ldx;
  w.Pn = w.Dinv + size_t(w.rp / NB) * NB * NBL;
  w.Tb = w.Pn + size_t(w.rp) * NBL;
  return w;
}

// Problem b: D (r0 x r0, ld r0) at D + b sD, leading rb = dims[b] block used; B, X likewise.  factor: D is
// factored (L written back); otherwise D holds the factor from an earlier call.  In LDS the factor is padded
// with the identity and the right-hand sides with zeros to whole 16-wide tiles.
template <int kLds>
__global__ __launch_bounds__(NT) void k_small_chol_solve(int r0, const int* __restrict__ dims, double* D, int64_t sD,
                                                         const double* B, int64_t ldb, int64_t sB, double* X,
                                                         int64_t ldx, int64_t sX, int s, int s0, double alpha,
                                                         int* flag, int factor, double* gw, int64_t gws) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  const int b = blockIdx.x;
  const int r = dims ? dims[b] : r0;
  D += b * sD;
  B += b * sB;
  X += b * sX;
  // rows r .. s0 - 1 of X are zero (directions this problem does not have)
  for (int e = threadIdx.x; e < (s0 - r) * s; e += NT) X[(r + e / s) * ldx + e % s] = 0.0;
  if (r == 0) return;
  CholWs w = chol_carve(kLds ? sm : gw + b * gws, r, s);
  const int rp = w.rp, cp = w.cp;
  for (int e = threadIdx.x; e < rp * rp; e += NT) {
    const int i = e / rp, j = e - i * rp;
    w.L[i * w.ldl + j] = (i < r && j < r) ? D[i * r0 + j] : (i == j ? 1.0 : 0.0);
  }
  for (int e = threadIdx.x; e < rp * cp; e += NT) {
    const int i = e / cp, j = e - i * cp;
    w.X[i * w.ldx + j] = (i < r && j < s) ? B[i * ldb + j] : 0.0;
  }
  __syncthreads();
  if (factor) {
    const int info = chol_blocked(w.L, rp, w.ldl, w.Dinv, w.Pn, &sinfo);
    if (info && threadIdx.x == 0) flag[0] = 1;
    for (int e = threadIdx.x; e < r * r; e += NT) {
      const int i = e / r, j = e % r;
      D[i * r0 + j] = j <= i ? w.L[i * w.ldl + j] : 0.0;
    }
  } else {
    diag_inverses(w.L, rp, w.ldl, w.Dinv);
  }
  if (s == 0) return;
  chol_solve_blocked(w.L, rp, w.ldl, w.Dinv, w.X, w.ldx, cp, w.Tb);
  for (int e = threadIdx.x; e < r * s; e += NT) X[(e / s) * ldx + e % s] = alpha * w.X[(e / s) * w.ldx + e % s];
}

// Workspace for the Jacobi kernels: two n x (n+1) matrices + small arrays, in
// LDS when they fit, else in the caller's global scratch `gw`.
struct EvdSpace {
  double *A, *V, *cs, *d;
  int *pr, *ord;
  int ld;
};

__device__ __forceinline__ EvdSpace evd_space(int n, double* base, double* small_d, int* small_i) {
  EvdSpace e;
  e.ld = n + 1;
  e.A = base;
  e.V = base + size_t(n) * e.ld;
  e.cs = small_d;
  e.d = small_d + 2 * n;
  e.pr = small_i;
  e.ord = small_i + 2 * n;
  return e;
}

template <int kLds>
__global__ __launch_bounds__(NT) void k_small_svqb(int s, const double* G, int64_t sG, double drop2, double* T,
                                                   int64_t sT, int* out, const int* skip, double* gw, int64_t gws) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  const int b = blockIdx.x;
  if (skip && skip[b]) return;
  G += b * sG;
  T += b * sT;
  EvdSpace w = evd_space(s, kLds ? sm : gw + b * gws, sd, si);
  const int ld = w.ld;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    w.A[i * ld + j] = 0.5 * (G[i * s + j] + G[j * s + i]);
  }
  __syncthreads();
  jacobi(w.A, w.V, s, ld, w.cs, w.pr, red);
  for (int i = threadIdx.x; i < s; i += NT) w.d[i] = w.A[i * ld + i];
  __syncthreads();
  sort_desc(w.d, s, w.ord);
  const double lmax = w.d[w.ord[0]];
  int kept = 0;
  for (int c = 0; c < s; ++c) {
    const double l = w.d[w.ord[c]];
    if (l > 0.0 && l > drop2 * lmax)
      ++kept;
    else
      break;
  }
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, c = e % s;
    T[e] = c < kept ? w.V[i * ld + w.ord[c]] / sqrt(w.d[w.ord[c]]) : 0.0;
  }
  if (threadIdx.x == 0) out[b] = kept;
}

// Problem b: G (s x s) at G + b sG; the leading n = dims[b] block is factored, everything else of Rinv and
// Racc is zero.
template <int kLds>
__global__ __launch_bounds__(NT) void k_small_cholqr(int s, const int* __restrict__ dims, const double* G, int64_t sG,
                                                     const double* shift_coef, double* Rinv, double* Racc, int init,
                                                     int* flag, double* gw, int64_t gws, double certify,
                                                     int* ok, double single_thr, int* single) {
  extern __shared__ double sm[];
  __shared__ int sinfo, refine;
  double lmax_c = 0.0;
  __shared__ double red[NT];
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : s;
  const int wave = threadIdx.x >> 6;
  G += b * sG;
  Rinv += b * int64_t(s) * s;
  Racc += b * int64_t(s) * s;
  if (n == 0) {
    for (int e = threadIdx.x; e < s * s; e += NT) Rinv[e] = Racc[e] = 0.0;
    if (ok && threadIdx.x == 0) ok[b] = 0;
    if (single && threadIdx.x == 0) single[b] = 0;
    return;
  }
  double tr = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) tr += G[i * s + i];
  if (threadIdx.x == 0) refine = 0;
  tr = block_sum(tr, red);
  const double shift = (shift_coef ? shift_coef[b] : 0.0) * tr;
  CholWs w = chol_carve(kLds ? sm : gw + b * gws, n, n);
  const int np = w.rp, ld = w.ldl;
  double* A = w.L;
  double* X = w.X;
  for (int e = threadIdx.x; e < np * np; e += NT) {
    const int i = e / np, j = e - i * np;
    A[i * ld + j] = (i < n && j < n) ? 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift : 0.0)
                                     : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (chol_blocked(A, np, ld, w.Dinv, w.Pn, &sinfo) && threadIdx.x == 0) flag[0] = 1;
  tri_inverse_blocked(A, np, ld, w.Dinv, X, w.Tb);  // X = L^{-1}
  for (int e = threadIdx.x; e < np * np; e += NT) {  // the factorisation leaves values above the diagonal
    const int i = e / np, j = e - i * np;
    if (j > i) A[i * ld + j] = 0.0;
  }
  // Rinv = (L^{-1})^T (upper) in the leading block, zero elsewhere; R = L^T
  // fsc: ||L^{-1} D^{-1}||_F^2 with D^{-2} = diag(G + shift I), the same bound for the column-equilibrated
  // Gram matrix D (G + shift I) D, whose trace is n
  double fro = 0.0, fsc = 0.0;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    const double x = (i < n && j < n) ? X[j * ld + i] : 0.0;
    Rinv[e] = x;
    fro += x * x;
    if (single && i < n) fsc += x * x * (G[i * s + i] + shift);
  }
  if (single) fsc = block_sum(fsc, red);
  if (ok) {
    // certify that no singular value ratio of the block is at or below the drop tolerance, from guaranteed
    // bounds: lambda_min(G) = 1 / ||L^{-1}||_2^2 >= 1 / min(||L^{-1}||_F^2, ||L^{-1}||_1 ||L^{-1}||_inf) (Hoelder)
    // and lambda_max(G) <= min(trace(G), ||G||_inf); the norms of L^{-1} from its rows and columns in X
    const double f = block_sum(fro, red);
    double rmax = 0.0, cmax = 0.0, gmax = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
      double rs = 0.0, cs = 0.0, gs = 0.0;
      for (int j = 0; j < n; ++j) {
        rs += fabs(X[i * ld + j]);   // row i of L^{-1}
        cs += fabs(X[j * ld + i]);   // column i of L^{-1}
        gs += fabs(0.5 * (G[i * s + j] + G[j * s + i]));
      }
      rmax = fmax(rmax, rs);
      cmax = fmax(cmax, cs);
      gmax = fmax(gmax, gs);
    }
    red[threadIdx.x] = rmax;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    rmax = red[0];
    __syncthreads();
    red[threadIdx.x] = cmax;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    cmax = red[0];
    __syncthreads();
    red[threadIdx.x] = gmax;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    gmax = red[0];
    __syncthreads();
    const double lmin = 1.0 / fmin(f, rmax * cmax);
    lmax_c = fmin(tr, gmax);
    if (threadIdx.x == 0) {
      const int okb = (sinfo == 0 && lmin > certify * lmax_c) ? 1 : 0;
      ok[b] = okb;
      refine = sinfo == 0 && !okb;
      if (single) single[b] = (sinfo == 0 && fsc > 0.0 && 1.0 / fsc > single_thr * n) ? 1 : 0;
    }
  }
  __syncthreads();
  // the norm bounds above are loose by up to a factor of about n each: where they fail, the Cholesky of
  // G + shift I - tau I with tau = certify * lambda_max bound + its backward-error bound decides; success proves
  // lambda_min > certify * lambda_max (the factor in A is no longer needed once Rinv and Racc are out)
  auto refine_certificate = [&]() {
    if (!ok || !refine) return;
    const double g = double(n + 1) * 0x1p-53 / (1.0 - double(n + 1) * 0x1p-53);
    const double tau = certify * lmax_c + 1.01 * g * (tr + double(n) * shift);
    __syncthreads();
    for (int e = threadIdx.x; e < np * np; e += NT) {
      const int i = e / np, j = e - i * np;
      A[i * ld + j] = (i < n && j < n) ? 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift - tau : 0.0)
                                       : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    const int info2 = chol_blocked(A, np, ld, w.Dinv, w.Pn, &sinfo);
    if (threadIdx.x == 0) ok[b] = info2 == 0 ? 1 : 0;
  };
  if (init) {
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const int i = e / s, j = e % s;
      Racc[e] = (i < n && j < n && j >= i) ? A[j * ld + i] : 0.0;
    }
    refine_certificate();
    return;
  }
  // Racc <- R * Racc (R = L^T), with Racc staged in X (zero-padded)
  for (int e = threadIdx.x; e < np * np; e += NT) {
    const int i = e / np, j = e - i * np;
    X[i * ld + j] = (i < n && j < n) ? Racc[i * s + j] : 0.0;
  }
  __syncthreads();
  const int nt = np / NB;
  for (int t = wave; t < nt * nt; t += NW) {
    const int ti = t / nt, tj = t - ti * nt;
    sv4d acc = {0.0, 0.0, 0.0, 0.0};
    acc = mma16(acc, A + NB * ti, 1, ld, X + NB * tj, ld, 1, np);  // R(i, m) = L(m, i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = NB * ti + tile_row(v), j = NB * tj + tile_col();
      if (i < s && j < s) Racc[i * s + j] = (i < n && j < n && j >= i) ? acc[v] : 0.0;
    }
  }
  // rows and columns of Racc beyond the padded tiles (none when s <= np) are zero
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    if (i >= np || j >= np) Racc[e] = 0.0;
  }
  refine_certificate();
}

// Nystrom core of one problem.  C = Omega^T Y (s x s) and the Cholesky-QR factor R of Y give
// T = R C_1^+ R^T over the eigenpairs of sym(C) with lambda >= eps_rel lambda_max, whose EVD yields the
// basis.  When a Cholesky C = L L^T succeeds with 1/||L^{-1}||_F^2 >= eps_rel trace(C) (a lower bound of
// lambda_min against an upper bound of lambda_max), every eigenpair passes the threshold and
// T = R C^{-1} R^T = H^T H with H = L^{-1} R^T: the EVD of C is skipped.
template <int kLds>
__global__ __launch_bounds__(NT) void k_small_nystrom(int s, int k, const double* C, const double* R, double eps_rel,
                                                      double* Wk, double* Ek, int* out, double* gw, int64_t gws,
                                                      const int* run_if) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  __shared__ double dkeep[SMAX];
  __shared__ int ikeep[SMAX];
  __shared__ int nkeep, sinfo;
  const int b = blockIdx.x;
  if (run_if && run_if[b] != 1) return;  // (the packed kernels served this problem)
  const int wave = threadIdx.x >> 6;
  C += b * int64_t(s) * s;
  R += b * int64_t(s) * s;
  Wk += b * int64_t(s) * k;
  Ek += b * int64_t(k);
  out += 2 * b;
  CholWs cw = chol_carve(kLds ? sm : gw + b * gws, s, s);  // regions L and X double as the EVD's matrices
  const int np = cw.rp, ld = cw.ldl;
  double* A = cw.L;
  double* V = cw.X;
  double* cs = sd;
  double* d = sd + 2 * s;
  int* pr = si;
  int* ord = si + 2 * s;
  for (int e = threadIdx.x; e < np * np; e += NT) {  // symmetrised C, identity-padded
    const int i = e / np, j = e - i * np;
    A[i * ld + j] = (i < s && j < s) ? 0.5 * (C[i * s + j] + C[j * s + i]) : (i == j ? 1.0 : 0.0);
  }
  double tr = 0.0;
  for (int i = threadIdx.x; i < s; i += NT) tr += C[i * s + i];
  tr = block_sum(tr, red);
  const int info = chol_blocked(A, np, ld, cw.Dinv, cw.Pn, &sinfo);
  bool certified = false;
  if (info == 0) {
    tri_inverse_blocked(A, np, ld, cw.Dinv, V, cw.Tb);  // V = L^{-1}
    double fro = 0.0;
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const double x = V[(e / s) * ld + e % s];
      fro += x * x;
    }
    fro = block_sum(fro, red);
    certified = tr > 0.0 && 1.0 / fro >= eps_rel * tr;
  }
  double* Tm;  // T
  double* Ev;  // its eigenvectors
  int r;
  if (certified) {
    r = s;
    for (int e = threadIdx.x; e < np * np; e += NT) {  // V = R^T (zero-padded)
      const int i = e / np, j = e - i * np;
      V[i * ld + j] = (i < s && j < s) ? R[j * s + i] : 0.0;
    }
    __syncthreads();
    // H = L^{-1} R^T: the forward block sweep of chol_solve_blocked
    for (int bk = 0; bk < np / NB; ++bk) {
      const int i0 = bk * NB, lt = np + 1;
      const double* Di = cw.Dinv + bk * (NB * NBL);
      for (int jt = wave; jt < np / NB; jt += NW) {
        sv4d acc = {0.0, 0.0, 0.0, 0.0};
        acc = mma16(acc, A + i0 * ld, ld, 1, V + NB * jt, ld, 1, i0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = tile_row(v), j = NB * jt + tile_col();
          cw.Tb[a * lt + j] = V[(i0 + a) * ld + j] - acc[v];
        }
      }
      __syncthreads();
      for (int jt = wave; jt < np / NB; jt += NW) {
        sv4d acc = {0.0, 0.0, 0.0, 0.0};
        acc = mma16(acc, Di, NBL, 1, cw.Tb + NB * jt, lt, 1, NB);
#pragma unroll
        for (int v = 0; v < 4; ++v) V[(i0 + tile_row(v)) * ld + NB * jt + tile_col()] = acc[v];
      }
      __syncthreads();
    }
    // T = H^T H into A (the factor is no longer needed)
    const int nt = np / NB;
    for (int t = wave; t < nt * nt; t += NW) {
      const int ti = t / nt, tj = t - ti * nt;
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, V + NB * ti, 1, ld, V + NB * tj, ld, 1, np);
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(NB * ti + tile_row(v)) * ld + NB * tj + tile_col()] = acc[v];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < s * s; e += NT) {  // exact symmetry
      const int i = e / s, j = e % s;
      if (j < i) {
        const double x = 0.5 * (A[i * ld + j] + A[j * ld + i]);
        A[i * ld + j] = x;
        A[j * ld + i] = x;
      }
    }
    __syncthreads();
    Tm = A;
    Ev = V;
  } else {
    for (int e = threadIdx.x; e < s * s; e += NT) {  // symmetrised C again (the factorisation overwrote it)
      const int i = e / s, j = e % s;
      A[i * ld + j] = 0.5 * (C[i * s + j] + C[j * s + i]);
    }
    __syncthreads();
    jacobi(A, V, s, ld, cs, pr, red);
    for (int i = threadIdx.x; i < s; i += NT) d[i] = A[i * ld + i];
    __syncthreads();
    if (threadIdx.x == 0) {
      double dmax = d[0];
      for (int i = 1; i < s; ++i) dmax = d[i] > dmax ? d[i] : dmax;
      int q = 0;
      if (dmax > 0.0)
        for (int i = 0; i < s; ++i)
          if (d[i] >= eps_rel * dmax) {
            ikeep[q] = i;
            dkeep[q] = d[i];
            ++q;
          }
      nkeep = q;
    }
    __syncthreads();
    r = nkeep;
    // M = R V_1 (s x r) into A (stride ld >= r)
    for (int e = threadIdx.x; e < s * r; e += NT) {
      const int i = e / r, c = e % r;
      double acc = 0.0;
      for (int m = i; m < s; ++m) acc += R[i * s + m] * V[m * ld + ikeep[c]];
      A[i * ld + c] = acc;
    }
    __syncthreads();
    // T = M D_1^{-1} M^T into V, symmetric by construction of the sum
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const int i = e / s, j = e % s;
      if (j > i) continue;
      double acc = 0.0;
      for (int c = 0; c < r; ++c) acc += A[i * ld + c] * A[j * ld + c] / dkeep[c];
      V[i * ld + j] = acc;
      V[j * ld + i] = acc;
    }
    __syncthreads();
    Tm = V;
    Ev = A;
  }
  jacobi(Tm, Ev, s, ld, cs, pr, red);  // EVD of T
  for (int i = threadIdx.x; i < s; i += NT) d[i] = Tm[i * ld + i];
  __syncthreads();
  sort_desc(d, s, ord);
  const int kk = k < r ? k : r;
  for (int e = threadIdx.x; e < s * k; e += NT) {
    const int i = e / k, c = e % k;
    Wk[e] = c < kk ? Ev[i * ld + ord[c]] : 0.0;
  }
  for (int c = threadIdx.x; c < k; c += NT) Ek[c] = c < kk ? d[ord[c]] : 0.0;
  if (threadIdx.x == 0) {
    out[0] = r;
    out[1] = kk;
  }
}


template <int kLds>
__global__ __launch_bounds__(NT) void k_small_sym_evd(int m, const double* Ain, double* W, double* E, double* gw) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  EvdSpace w = evd_space(m, kLds ? sm : gw, sd, si);
  const int ld = w.ld;
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e / m, j = e % m;
    w.A[i * ld + j] = 0.5 * (Ain[i * m + j] + Ain[j * m + i]);
  }
  __syncthreads();
  jacobi(w.A, w.V, m, ld, w.cs, w.pr, red);
  for (int i = threadIdx.x; i < m; i += NT) w.d[i] = w.A[i * ld + i];
  __syncthreads();
  sort_desc(w.d, m, w.ord);
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e / m, c = e % m;
    W[e] = w.V[i * ld + w.ord[c]];
  }
  for (int c = threadIdx.x; c < m; c += NT) E[c] = w.d[w.ord[c]];
}

// Generalised symmetric eigenproblem A c = lambda B c, step 1: B = L L^T (Cholesky), Linv = L^{-1},
// M = Linv sym(A) Linv^T (all k x k row-major in global memory; one workgroup).
__global__ __launch_bounds__(NT) void k_gevd_reduce(int k, const double* A, const double* B, double* L,
                                                    double* Linv, double* M, int* flag) {
  __shared__ int sinfo;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int e = threadIdx.x; e < k * k; e += NT) {
    const int i = e / k, j = e % k;
    L[e] = 0.5 * (B[i * k + j] + B[j * k + i]);
    Linv[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  if (chol_dev(L, k, k, &sinfo) && threadIdx.x == 0) flag[0] = 1;
  for (int m = 0; m < k; ++m) {  // Linv = L^{-1} by a forward sweep on the identity
    const double inv = 1.0 / L[m * k + m];
    for (int j = threadIdx.x; j <= m; j += NT) Linv[m * k + j] *= inv;
    __syncthreads();
    for (int i = m + 1 + ty; i < k; i += 32) {
      const double l = L[i * k + m];
      for (int j = tx; j <= m; j += 32) Linv[i * k + j] -= l * Linv[m * k + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < k * k; e += NT) {  // L <- Linv sym(A)  (L is no longer needed)
    const int i = e / k, j = e % k;
    double acc = 0.0;
    for (int c = 0; c <= i; ++c) acc += Linv[i * k + c] * 0.5 * (A[c * k + j] + A[j * k + c]);
    L[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * k; e += NT) {  // M = (Linv sym(A)) Linv^T
    const int i = e / k, j = e % k;
    double acc = 0.0;
    for (int c = 0; c <= j; ++c) acc += L[i * k + c] * Linv[j * k + c];
    M[e] = acc;
  }
}

// step 3: ascending order; C = Linv^T W (B-orthonormal eigenvectors), Cl = -C diag(lambda)
__global__ void k_gevd_back(int k, const double* Linv, const double* W, const double* E, double* lam, double* C,
                            double* Cl) {
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;  // C(i, j): column j <- eigenpair k - 1 - j of the descending EVD
    const int jj = k - 1 - j;
    double acc = 0.0;
    for (int c = i; c < k; ++c) acc += Linv[c * k + i] * W[c * k + jj];
    C[e] = acc;
    Cl[e] = -acc * E[jj];
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) lam[j] = E[k - 1 - j];
}

// ---------------------------------------------------------------- packed tiles (s up to 160 past the LDS limit)
// When the dense workspaces above exceed the LDS, the Cholesky kernels keep only the lower 16 x 16 tiles of the
// factor, packed in LDS: tile (i, j), i >= j, at index i (i + 1) / 2 + j, rows of PTL = 17 doubles (bank
// spread).  The triangular solves then run one 16-column chunk per wave with the whole chunk in registers: the
// FP64 MFMA accumulator layout (element v of lane l is row 4 v + l / 16, column l % 16) is also the B-operand
// layout of the k-steps 4 v .. 4 v + 3 of the same tile, so each solved tile feeds the next tile rows'
// products directly and only the factor is read from LDS.  No workgroup barrier inside a sweep.
constexpr int NTP = 512;         // threads of the packed kernels: 2 waves per SIMD leave 256 VGPRs for a chunk
constexpr int NWP = NTP / 64;
constexpr int PTL = NB + 1;
constexpr int PTS = NB * PTL;
constexpr int PNT = 10;           // tile rows of the largest packed factor
constexpr int PSMAX = PNT * NB;   // 160
__host__ __device__ inline int ptile_count(int nt) { return nt * (nt + 1) / 2; }
__host__ __device__ inline size_t ptiles_elems(int nt) {
  return size_t(ptile_count(nt)) * PTS + size_t(nt) * NB * NBL;  // tiles + diagonal-tile inverses
}
__device__ __forceinline__ double* ptile(double* pt, int i, int j) { return pt + (i * (i + 1) / 2 + j) * PTS; }
__device__ __forceinline__ const double* ptile(const double* pt, int i, int j) {
  return pt + (i * (i + 1) / 2 + j) * PTS;
}
__device__ __forceinline__ int tri_row(int u) {  // row of the u-th entry of a row-wise packed lower triangle
  int t = 0;
  while ((t + 1) * (t + 2) / 2 <= u) ++t;
  return t;
}

// Lower tiles of an n x n matrix, padded with the identity to nt tiles: val(i, j) for i, j < n.  Eight values
// per thread are loaded (from clamped, in-bounds positions) before the first is stored.
template <class F>
__device__ __forceinline__ void ptiles_fill(double* pt, int n, int nt, F val) {
  const int ne = ptile_count(nt) * NB * NB;
  for (int e0 = threadIdx.x; e0 < ne; e0 += 8 * NTP) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + u * NTP, ne - 1);
      const int t = e >> 8, a = (e >> 4) & 15, c = e & 15;
      const int ti = tri_row(t), tj = t - ti * (ti + 1) / 2;
      v[u] = val(min(ti * NB + a, n - 1), min(tj * NB + c, n - 1));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NTP;
      if (e < ne) {
        const int t = e >> 8, a = (e >> 4) & 15, c = e & 15;
        const int ti = tri_row(t), tj = t - ti * (ti + 1) / 2;
        const int i = ti * NB + a, j = tj * NB + c;
        pt[t * PTS + a * PTL + c] = (i < n && j < n) ? v[u] : (i == j ? 1.0 : 0.0);
      }
    }
  }
}

// Right-looking Cholesky on the packed tiles (lower parts of the diagonal tiles and the tiles below are the
// factor on return; Dinv: inverses of the diagonal tiles).  Returns 0 or the 1-based first pivot <= 0.
__device__ __forceinline__ int chol_ptiles(double* pt, int nt, double* Dinv, int* sinfo) {
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) *sinfo = 0;
  __syncthreads();
  // one step of look-ahead: wave 0 updates the next diagonal tile first and factors it while the other waves
  // update the rest of the trailing tiles (the serial 16x16 factor no longer waits for the whole update)
  auto diag = [&](int j) {
    const int bad = diag_factor_wave(ptile(pt, j, j), PTL, 0, NB, Dinv + j * (NB * NBL));
    if (bad && (threadIdx.x & 63) == 0 && *sinfo == 0) *sinfo = j * NB + bad;
  };
  auto update = [&](int j, int u) {  // A_iq -= L_ij L_qj^T for the u-th lower tile of the trailing matrix
    const int ti = tri_row(u), tq = u - ti * (ti + 1) / 2;
    const int i = j + 1 + ti, q = j + 1 + tq;
    sv4d acc = {0.0, 0.0, 0.0, 0.0};
    acc = mma16(acc, ptile(pt, i, j), PTL, 1, ptile(pt, q, j), 1, PTL, NB);
    double* T = ptile(pt, i, q);
#pragma unroll
    for (int v = 0; v < 4; ++v) T[tile_row(v) * PTL + tile_col()] -= acc[v];
  };
  if (wave == 0) diag(0);
  __syncthreads();
  for (int j = 0; j < nt; ++j) {
    const double* Di = Dinv + j * (NB * NBL);
    for (int i = j + 1 + wave; i < nt; i += NWP) {  // L_ij = A_ij L_jj^{-T}
      double* T = ptile(pt, i, j);
      sv4d acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma16(acc, T, PTL, 1, Di, 1, NBL, NB);
#pragma unroll
      for (int v = 0; v < 4; ++v) T[tile_row(v) * PTL + tile_col()] = acc[v];
    }
    __syncthreads();
    const int mt = nt - j - 1;
    if (mt > 0) {
      if (wave == 0) {  // tile (j + 1, j + 1), then its factor (LDS accesses of one wave complete in order)
        update(j, 0);
        diag(j + 1);
      } else {
        for (int u = wave; u < ptile_count(mt); u += NWP - 1) update(j, u);
      }
    }
    __syncthreads();
  }
  const int info = *sinfo;
  __syncthreads();
  return info;
}

// Inverses of the diagonal tiles of an existing packed factor, one wave per tile.
__device__ __forceinline__ void ptiles_diag_inverses(const double* pt, int nt, double* Dinv) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int bk = wave; bk < nt; bk += NWP) {
    const double* T = ptile(pt, bk, bk);
    double x[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double acc = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < i; ++t) acc -= T[i * PTL + t] * x[t];
      x[i] = acc / T[i * PTL + i];
    }
    if (lane < NB) {
#pragma unroll
      for (int i = 0; i < NB; ++i) Dinv[bk * (NB * NBL) + i * NBL + lane] = x[i];
    }
  }
  __syncthreads();
}

// One wave, one 16-column chunk in registers: X <- L^{-1} X (tiles before i0 are zero and stay zero).
__device__ __forceinline__ void wave_fwd(const double* pt, const double* Dinv, int nt, int i0, sv4d (&X)[PNT]) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int i = 0; i < PNT; ++i) {
    if (i < i0 || i >= nt) continue;
    sv4d sum = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < PNT; ++k) {
      if (k >= i0 && k < i) {
        const double* T = ptile(pt, i, k) + li * PTL + lk;
#pragma unroll
        for (int v = 0; v < 4; ++v) sum = __builtin_amdgcn_mfma_f64_16x16x4f64(T[4 * v], X[k][v], sum, 0, 0, 0);
      }
    }
    const sv4d t = X[i] - sum;
    const double* Di = Dinv + i * (NB * NBL) + li * NBL + lk;
    sv4d y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) y = __builtin_amdgcn_mfma_f64_16x16x4f64(Di[4 * v], t[v], y, 0, 0, 0);
    X[i] = y;
    __builtin_amdgcn_sched_barrier(0);  // one tile row's operand loads at a time (register pressure)
  }
}

// One wave, one chunk in registers: X <- L^{-T} X.
__device__ __forceinline__ void wave_bwd(const double* pt, const double* Dinv, int nt, sv4d (&X)[PNT]) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int i = PNT - 1; i >= 0; --i) {
    if (i >= nt) continue;
    sv4d sum = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < PNT; ++k) {
      if (k > i && k < nt) {
        const double* T = ptile(pt, k, i) + lk * PTL + li;  // (L_ki)^T (li, 4 v + lk) = L_ki (4 v + lk, li)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sum = __builtin_amdgcn_mfma_f64_16x16x4f64(T[4 * v * PTL], X[k][v], sum, 0, 0, 0);
      }
    }
    const sv4d t = X[i] - sum;
    const double* Di = Dinv + i * (NB * NBL) + lk * NBL + li;
    sv4d y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) y = __builtin_amdgcn_mfma_f64_16x16x4f64(Di[4 * v * NBL], t[v], y, 0, 0, 0);
    X[i] = y;
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// Workgroup sum / max through one value per wave (red: NWP doubles); every thread gets the result.
__device__ __forceinline__ double group_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NWP; ++w) r += red[w];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double group_max(double v, double* red) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
#pragma unroll
  for (int w = 1; w < NWP; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// k_small_chol_solve for factors of 17..160 rows whose dense workspace exceeds the LDS: same arguments and
// results; the factor is packed in LDS and each wave solves 16-column chunks of the right-hand sides.
__global__ __launch_bounds__(NTP) void k_small_chol_solve_p(int r0, const int* __restrict__ dims, double* D,
                                                           int64_t sD, const double* B, int64_t ldb, int64_t sB,
                                                           double* X, int64_t ldx, int64_t sX, int s, int s0,
                                                           double alpha, int* flag, int factor) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  const int b = blockIdx.x;
  const int r = dims ? dims[b] : r0;
  D += b * sD;
  B += b * sB;
  X += b * sX;
  for (int e = threadIdx.x; e < (s0 - r) * s; e += NTP) X[(r + e / s) * ldx + e % s] = 0.0;
  if (r == 0) return;
  const int nt = (r + NB - 1) / NB;
  double* pt = sm;
  double* Dinv = sm + size_t(ptile_count(nt)) * PTS;
  ptiles_fill(pt, r, nt, [&](int i, int j) { return D[i * r0 + j]; });
  __syncthreads();
  if (factor) {
    if (chol_ptiles(pt, nt, Dinv, &sinfo) && threadIdx.x == 0) flag[0] = 1;
    for (int e = threadIdx.x; e < r * r; e += NTP) {
      const int i = e / r, j = e - i * r;
      D[i * r0 + j] = j <= i ? ptile(pt, i / NB, j / NB)[(i % NB) * PTL + j % NB] : 0.0;
    }
  } else {
    ptiles_diag_inverses(pt, nt, Dinv);
  }
  if (s == 0) return;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  for (int c0 = wave * NB; c0 < s; c0 += NWP * NB) {
    const int col = c0 + li;
    const bool cin = col < s;
    const int cc = min(col, s - 1), ldb32 = int(ldb);
    sv4d Xr[PNT];
    // loads from clamped, in-bounds rows (32-bit offsets from the problem's base), half the tiles at a time;
    // out-of-range values zeroed afterwards
#pragma unroll
    for (int i = 0; i < PNT / 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) Xr[i][v] = B[min(NB * i + 4 * v + lk, r - 1) * ldb32 + cc];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = PNT / 2; i < PNT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) Xr[i][v] = B[min(NB * i + 4 * v + lk, r - 1) * ldb32 + cc];
#pragma unroll
    for (int i = 0; i < PNT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = NB * i + 4 * v + lk;
        if (!(i < nt && row < r && cin)) Xr[i][v] = 0.0;
      }
    wave_fwd(pt, Dinv, nt, 0, Xr);
    wave_bwd(pt, Dinv, nt, Xr);
#pragma unroll
    for (int i = 0; i < PNT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = NB * i + 4 * v + lk;
        if (i < nt && row < r && cin) X[row * ldx + col] = alpha * Xr[i][v];
      }
  }
}

// The triangular solves of k_small_chol_solve_p with an existing factor (D holds L, zero above the diagonal),
// one 16-column chunk of the right-hand sides per workgroup (grid: chunks x problems), so that the chunks run
// on as many compute units instead of two rounds on one: every workgroup packs the factor into LDS and inverts
// its diagonal tiles, then its first wave sweeps its chunk forward and backward in registers.
__global__ __launch_bounds__(NTP) void k_small_chol_apply_p(int r0, const int* __restrict__ dims, const double* D,
                                                           int64_t sD, const double* B, int64_t ldb, int64_t sB,
                                                           double* X, int64_t ldx, int64_t sX, int s, int s0,
                                                           double alpha) {
  extern __shared__ double sm[];
  const int b = blockIdx.y;
  const int r = dims ? dims[b] : r0;
  const int c0 = blockIdx.x * NB;
  D += b * sD;
  B += b * sB;
  X += b * sX;
  for (int e = threadIdx.x; e < (s0 - r) * NB; e += NTP) {  // rows past the problem's dimension: zero
    const int col = c0 + e % NB;
    if (col < s) X[(r + e / NB) * ldx + col] = 0.0;
  }
  if (r == 0) return;
  const int nt = (r + NB - 1) / NB;
  double* pt = sm;
  double* Dinv = sm + size_t(ptile_count(nt)) * PTS;
  ptiles_fill(pt, r, nt, [&](int i, int j) { return D[i * r0 + j]; });
  __syncthreads();
  ptiles_diag_inverses(pt, nt, Dinv);
  if ((threadIdx.x >> 6) != 0) return;
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  const int col = c0 + li;
  const bool cin = col < s;
  const int cc = min(col, s - 1), ldb32 = int(ldb);
  sv4d Xr[PNT];
  // loads from clamped, in-bounds rows, half the tiles at a time; out-of-range values zeroed afterwards
#pragma unroll
  for (int i = 0; i < PNT / 2; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) Xr[i][v] = B[min(NB * i + 4 * v + lk, r - 1) * ldb32 + cc];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = PNT / 2; i < PNT; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) Xr[i][v] = B[min(NB * i + 4 * v + lk, r - 1) * ldb32 + cc];
#pragma unroll
  for (int i = 0; i < PNT; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = NB * i + 4 * v + lk;
      if (!(i < nt && row < r && cin)) Xr[i][v] = 0.0;
    }
  wave_fwd(pt, Dinv, nt, 0, Xr);
  wave_bwd(pt, Dinv, nt, Xr);
#pragma unroll
  for (int i = 0; i < PNT; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = NB * i + 4 * v + lk;
      if (i < nt && row < r && cin) X[row * ldx + col] = alpha * Xr[i][v];
    }
}

// k_small_cholqr for 17..160 columns whose dense workspace exceeds the LDS: same arguments and results.  The
// factor is packed in LDS; each wave forms block columns of L^{-1} in registers (writing Rinv and the norms of
// the certificate from them); R Racc is staged through the caller's global scratch gw (s x s per problem).
__global__ __launch_bounds__(NTP) void k_small_cholqr_p(int s, const int* __restrict__ dims, const double* G,
                                                       int64_t sG, const double* shift_coef, double* Rinv,
                                                       double* Racc, int init, int* flag, double* gw, int64_t gws,
                                                       double certify, int* ok, double single_thr, int* single) {
  extern __shared__ double sm[];
  __shared__ int sinfo, refine;
  __shared__ double red[NWP];
  __shared__ double rowsum[PSMAX];
  double lmax_c = 0.0;
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : s;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  G += b * sG;
  Rinv += b * int64_t(s) * s;
  Racc += b * int64_t(s) * s;
  if (n == 0) {
    for (int e = threadIdx.x; e < s * s; e += NTP) Rinv[e] = Racc[e] = 0.0;
    if (ok && threadIdx.x == 0) ok[b] = 0;
    if (single && threadIdx.x == 0) single[b] = 0;
    return;
  }
  double tr = 0.0;
  for (int i = threadIdx.x; i < n; i += NTP) tr += G[i * s + i];
  if (threadIdx.x == 0) refine = 0;
  tr = group_sum(tr, red);
  const double shift = (shift_coef ? shift_coef[b] : 0.0) * tr;
  const int nt = (n + NB - 1) / NB, np = nt * NB;
  double* pt = sm;
  double* Dinv = sm + size_t(ptile_count(nt)) * PTS;
  ptiles_fill(pt, n, nt, [&](int i, int j) { return 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift : 0.0); });
  for (int i = threadIdx.x; i < PSMAX; i += NTP) rowsum[i] = 0.0;
  __syncthreads();
  // ||sym(G)||_inf from the tiles (unshifted), before the factorisation overwrites them
  double gmax = 0.0;
  if (ok) {
    for (int i = threadIdx.x; i < n; i += NTP) {
      const int ti = i / NB, a = i % NB;
      double gs = 0.0;
      for (int tj = 0; tj < nt; ++tj) {
        double x[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c)  // row i of tile (ti, tj), or column i of tile (tj, ti) above the diagonal
          x[c] = tj <= ti ? ptile(pt, ti, tj)[a * PTL + c] : ptile(pt, tj, ti)[c * PTL + a];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const int j = tj * NB + c;
          if (j < n) gs += fabs(j == i ? x[c] - shift : x[c]);
        }
      }
      gmax = fmax(gmax, gs);
    }
  }
  __syncthreads();
  if (chol_ptiles(pt, nt, Dinv, &sinfo) && threadIdx.x == 0) flag[0] = 1;
  for (int e = threadIdx.x; e < nt * NB * NB; e += NTP) {  // the factorisation leaves values above the diagonal
    const int j = e >> 8, a = (e >> 4) & 15, c = e & 15;
    if (c > a) ptile(pt, j, j)[a * PTL + c] = 0.0;
  }
  __syncthreads();
  // Rinv = (L^{-1})^T in the leading n x n block, zero elsewhere; Frobenius, column and row sums of |L^{-1}|
  double fro = 0.0, fsc = 0.0, cmax = 0.0;  // fsc: as fro for the column-equilibrated Gram matrix
  for (int j = wave; j < nt; j += NWP) {
    sv4d Xr[PNT];
#pragma unroll
    for (int i = 0; i < PNT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) Xr[i][v] = (i == j && 4 * v + lk == li) ? 1.0 : 0.0;
    wave_fwd(pt, Dinv, nt, j, Xr);
    const int col = NB * j + li;
    const double gcc = G[min(col, n - 1) * s + min(col, n - 1)] + shift;
    double csum = 0.0, cf = 0.0;
#pragma unroll
    for (int i = 0; i < PNT; ++i) {
      if (i >= nt) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = NB * i + 4 * v + lk;
        const double x = (row < n && col < n) ? Xr[i][v] : 0.0;
        if (row < s && col < s) Rinv[col * s + row] = x;
        cf += x * x;
        csum += fabs(x);
        if (row < n && x != 0.0) atomicAdd(&rowsum[row], fabs(x));
      }
    }
    fro += cf;
    fsc += cf * gcc;
    csum += __shfl_xor(csum, 16);
    csum += __shfl_xor(csum, 32);
    cmax = fmax(cmax, csum);
  }
  for (int e = threadIdx.x; e < s * s; e += NTP) {  // rows and columns past the tiles
    const int i = e / s, j = e - i * s;
    if (i >= np || j >= np) Rinv[e] = 0.0;
  }
  fro = group_sum(fro, red);
  fsc = group_sum(fsc, red);
  cmax = group_max(cmax, red);
  if (ok) {
    double rmax = 0.0;
    for (int i = threadIdx.x; i < n; i += NTP) rmax = fmax(rmax, rowsum[i]);
    rmax = group_max(rmax, red);
    gmax = group_max(gmax, red);
    const double lmin = 1.0 / fmin(fro, rmax * cmax);
    lmax_c = fmin(tr, gmax);
    if (threadIdx.x == 0) {
      const int okb = (sinfo == 0 && lmin > certify * lmax_c) ? 1 : 0;
      ok[b] = okb;
      refine = sinfo == 0 && !okb;
      if (single) single[b] = (sinfo == 0 && fsc > 0.0 && 1.0 / fsc > single_thr * n) ? 1 : 0;
    }
  }
  __syncthreads();
  // where the norm bounds fail, the Cholesky of G + shift I - tau I decides (as in k_small_cholqr)
  auto refine_certificate = [&]() {
    if (!ok || !refine) return;
    const double g = double(n + 1) * 0x1p-53 / (1.0 - double(n + 1) * 0x1p-53);
    const double tau = certify * lmax_c + 1.01 * g * (tr + double(n) * shift);
    __syncthreads();
    ptiles_fill(pt, n, nt, [&](int i, int j) {
      return 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift - tau : 0.0);
    });
    __syncthreads();
    const int info2 = chol_ptiles(pt, nt, Dinv, &sinfo);
    if (threadIdx.x == 0) ok[b] = info2 == 0 ? 1 : 0;
  };
  if (init) {
    for (int e = threadIdx.x; e < s * s; e += NTP) {
      const int i = e / s, j = e - i * s;
      Racc[e] = (i < n && j < n && j >= i) ? ptile(pt, j / NB, i / NB)[(j % NB) * PTL + i % NB] : 0.0;
    }
    refine_certificate();
    return;
  }
  // Racc <- R Racc, R = L^T upper: output tile (ti, tj), ti <= tj, sums over the tiles m = ti .. tj
  double* Ra = gw + b * gws;
  for (int e0 = threadIdx.x; e0 < np * np; e0 += 8 * NTP) {
    double v8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + u * NTP, np * np - 1);
      const int i = e / np, j = e - i * np;
      v8[u] = Racc[min(i, n - 1) * s + min(j, n - 1)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NTP;
      if (e < np * np) {
        const int i = e / np, j = e - i * np;
        Ra[e] = (i < n && j < n) ? v8[u] : 0.0;
      }
    }
  }
  __syncthreads();
  for (int u = wave; u < nt * nt; u += NWP) {
    const int ti = u / nt, tj = u - ti * nt;
    double q[PNT][4];  // the B operands of every k-step, loaded together
#pragma unroll
    for (int m = 0; m < PNT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int mm = min(max(m, ti), tj);
        q[m][v] = Ra[int64_t(NB * mm + 4 * v + lk) * np + NB * tj + li];
      }
    sv4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < PNT; ++m) {
      if (m < ti || m > tj) continue;
      const double* T = ptile(pt, m, ti) + lk * PTL + li;  // R(ti, m) (li, 4 v + lk) = L(m, ti) (4 v + lk, li)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[4 * v * PTL], q[m][v], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = NB * ti + tile_row(v), j = NB * tj + tile_col();
      if (i < s && j < s) Racc[i * s + j] = (i < n && j < n && j >= i) ? acc[v] : 0.0;
    }
  }
  for (int e = threadIdx.x; e < s * s; e += NTP) {
    const int i = e / s, j = e % s;
    if (i >= np || j >= np) Racc[e] = 0.0;
  }
  refine_certificate();
}

// ---------------------------------------------------------------- packed Jacobi (n up to 160 past the LDS limit)
// The eigen-decompositions keep the lower triangle of the symmetric matrix packed by rows in LDS (element
// (i, j), i >= j, at i (i + 1) / 2 + j: 103 KB at n = 160) and write each round's rotations (c, s) to a log in
// global memory instead of applying them to V; k_jacobi_rows then forms rows of V = J_1 J_2 ... (the
// identity's rows with every logged round applied in order), one wave per row, in parallel over the rows.
// Rounds follow the same round-robin ordering and rotation formulas as jacobi() above.
constexpr int JSWEEPS_P = 40;  // sweep limit of the packed Jacobi (bounds the log)
__host__ __device__ inline int64_t jlog_stride(int n) {  // header (rounds, kept), order, scales, rotations
  const int m = n + (n & 1);
  return int64_t(2 + 2 * n + 1) / 2 * 2 + int64_t(JSWEEPS_P) * (m - 1) * m;
}
__device__ __forceinline__ int pidx(int i, int j) {
  return i >= j ? ((i * (i + 1)) >> 1) + j : ((j * (j + 1)) >> 1) + i;
}
__device__ __forceinline__ int tri_row_fast(int e) {
  int i = int((sqrt(8.0 * double(e) + 1.0) - 1.0) * 0.5);
  while (((i + 1) * (i + 2)) / 2 <= e) ++i;
  while ((i * (i + 1)) / 2 > e) --i;
  return i;
}
__device__ __forceinline__ int rr_pos(int x, int round, int m) { return x == 0 ? 0 : 1 + (x - 1 + round) % (m - 1); }

// Cyclic Jacobi on the packed lower triangle A (n x n); rotations logged at rot[round * m + 2 t + {0, 1}].
// Returns the number of rounds run (stops at the rounding floor, after JSWEEPS_P sweeps at most).
__device__ int jacobi_packed(double* A, int n, double* cs, int* pr, double* red, double* rot) {
  const int tid = threadIdx.x;
  if (n < 2) return 0;
  const int m = n + (n & 1), half = m / 2, nblk = half * (half + 1) / 2, ne = n * (n + 1) / 2;
  int rounds = 0;
  for (int sweep = 0; sweep < JSWEEPS_P; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < ne; e += NT) {
      const int i = tri_row_fast(e), j = e - ((i * (i + 1)) >> 1);
      const double v = A[e] * A[e];
      tot += i == j ? v : 2.0 * v;
      if (i != j) off += 2.0 * v;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (!(off > 2e-31 * double(n) * double(n) * tot)) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < half) {
        int p = rr_pos(tid, round, m), q = rr_pos(m - 1 - tid, round, m);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[pidx(q, p)];
          const double app = A[pidx(p, p)], aqq = A[pidx(q, q)];
          if (apq * apq > 1e-36 * fabs(app * aqq) && fabs(apq) > 1e-300) {
            const double tau = (aqq - app) * rcp_nr(2.0 * apq);
            const double at = fabs(tau);
            double tf;
            if (at > 1e15) {
              tf = 0.5 * rcp_nr(at);
            } else {
              const double u = 1.0 + at * at;
              tf = rcp_nr(at + u * rsqrt_nr(u));
            }
            const double t = tau >= 0.0 ? tf : -tf;
            c = rsqrt_nr(1.0 + t * t);
            s = t * c;
          }
        }
        pr[2 * tid] = p;
        pr[2 * tid + 1] = q;
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
        rot[int64_t(rounds + round) * m + 2 * tid] = c;
        rot[int64_t(rounds + round) * m + 2 * tid + 1] = s;
      }
      __syncthreads();
      // A <- J^T A J on the stored 2 x 2 blocks (pair P rows, pair Q columns, P >= Q): as jacobi(), the
      // columns rotated first, then the rows
      for (int t = tid; t < nblk; t += NT) {
        const int P = tri_row_fast(t), Q = t - ((P * (P + 1)) >> 1);
        const int p = pr[2 * P], q = pr[2 * P + 1];
        const bool hq = q < n;
        const double c1 = cs[2 * P], s1 = cs[2 * P + 1];
        if (P == Q) {
          const double a = A[pidx(p, p)], b = hq ? A[pidx(q, p)] : 0.0, d = hq ? A[pidx(q, q)] : 0.0;
          const double a1 = c1 * a - s1 * b, b1 = s1 * a + c1 * b;
          const double c3 = c1 * b - s1 * d, d1 = s1 * b + c1 * d;
          A[pidx(p, p)] = c1 * a1 - s1 * c3;
          if (hq) {
            A[pidx(q, p)] = 0.5 * ((c1 * b1 - s1 * d1) + (s1 * a1 + c1 * c3));
            A[pidx(q, q)] = s1 * b1 + c1 * d1;
          }
        } else {
          const int p2 = pr[2 * Q], q2 = pr[2 * Q + 1];
          const bool hq2 = q2 < n;
          const double c2 = cs[2 * Q], s2 = cs[2 * Q + 1];
          const double a = A[pidx(p, p2)], b = hq2 ? A[pidx(p, q2)] : 0.0;
          const double c = hq ? A[pidx(q, p2)] : 0.0, d = (hq && hq2) ? A[pidx(q, q2)] : 0.0;
          const double a1 = c2 * a - s2 * b, b1 = s2 * a + c2 * b;
          const double c3 = c2 * c - s2 * d, d1 = s2 * c + c2 * d;
          A[pidx(p, p2)] = c1 * a1 - s1 * c3;
          if (hq2) A[pidx(p, q2)] = c1 * b1 - s1 * d1;
          if (hq) {
            A[pidx(q, p2)] = s1 * a1 + c1 * c3;
            if (hq2) A[pidx(q, q2)] = s1 * b1 + c1 * d1;
          }
        }
      }
      __syncthreads();
    }
    rounds += m - 1;
  }
  return rounds;
}

// Eigen-decomposition of sym(M) (n x n, problem b at M + b sM) on the packed triangle.  mode 0 (Nystrom core):
// eigenvalues descending, kept = min(k, n), E[c] = lambda_c for c < kept (zero up to k), out[2 b] = n,
// out[2 b + 1] = kept.  mode 1 (orthonormalisation): kept = leading eigenvalues > 0 and > drop2 lambda_max,
// scale_c = 1 / sqrt(lambda_c), out[b] = kept.  The log receives the rounds, kept, order and scales for
// k_jacobi_rows.  Problems with skip[b] == 1 are left alone.
__global__ __launch_bounds__(NT) void k_jacobi_p(int n, const double* M, int64_t sM, int mode, int k, double drop2,
                                                 double* E, int* out, const int* skip, double* jlog, int64_t jls) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double cs[PSMAX], d[PSMAX];
  __shared__ int pr[PSMAX], ord[PSMAX];
  const int b = blockIdx.x;
  if (skip && skip[b] == 1) return;
  M += b * sM;
  double* jl = jlog + b * jls;
  const int ne = n * (n + 1) / 2;
  for (int e = threadIdx.x; e < ne; e += NT) {
    const int i = tri_row_fast(e), j = e - ((i * (i + 1)) >> 1);
    sm[e] = i == j ? M[i * n + i] : 0.5 * (M[i * n + j] + M[j * n + i]);
  }
  __syncthreads();
  const int hdr = int(jlog_stride(n) - int64_t(JSWEEPS_P) * ((n + (n & 1)) - 1) * (n + (n & 1)));
  const int rounds = jacobi_packed(sm, n, cs, pr, red, jl + hdr);
  for (int i = threadIdx.x; i < n; i += NT) d[i] = sm[pidx(i, i)];
  __syncthreads();
  sort_desc(d, n, ord);
  int kept;
  if (mode == 0) {
    kept = k < n ? k : n;
  } else {
    const double lmax = d[ord[0]];
    kept = 0;
    while (kept < n && d[ord[kept]] > 0.0 && d[ord[kept]] > drop2 * lmax) ++kept;
  }
  for (int c = threadIdx.x; c < n; c += NT) {
    jl[2 + c] = double(ord[c]);
    jl[2 + n + c] = (mode == 1 && c < kept) ? 1.0 / sqrt(d[ord[c]]) : 1.0;
  }
  if (threadIdx.x == 0) {
    jl[0] = double(rounds);
    jl[1] = double(kept);
    if (mode == 0) {
      out[2 * b] = n;
      out[2 * b + 1] = kept;
    } else {
      out[b] = kept;
    }
  }
  if (mode == 0)
    for (int c = threadIdx.x; c < k; c += NT) E[int64_t(b) * k + c] = c < kept ? d[ord[c]] : 0.0;
}

// Rows of the eigenvector matrix from the rotation log: row i of V is e_i^T J_1 J_2 ... (V <- V J per round, as
// jacobi()); out[i][c] = V[i][order[c]] scale_c for c < kept, zero for kept <= c < ncol.  Four rows (waves) per
// workgroup, each row in LDS; the log passes through LDS in chunks of JCH rounds shared by the four waves.
constexpr int JCH = 32;
__global__ __launch_bounds__(256) void k_jacobi_rows(int n, const double* jlog, int64_t jls, double* out, int64_t ldo,
                                                     int64_t so, int ncol, const int* skip) {
  __shared__ double rowv[4][PSMAX];
  __shared__ double chunk[JCH * PSMAX];
  const int b = blockIdx.y;
  if (skip && skip[b] == 1) return;
  const double* jl = jlog + b * jls;
  const int m = n + (n & 1), half = m / 2;
  const int hdr = int(jlog_stride(n) - int64_t(JSWEEPS_P) * (m - 1) * m);
  const double* rot = jl + hdr;
  const int rounds = int(jl[0]), kept = int(jl[1]);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  const bool valid = i < n;
  double* rv = rowv[wave];
  for (int j = lane; j < n; j += 64) rv[j] = j == i ? 1.0 : 0.0;
  for (int r0 = 0; r0 < rounds; r0 += JCH) {
    const int nr = rounds - r0 < JCH ? rounds - r0 : JCH;
    __syncthreads();
    for (int e = threadIdx.x; e < nr * m; e += 256) chunk[e] = rot[int64_t(r0) * m + e];
    __syncthreads();
    if (valid) {
      for (int rr = 0; rr < nr; ++rr) {
        const int round = (r0 + rr) % (m - 1);
        for (int t = lane; t < half; t += 64) {
          int p = rr_pos(t, round, m), q = rr_pos(m - 1 - t, round, m);
          if (p > q) {
            const int x = p;
            p = q;
            q = x;
          }
          if (q < n) {
            const double c = chunk[rr * m + 2 * t], s = chunk[rr * m + 2 * t + 1];
            const double vp = rv[p], vq = rv[q];
            rv[p] = c * vp - s * vq;
            rv[q] = s * vp + c * vq;
          }
        }
        // the next round's pairs read what other lanes of this wave wrote
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  if (!valid) return;
  for (int c = lane; c < ncol; c += 64)
    out[b * so + int64_t(i) * ldo + c] = c < kept ? rv[int(jl[2 + c])] * jl[2 + n + c] : 0.0;
}

// Nystrom core, certified path, for 17..160 columns past the LDS limit: C = L L^T (packed tiles), the
// certificate 1 / ||L^{-1}||_F^2 >= eps_rel trace(C), H = L^{-1} R^T (register sweeps; to gw), T = H^T H (to gw
// after H).  stat[b] = 0: T is ready for the packed Jacobi; 1: not certified (the dense kernel then runs).
__global__ __launch_bounds__(NTP) void k_nys_prep_p(int s, const double* C, const double* R, double eps_rel,
                                                    double* gw, int64_t gws, int* stat) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  __shared__ double red[NWP];
  const int b = blockIdx.x;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  C += b * int64_t(s) * s;
  R += b * int64_t(s) * s;
  const int nt = (s + NB - 1) / NB, np = nt * NB;
  double* H = gw + b * gws;
  double* T = H + int64_t(np) * np;
  double* pt = sm;
  double* Dinv = sm + size_t(ptile_count(nt)) * PTS;
  double tr = 0.0;
  for (int i = threadIdx.x; i < s; i += NTP) tr += C[i * s + i];
  tr = group_sum(tr, red);
  ptiles_fill(pt, s, nt, [&](int i, int j) { return 0.5 * (C[i * s + j] + C[j * s + i]); });
  __syncthreads();
  const int info = chol_ptiles(pt, nt, Dinv, &sinfo);
  double fro = 0.0;
  if (info == 0) {
    for (int j = wave; j < nt; j += NWP) {
      sv4d Xr[PNT];
#pragma unroll
      for (int i = 0; i < PNT; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) Xr[i][v] = (i == j && 4 * v + lk == li) ? 1.0 : 0.0;
      wave_fwd(pt, Dinv, nt, j, Xr);
      const int col = NB * j + li;
#pragma unroll
      for (int i = 0; i < PNT; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = NB * i + 4 * v + lk;
          const double x = (i < nt && row < s && col < s) ? Xr[i][v] : 0.0;
          fro += x * x;
        }
    }
  }
  fro = group_sum(fro, red);
  const bool certified = info == 0 && tr > 0.0 && 1.0 / fro >= eps_rel * tr;
  if (threadIdx.x == 0) stat[b] = certified ? 0 : 1;
  if (!certified) return;
  // H = L^{-1} R^T by 16-column chunks (R upper: R^T (i, c) = R[c][i]); rows and columns past s are zero
  for (int c0 = wave * NB; c0 < np; c0 += NWP * NB) {
    const int col = c0 + li;
    const int cb = min(col, s - 1) * s;
    sv4d Xr[PNT];
#pragma unroll
    for (int i = 0; i < PNT / 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) Xr[i][v] = R[cb + min(NB * i + 4 * v + lk, s - 1)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = PNT / 2; i < PNT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) Xr[i][v] = R[cb + min(NB * i + 4 * v + lk, s - 1)];
#pragma unroll
    for (int i = 0; i < PNT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = NB * i + 4 * v + lk;
        if (!(i < nt && row < s && col < s)) Xr[i][v] = 0.0;
      }
    wave_fwd(pt, Dinv, nt, 0, Xr);
#pragma unroll
    for (int i = 0; i < PNT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = NB * i + 4 * v + lk;
        if (i < nt) H[int64_t(row) * np + col] = (row < s && col < s) ? Xr[i][v] : 0.0;
      }
  }
  __syncthreads();
  // T = H^T H, all s x s tiles (the Jacobi kernel symmetrises on load)
  for (int u = wave; u < nt * nt; u += NWP) {
    const int ti = u / nt, tj = u - ti * nt;
    const double* A0 = H + int64_t(lk) * np + NB * ti + li;  // H^T (li, 4 v + lk) = H (4 v + lk, li)
    const double* B0 = H + int64_t(lk) * np + NB * tj + li;
    sv4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < np; kk += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A0[int64_t(kk) * np], B0[int64_t(kk) * np], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = NB * ti + tile_row(v), j = NB * tj + tile_col();
      if (i < s && j < s) T[int64_t(i) * s + j] = acc[v];
    }
  }
}

// Where a launch's workspace lives: LDS when it fits, else the caller's global scratch (checked).
int ws_mode(const SmallWs& ws, size_t elems, int r, int c) {
  if (elems * sizeof(double) <= LDS_LIMIT) return 1;
  if (!ws.p || r > ws.n || c > ws.c)
    fail(INVALID_ARG, "small dense workspace missing or too small for " + std::to_string(r) + " x " +
                          std::to_string(c));
  return 0;
}
size_t dyn_lds(int mode, size_t elems) { return mode ? elems * sizeof(double) : 0; }
// The packed-tile Cholesky kernels serve factors of up to 160 rows whose dense workspace does not fit in LDS.
bool packed_chol(size_t dense_elems, int r) {
  return dense_elems * sizeof(double) > LDS_LIMIT && r >= 1 && r <= PSMAX;
}
size_t packed_lds(int r) { return ptiles_elems((r + NB - 1) / NB) * sizeof(double); }

}  // namespace

size_t small_scratch_elems(int n, int c) {
  const size_t e = std::max(chol_ws(n, std::max(n, c)), evd_elems(n));
  return e * sizeof(double) <= LDS_LIMIT ? 0 : e;
}

size_t small_chol_scratch_elems(int r, int c) {
  const size_t e = chol_ws(r, c);
  return e * sizeof(double) <= LDS_LIMIT ? 0 : e;
}

SmallWs small_ws(DBuf<double>& buf, int nb, int n, int c, bool evd) {
  SmallWs w;
  w.n = n;
  w.c = c;
  w.stride = int64_t(small_scratch_elems(n, c));
  const bool logs = evd && w.stride > 0 && evd_elems(n) * sizeof(double) > LDS_LIMIT && n <= PSMAX;
  w.jstride = logs ? jlog_stride(n) : 0;
  const size_t nbs = size_t(std::max(nb, 1));
  const size_t total = size_t(w.stride) * nbs + size_t(w.jstride) * nbs + (logs ? (nbs + 1) / 2 + 1 : 0);
  if (total > 0) {
    buf.alloc(total);
    w.p = w.stride > 0 ? buf.p : nullptr;
    if (logs) {
      w.jlog = buf.p + size_t(w.stride) * nbs;
      w.jstat = reinterpret_cast<int*>(w.jlog + size_t(w.jstride) * nbs);
    }
  }
  return w;
}

void small_chol_solve(Batch bt, int r, double* D, int64_t sD, const double* B, int64_t ldb, int64_t sB, double* X,
                      int64_t ldx, int64_t sX, int s, int s0, double alpha, int* flag, const SmallWs& ws,
                      hipStream_t st) {
  KScope ks_small(KF_SMALL, st);
  if (bt.nb <= 0 || (r <= 0 && s0 <= 0)) return;  // s == 0: factor only
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t el = chol_ws(r, s);
  if (packed_chol(el, r)) {  // the factorisation on one workgroup, then the chunks of the solve side by side
    k_small_chol_solve_p<<<bt.nb, NTP, packed_lds(r), st>>>(r, bt.dims, D, sD, B, ldb, sB, X, ldx, sX, 0, s0, alpha,
                                                           flag, 1);
    NS_LAUNCH_CHECK();
    if (s > 0) {
      k_small_chol_apply_p<<<dim3(unsigned((s + NB - 1) / NB), unsigned(bt.nb)), NTP, packed_lds(r), st>>>(
          r, bt.dims, D, sD, B, ldb, sB, X, ldx, sX, s, s0, alpha);
      NS_LAUNCH_CHECK();
    }
    return;
  }
  const int mode = ws_mode(ws, el, r, s);
  if (mode)
    k_small_chol_solve<1><<<bt.nb, NT, dyn_lds(mode, el), st>>>(r, bt.dims, D, sD, B, ldb, sB, X, ldx, sX, s, s0,
                                                                alpha, flag, 1, ws.p, ws.stride);
  else
    k_small_chol_solve<0><<<bt.nb, NT, 0, st>>>(r, bt.dims, D, sD, B, ldb, sB, X, ldx, sX, s, s0, alpha, flag, 1, ws.p,
                                               ws.stride);
  NS_LAUNCH_CHECK();
}

void small_chol_apply(Batch bt, int r, const double* L, int64_t sL, const double* B, int64_t ldb, int64_t sB,
                      double* X, int64_t ldx, int64_t sX, int s, int s0, double alpha, const SmallWs& ws,
                      hipStream_t st) {
  KScope ks_small(KF_SMALL, st);
  if (bt.nb <= 0 || (r <= 0 && s0 <= 0) || s <= 0) return;
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t el = chol_ws(r, s);
  if (packed_chol(el, r)) {
    k_small_chol_apply_p<<<dim3(unsigned((s + NB - 1) / NB), unsigned(bt.nb)), NTP, packed_lds(r), st>>>(
        r, bt.dims, L, sL, B, ldb, sB, X, ldx, sX, s, s0, alpha);
    NS_LAUNCH_CHECK();
    return;
  }
  const int mode = ws_mode(ws, el, r, s);
  if (mode)
    k_small_chol_solve<1><<<bt.nb, NT, dyn_lds(mode, el), st>>>(r, bt.dims, const_cast<double*>(L), sL, B, ldb, sB,
                                                                X, ldx, sX, s, s0, alpha, nullptr, 0, ws.p, ws.stride);
  else
    k_small_chol_solve<0><<<bt.nb, NT, 0, st>>>(r, bt.dims, const_cast<double*>(L), sL, B, ldb, sB, X, ldx, sX, s, s0,
                                               alpha, nullptr, 0, ws.p, ws.stride);
  NS_LAUNCH_CHECK();
}

void small_svqb(int nb, int s, const double* G, int64_t sG, double drop2, double* T, int64_t sT, int* out,
                const int* skip, const SmallWs& ws, hipStream_t st) {
  KScope ks_small(KF_SMALL, st);
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  const size_t el = evd_elems(s);
  const int mode = ws_mode(ws, el, s, s);
  if (mode) {
    k_small_svqb<1><<<nb, NT, dyn_lds(mode, el), st>>>(s, G, sG, drop2, T, sT, out, skip, ws.p, ws.stride);
  } else if (s <= PSMAX && ws.jlog) {
    k_jacobi_p<<<nb, NT, size_t(s) * (s + 1) / 2 * sizeof(double), st>>>(s, G, sG, 1, 0, drop2, nullptr, out, skip,
                                                                        ws.jlog, ws.jstride);
    NS_LAUNCH_CHECK();
    k_jacobi_rows<<<dim3(unsigned((s + 3) / 4), unsigned(nb)), 256, 0, st>>>(s, ws.jlog, ws.jstride, T, s, sT, s,
                                                                            skip);
  } else {
    k_small_svqb<0><<<nb, NT, 0, st>>>(s, G, sG, drop2, T, sT, out, skip, ws.p, ws.stride);
  }
  NS_LAUNCH_CHECK();
}

void small_cholqr(Batch bt, int s, const double* G, int64_t sG, const double* shift, double* Rinv, double* Racc,
                  int init, int* flag, const SmallWs& ws, hipStream_t st, double certify, int* ok, double single_thr,
                  int* single) {
  KScope ks_small(KF_SMALL, st);
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  const size_t el = chol_ws(s, s);
  const int mode = ws_mode(ws, el, s, s);
  if (packed_chol(el, s)) {  // (its R Racc staging uses the global scratch that ws_mode checked)
    k_small_cholqr_p<<<bt.nb, NTP, packed_lds(s), st>>>(s, bt.dims, G, sG, shift, Rinv, Racc, init, flag, ws.p,
                                                        ws.stride, certify, ok, single_thr, single);
    NS_LAUNCH_CHECK();
    return;
  }
  if (mode)
    k_small_cholqr<1><<<bt.nb, NT, dyn_lds(mode, el), st>>>(s, bt.dims, G, sG, shift, Rinv, Racc, init, flag, ws.p,
                                                            ws.stride, certify, ok, single_thr, single);
  else
    k_small_cholqr<0><<<bt.nb, NT, 0, st>>>(s, bt.dims, G, sG, shift, Rinv, Racc, init, flag, ws.p, ws.stride, certify,
                                           ok, single_thr, single);
  NS_LAUNCH_CHECK();
}

void small_nystrom(int nb, int s, int k, const double* C, const double* R, double eps_rel, double* Wk, double* Ek,
                   int* out, const SmallWs& ws, hipStream_t st) {
  KScope ks_small(KF_SMALL, st);
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  const size_t el = chol_ws(s, s);
  const int mode = ws_mode(ws, el, s, s);
  if (mode) {
    k_small_nystrom<1><<<nb, NT, dyn_lds(mode, el), st>>>(s, k, C, R, eps_rel, Wk, Ek, out, ws.p, ws.stride, nullptr);
  } else if (s <= PSMAX && ws.jlog) {
    // packed kernels for the certified problems (jstat 0), the dense kernel in global memory for the others
    const int np = pad16(s);
    k_nys_prep_p<<<nb, NTP, packed_lds(s), st>>>(s, C, R, eps_rel, ws.p, ws.stride, ws.jstat);
    NS_LAUNCH_CHECK();
    k_jacobi_p<<<nb, NT, size_t(s) * (s + 1) / 2 * sizeof(double), st>>>(
        s, ws.p + int64_t(np) * np, ws.stride, 0, k, 0.0, Ek, out, ws.jstat, ws.jlog, ws.jstride);
    NS_LAUNCH_CHECK();
    k_jacobi_rows<<<dim3(unsigned((s + 3) / 4), unsigned(nb)), 256, 0, st>>>(s, ws.jlog, ws.jstride, Wk, k,
                                                                            int64_t(s) * k, k, ws.jstat);
    NS_LAUNCH_CHECK();
    k_small_nystrom<0><<<nb, NT, 0, st>>>(s, k, C, R, eps_rel, Wk, Ek, out, ws.p, ws.stride, ws.jstat);
  } else {
    k_small_nystrom<0><<<nb, NT, 0, st>>>(s, k, C, R, eps_rel, Wk, Ek, out, ws.p, ws.stride, nullptr);
  }
  NS_LAUNCH_CHECK();
}


void small_gevd(int k, const double* A, const double* B, double* lam, double* C, double* Cl, int* flag, double* ws,
                const SmallWs& sw, hipStream_t st) {
  KScope ks_small(KF_SMALL, st);
  if (k > SMAX) fail(INVALID_ARG, "matrix too large for the small dense kernels (limit 256)");
  double* L = ws;
  double* Linv = ws + size_t(k) * k;
  double* M = Linv + size_t(k) * k;
  double* W = M + size_t(k) * k;
  double* E = W + size_t(k) * k;
  k_gevd_reduce<<<1, NT, 0, st>>>(k, A, B, L, Linv, M, flag);
  NS_LAUNCH_CHECK();
  small_sym_evd(k, M, W, E, sw, st);
  k_gevd_back<<<1, 256, 0, st>>>(k, Linv, W, E, lam, C, Cl);
  NS_LAUNCH_CHECK();
}

void small_sym_evd(int m, const double* A, double* W, double* E, const SmallWs& ws, hipStream_t st) {
  KScope ks_small(KF_SMALL, st);
  if (m > SMAX) fail(INVALID_ARG, "matrix too large for the small dense kernels (limit 256)");
  const size_t el = evd_elems(m);
  const int mode = ws_mode(ws, el, m, m);
  if (mode)
    k_small_sym_evd<1><<<1, NT, dyn_lds(mode, el), st>>>(m, A, W, E, ws.p);
  else
    k_small_sym_evd<0><<<1, NT, 0, st>>>(m, A, W, E, ws.p);
  NS_LAUNCH_CHECK();
}

}  // namespace ns
