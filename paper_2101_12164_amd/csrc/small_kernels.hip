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

// Workspace (doubles) of the blocked Cholesky kernels: factor L (r x (r+1)), right-hand sides / inverse
// X (r x (c+1)), diagonal-block inverses, panel buffer (r x NBL) and block-row buffer (NB x (c+1)).
__host__ __device__ inline size_t chol_ws(int r, int c) {
  const size_t nbk = size_t((r + NB - 1) / NB);
  return size_t(r) * (r + 1) + size_t(r) * (c + 1) + nbk * NB * NBL + size_t(r) * NBL + size_t(NB) * (c + 1);
}
__host__ __device__ inline size_t evd_elems(int n) { return size_t(2) * n * (n + 1); }

__device__ double block_sum(double v, double* red) {
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
// pr: n+2 ints.  Each round applies the n/2 disjoint rotations of a
// round-robin ordering at once: every 2x2 block (pair P rows, pair Q columns)
// of A becomes J_P^T B J_Q, and V's column pairs become V J_Q.
__device__ void jacobi(double* A, double* V, int n, int ld, double* cs, int* pr, double* red) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    V[i * ld + j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  if (n < 2) return;
  const int m = n + (n & 1);
  const int half = m / 2;
  const float inv_half = 1.0f / float(half);
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
          if (fabs(apq) > 1e-18 * sqrt(fabs(A[p * ld + p] * A[q * ld + q])) && fabs(apq) > 1e-300) {
            const double tau = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pr[2 * tid] = p;
        pr[2 * tid + 1] = q;  // q == n marks the dummy partner of an odd n
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
      }
      __syncthreads();
      // A <- J^T A J on all 2x2 pair blocks
      for (int t = tid; t < half * half; t += NT) {
        const int P = int((float(t) + 0.5f) * inv_half), Q = t - P * half;
        const int p0 = pr[2 * P], q0 = pr[2 * P + 1], p1 = pr[2 * Q], q1 = pr[2 * Q + 1];
        const double cP = cs[2 * P], sP = cs[2 * P + 1], cQ = cs[2 * Q], sQ = cs[2 * Q + 1];
        const bool hq0 = q0 < n, hq1 = q1 < n;
        const double b00 = A[p0 * ld + p1];
        const double b01 = hq1 ? A[p0 * ld + q1] : 0.0;
        const double b10 = hq0 ? A[q0 * ld + p1] : 0.0;
        const double b11 = (hq0 && hq1) ? A[q0 * ld + q1] : 0.0;
        const double x00 = cP * b00 - sP * b10, x01 = cP * b01 - sP * b11;  // J_P^T B
        const double x10 = sP * b00 + cP * b10, x11 = sP * b01 + cP * b11;
        A[p0 * ld + p1] = x00 * cQ - x01 * sQ;
        if (hq1) A[p0 * ld + q1] = x00 * sQ + x01 * cQ;
        if (hq0) A[q0 * ld + p1] = x10 * cQ - x11 * sQ;
        if (hq0 && hq1) A[q0 * ld + q1] = x10 * sQ + x11 * cQ;
      }
      // V <- V J
      for (int t = tid; t < n * half; t += NT) {
        const int i = int((float(t) + 0.5f) * inv_half), Q = t - i * half;
        const int p1 = pr[2 * Q], q1 = pr[2 * Q + 1];
        if (q1 >= n) continue;
        const double cQ = cs[2 * Q], sQ = cs[2 * Q + 1];
        const double vp = V[i * ld + p1], vq = V[i * ld + q1];
        V[i * ld + p1] = cQ * vp - sQ * vq;
        V[i * ld + q1] = sQ * vp + cQ * vq;
      }
      __syncthreads();
    }
  }
}

// order[i] = index of the i-th largest of d[0..n) (ties by index).
__device__ void sort_desc(const double* d, int n, int* order) {
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
__device__ int chol_dev(double* A, int n, int lda, int* sinfo) {
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
__device__ void chol_solve_inplace(const double* L, int r, int ldl, double* X, int ldx, int s) {
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
__device__ int diag_factor_wave(double* A, int ld, int j0, int jb, double* Di) {
  const int lane = threadIdx.x & 63;
  double r[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) r[t] = (lane < jb && t <= lane) ? A[(j0 + lane) * ld + j0 + t] : 0.0;
  int bad = 0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < jb) {
      double d = lane_of(r[c], c);
      if (!(d > 0.0)) {
        if (!bad) bad = c + 1;
        d = 1.0;
      }
      const double sq = sqrt(d), inv = 1.0 / sq;
      r[c] = lane == c ? sq : (lane > c ? r[c] * inv : 0.0);
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
    x[i] = (i < jb) ? acc / lane_of(r[i], i) : 0.0;
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

// In-place lower Cholesky of A (n x n, stride ld).  Dinv: ceil(n/NB) diagonal-block inverses (NB x NBL
// each), Pn: n x NBL panel scratch.  Returns 0 or the 1-based index of the first pivot <= 0.
__device__ int chol_blocked(double* A, int n, int ld, double* Dinv, double* Pn, int* sinfo) {
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) *sinfo = 0;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = n - j0 < NB ? n - j0 : NB;
    const double* Di = Dinv + (j0 / NB) * (NB * NBL);
    if (wave == 0) {
      const int bad = diag_factor_wave(A, ld, j0, jb, Dinv + (j0 / NB) * (NB * NBL));
      if (bad && (threadIdx.x & 63) == 0 && *sinfo == 0) *sinfo = j0 + bad;
    }
    __syncthreads();
    const int j1 = j0 + jb, m = n - j1;
    for (int e = threadIdx.x; e < m * jb; e += NT) {  // Pn = A21 L11^{-T}
      const int i = e / jb, c = e - i * jb;
      const double* a = A + (j1 + i) * ld + j0;
      double acc = 0.0;
      for (int t = 0; t <= c; ++t) acc += a[t] * Di[c * NBL + t];
      Pn[i * NBL + c] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * m; e += NT) {  // A22 -= L21 L21^T (lower)
      const int i = e / m, q = e - i * m;
      if (q > i) continue;
      double acc = A[(j1 + i) * ld + j1 + q];
      for (int t = 0; t < jb; ++t) acc -= Pn[i * NBL + t] * Pn[q * NBL + t];
      A[(j1 + i) * ld + j1 + q] = acc;
    }
    for (int e = threadIdx.x; e < m * jb; e += NT) {
      const int i = e / jb, c = e - i * jb;
      A[(j1 + i) * ld + j0 + c] = Pn[i * NBL + c];
    }
    __syncthreads();
  }
  const int info = *sinfo;
  __syncthreads();
  return info;
}

// Diagonal-block inverses of an existing factor L (n x n, stride ld): one wave per block.
__device__ void diag_inverses(const double* L, int n, int ld, double* Dinv) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nbk = (n + NB - 1) / NB;
  for (int bk = wave; bk < nbk; bk += NT / 64) {
    const int j0 = bk * NB, jb = n - j0 < NB ? n - j0 : NB;
    double x[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int ii = i < jb ? i : jb - 1;  // clamped: rows past the block are never read
      double acc = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < i; ++t) acc -= L[(j0 + ii) * ld + j0 + (t < ii ? t : ii)] * x[t];
      x[i] = (i < jb) ? acc / L[(j0 + ii) * ld + j0 + ii] : 0.0;
    }
    if (lane < NB) {
#pragma unroll
      for (int i = 0; i < NB; ++i) Dinv[bk * (NB * NBL) + i * NBL + lane] = (lane < jb && i < jb) ? x[i] : 0.0;
    }
  }
  __syncthreads();
}

// X (r x c, stride lx) <- (L L^T)^{-1} X by block rows: forward L Y = X, then backward L^T X = Y.
// Tb: NB x (c + 1) scratch.
__device__ void chol_solve_blocked(const double* L, int r, int ld, const double* Dinv, double* X, int lx, int c,
                                   double* Tb) {
  const int nbk = (r + NB - 1) / NB, lt = c + 1;
  for (int bk = 0; bk < nbk; ++bk) {
    const int i0 = bk * NB, ib = r - i0 < NB ? r - i0 : NB;
    const double* Di = Dinv + bk * (NB * NBL);
    for (int e = threadIdx.x; e < ib * c; e += NT) {  // Tb = X_i - L_{i,<i} Y_{<i}
      const int a = e / c, j = e - a * c;
      const double* l = L + (i0 + a) * ld;
      double acc = X[(i0 + a) * lx + j];
      for (int t = 0; t < i0; ++t) acc -= l[t] * X[t * lx + j];
      Tb[a * lt + j] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ib * c; e += NT) {  // Y_i = L_ii^{-1} Tb
      const int a = e / c, j = e - a * c;
      double acc = 0.0;
      for (int t = 0; t <= a; ++t) acc += Di[a * NBL + t] * Tb[t * lt + j];
      X[(i0 + a) * lx + j] = acc;
    }
    __syncthreads();
  }
  for (int bk = nbk - 1; bk >= 0; --bk) {
    const int i0 = bk * NB, ib = r - i0 < NB ? r - i0 : NB;
    const double* Di = Dinv + bk * (NB * NBL);
    for (int e = threadIdx.x; e < ib * c; e += NT) {  // Tb = Y_i - L_{>i,i}^T X_{>i}
      const int a = e / c, j = e - a * c;
      double acc = X[(i0 + a) * lx + j];
      for (int t = i0 + ib; t < r; ++t) acc -= L[t * ld + i0 + a] * X[t * lx + j];
      Tb[a * lt + j] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ib * c; e += NT) {  // X_i = L_ii^{-T} Tb
      const int a = e / c, j = e - a * c;
      double acc = 0.0;
      for (int t = a; t < ib; ++t) acc += Di[t * NBL + a] * Tb[t * lt + j];
      X[(i0 + a) * lx + j] = acc;
    }
    __syncthreads();
  }
}

// X = L^{-1} (n x n, stride ld, zero above the diagonal) from the factor and its diagonal-block inverses,
// by block rows: X_ij = -L_ii^{-1} sum_{j <= t < i} L_it X_tj.  Tb: NB x (n + 1) scratch.
__device__ void tri_inverse_blocked(const double* L, int n, int ld, const double* Dinv, double* X, double* Tb) {
  const int lt = n + 1;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e - i * n;
    const int bi = i / NB, bj = j / NB;
    X[i * ld + j] = (bi == bj && j <= i) ? Dinv[bi * (NB * NBL) + (i - bi * NB) * NBL + (j - bj * NB)] : 0.0;
  }
  __syncthreads();
  const int nbk = (n + NB - 1) / NB;
  for (int bk = 1; bk < nbk; ++bk) {
    const int i0 = bk * NB, ib = n - i0 < NB ? n - i0 : NB;
    const double* Di = Dinv + bk * (NB * NBL);
    for (int e = threadIdx.x; e < ib * i0; e += NT) {  // Tb[a][j] = sum_{j <= t < i0} L[i0+a][t] X[t][j]
      const int a = e / i0, j = e - a * i0;
      const double* l = L + (i0 + a) * ld;
      double acc = 0.0;
      for (int t = j; t < i0; ++t) acc += l[t] * X[t * ld + j];
      Tb[a * lt + j] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ib * i0; e += NT) {
      const int a = e / i0, j = e - a * i0;
      double acc = 0.0;
      for (int t = 0; t <= a; ++t) acc += Di[a * NBL + t] * Tb[t * lt + j];
      X[(i0 + a) * ld + j] = -acc;
    }
    __syncthreads();
  }
}

// Carve of a chol_ws(r, c) workspace.
struct CholWs {
  double *L, *X, *Dinv, *Pn, *Tb;
  int ldl, ldx;
};
__device__ CholWs chol_carve(double* base, int r, int c) {
  CholWs w;
  w.ldl = r + 1;
  w.ldx = c + 1;
  w.L = base;
  w.X = w.L + size_t(r) * w.ldl;
  w.Dinv = w.X + size_t(r) * w.ldx;
  w.Pn = w.Dinv + size_t((r + NB - 1) / NB) * NB * NBL;
  w.Tb = w.Pn + size_t(r) * NBL;
  return w;
}

// Problem b: D (r0 x r0, ld r0) at D + b sD, leading rb = dims[b] block used; B, X likewise.  factor: D is
// factored (L written back); otherwise D holds the factor from an earlier call.
__global__ __launch_bounds__(NT) void k_small_chol_solve(int r0, const int* __restrict__ dims, double* D, int64_t sD,
                                                         const double* B, int64_t ldb, int64_t sB, double* X,
                                                         int64_t ldx, int64_t sX, int s, int s0, double alpha,
                                                         int* flag, int factor, double* gw, int64_t gws, int lds) {
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
  CholWs w = chol_carve(lds ? sm : gw + b * gws, r, s);
  for (int e = threadIdx.x; e < r * r; e += NT) w.L[(e / r) * w.ldl + e % r] = D[(e / r) * r0 + e % r];
  for (int e = threadIdx.x; e < r * s; e += NT) w.X[(e / s) * w.ldx + e % s] = B[(e / s) * ldb + e % s];
  __syncthreads();
  if (factor) {
    const int info = chol_blocked(w.L, r, w.ldl, w.Dinv, w.Pn, &sinfo);
    if (info && threadIdx.x == 0) flag[0] = 1;
    for (int e = threadIdx.x; e < r * r; e += NT) D[(e / r) * r0 + e % r] = w.L[(e / r) * w.ldl + e % r];
  } else {
    diag_inverses(w.L, r, w.ldl, w.Dinv);
  }
  if (s == 0) return;
  chol_solve_blocked(w.L, r, w.ldl, w.Dinv, w.X, w.ldx, s, w.Tb);
  for (int e = threadIdx.x; e < r * s; e += NT) X[(e / s) * ldx + e % s] = alpha * w.X[(e / s) * w.ldx + e % s];
}

// Workspace for the Jacobi kernels: two n x (n+1) matrices + small arrays, in
// LDS when they fit, else in the caller's global scratch `gw`.
struct EvdSpace {
  double *A, *V, *cs, *d;
  int *pr, *ord;
  int ld;
};

__device__ EvdSpace evd_space(int n, double* base, double* small_d, int* small_i) {
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

__global__ __launch_bounds__(NT) void k_small_svqb(int s, const double* G, int64_t sG, double drop2, double* T,
                                                   int64_t sT, int* out, const int* skip, double* gw, int64_t gws,
                                                   int lds) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  const int b = blockIdx.x;
  if (skip && skip[b]) return;
  G += b * sG;
  T += b * sT;
  EvdSpace w = evd_space(s, lds ? sm : gw + b * gws, sd, si);
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
__global__ __launch_bounds__(NT) void k_small_cholqr(int s, const int* __restrict__ dims, const double* G, int64_t sG,
                                                     const double* shift_coef, double* Rinv, double* Racc, int init,
                                                     int* flag, double* gw, int64_t gws, int lds, double certify,
                                                     int* ok) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  __shared__ double sshift, strace;
  __shared__ double red[NT];
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : s;
  G += b * sG;
  Rinv += b * int64_t(s) * s;
  Racc += b * int64_t(s) * s;
  if (n == 0) {
    for (int e = threadIdx.x; e < s * s; e += NT) Rinv[e] = Racc[e] = 0.0;
    if (ok && threadIdx.x == 0) ok[b] = 0;
    return;
  }
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += G[i * s + i];
    sshift = (shift_coef ? shift_coef[b] : 0.0) * tr;
    strace = tr;
  }
  __syncthreads();
  const double shift = sshift;
  CholWs w = chol_carve(lds ? sm : gw + b * gws, n, n);
  const int ld = w.ldl;
  double* A = w.L;
  double* X = w.X;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    A[i * ld + j] = 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift : 0.0);
  }
  __syncthreads();
  if (chol_blocked(A, n, ld, w.Dinv, w.Pn, &sinfo) && threadIdx.x == 0) flag[0] = 1;
  tri_inverse_blocked(A, n, ld, w.Dinv, X, w.Tb);  // X = L^{-1}
  // Rinv = (L^{-1})^T (upper) in the leading block, zero elsewhere; R = L^T
  double fro = 0.0;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    const double x = (i < n && j < n) ? X[j * ld + i] : 0.0;
    Rinv[e] = x;
    fro += x * x;
  }
  if (ok) {
    // lambda_min(G) >= 1 / ||L^{-1}||_F^2 and lambda_max(G) <= trace(G): certify that no
    // singular value ratio of the block is at or below the drop tolerance
    const double f = block_sum(fro, red);
    if (threadIdx.x == 0) ok[b] = (sinfo == 0 && 1.0 / f > certify * strace) ? 1 : 0;
  }
  __syncthreads();
  if (init) {
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const int i = e / s, j = e % s;
      Racc[e] = (i < n && j < n && j >= i) ? A[j * ld + i] : 0.0;
    }
    return;
  }
  // Racc <- R * Racc, with Racc staged in X
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    X[i * ld + j] = Racc[i * s + j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    double acc = 0.0;
    if (i < n && j < n)
      for (int m = i; m <= j; ++m) acc += A[m * ld + i] * X[m * ld + j];
    Racc[e] = acc;
  }
}

// Nystrom core of one problem.  C = Omega^T Y (s x s) and the Cholesky-QR factor R of Y give
// T = R C_1^+ R^T over the eigenpairs of sym(C) with lambda >= eps_rel lambda_max, whose EVD yields the
// basis.  When a Cholesky C = L L^T succeeds with 1/||L^{-1}||_F^2 >= eps_rel trace(C) (a lower bound of
// lambda_min against an upper bound of lambda_max), every eigenpair passes the threshold and
// T = R C^{-1} R^T = F F^T with F = R L^{-T}: the EVD of C is skipped.
__global__ __launch_bounds__(NT) void k_small_nystrom(int s, int k, const double* C, const double* R, double eps_rel,
                                                      double* Wk, double* Ek, int* out, double* gw, int64_t gws,
                                                      int lds) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  __shared__ double dkeep[SMAX];
  __shared__ int ikeep[SMAX];
  __shared__ int nkeep, sinfo;
  const int b = blockIdx.x;
  C += b * int64_t(s) * s;
  R += b * int64_t(s) * s;
  Wk += b * int64_t(s) * k;
  Ek += b * int64_t(k);
  out += 2 * b;
  CholWs cw = chol_carve(lds ? sm : gw + b * gws, s, s);  // regions L and X double as the EVD's A and V
  EvdSpace w = evd_space(s, cw.L, sd, si);
  const int ld = w.ld;
  for (int e = threadIdx.x; e < s * s; e += NT) {  // symmetrised C
    const int i = e / s, j = e % s;
    w.A[i * ld + j] = 0.5 * (C[i * s + j] + C[j * s + i]);
  }
  double tr = 0.0;
  for (int i = threadIdx.x; i < s; i += NT) tr += C[i * s + i];
  tr = block_sum(tr, red);
  const int info = chol_blocked(w.A, s, ld, cw.Dinv, cw.Pn, &sinfo);
  bool certified = false;
  if (info == 0) {
    tri_inverse_blocked(w.A, s, ld, cw.Dinv, w.V, cw.Tb);  // V = L^{-1}
    double fro = 0.0;
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const double x = w.V[(e / s) * ld + e % s];
      fro += x * x;
    }
    fro = block_sum(fro, red);
    certified = tr > 0.0 && 1.0 / fro >= eps_rel * tr;
  }
  int r;
  if (certified) {
    r = s;
    // F = R L^{-T} into A: F[i][j] = sum_{i <= m <= j} R[i][m] Linv[j][m]
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const int i = e / s, j = e % s;
      double acc = 0.0;
      for (int m = i; m <= j; ++m) acc += R[i * s + m] * w.V[j * ld + m];
      w.A[i * ld + j] = acc;
    }
    __syncthreads();
    // T = F F^T into V
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const int i = e / s, j = e % s;
      if (j > i) continue;
      double acc = 0.0;
      for (int m = 0; m < s; ++m) acc += w.A[i * ld + m] * w.A[j * ld + m];
      w.V[i * ld + j] = acc;
      w.V[j * ld + i] = acc;
    }
    __syncthreads();
  } else {
    for (int e = threadIdx.x; e < s * s; e += NT) {  // symmetrised C again (the factorisation overwrote it)
      const int i = e / s, j = e % s;
      w.A[i * ld + j] = 0.5 * (C[i * s + j] + C[j * s + i]);
    }
    __syncthreads();
    jacobi(w.A, w.V, s, ld, w.cs, w.pr, red);
    for (int i = threadIdx.x; i < s; i += NT) w.d[i] = w.A[i * ld + i];
    __syncthreads();
    if (threadIdx.x == 0) {
      double dmax = w.d[0];
      for (int i = 1; i < s; ++i) dmax = w.d[i] > dmax ? w.d[i] : dmax;
      int q = 0;
      if (dmax > 0.0)
        for (int i = 0; i < s; ++i)
          if (w.d[i] >= eps_rel * dmax) {
            ikeep[q] = i;
            dkeep[q] = w.d[i];
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
      for (int m = i; m < s; ++m) acc += R[i * s + m] * w.V[m * ld + ikeep[c]];
      w.A[i * ld + c] = acc;
    }
    __syncthreads();
    // T = M D_1^{-1} M^T into V, symmetric by construction of the sum
    for (int e = threadIdx.x; e < s * s; e += NT) {
      const int i = e / s, j = e % s;
      if (j > i) continue;
      double acc = 0.0;
      for (int c = 0; c < r; ++c) acc += w.A[i * ld + c] * w.A[j * ld + c] / dkeep[c];
      w.V[i * ld + j] = acc;
      w.V[j * ld + i] = acc;
    }
    __syncthreads();
  }
  jacobi(w.V, w.A, s, ld, w.cs, w.pr, red);  // EVD of T: eigenvectors in A
  for (int i = threadIdx.x; i < s; i += NT) w.d[i] = w.V[i * ld + i];
  __syncthreads();
  sort_desc(w.d, s, w.ord);
  const int kk = k < r ? k : r;
  for (int e = threadIdx.x; e < s * k; e += NT) {
    const int i = e / k, c = e % k;
    Wk[e] = c < kk ? w.A[i * ld + w.ord[c]] : 0.0;
  }
  for (int c = threadIdx.x; c < k; c += NT) Ek[c] = c < kk ? w.d[w.ord[c]] : 0.0;
  if (threadIdx.x == 0) {
    out[0] = r;
    out[1] = kk;
  }
}

__global__ void k_small_rowscale(int k, int ncols, const double* sigma, int64_t ssig, double* c, int64_t ldc,
                                 int64_t sc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= k * ncols) return;
  const int i = idx / ncols, j = idx % ncols;
  c[b * sc + i * ldc + j] *= sigma[b * ssig + i];
}

__global__ __launch_bounds__(NT) void k_small_sym_evd(int m, const double* Ain, double* W, double* E, double* gw,
                                                      int lds) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  EvdSpace w = evd_space(m, lds ? sm : gw, sd, si);
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

// Where a launch's workspace lives: LDS when it fits, else the caller's global scratch (checked).
int ws_mode(const SmallWs& ws, size_t elems, int r, int c) {
  if (elems * sizeof(double) <= LDS_LIMIT) return 1;
  if (!ws.p || r > ws.n || c > ws.c)
    fail(INVALID_ARG, "small dense workspace missing or too small for " + std::to_string(r) + " x " +
                          std::to_string(c));
  return 0;
}
size_t dyn_lds(int mode, size_t elems) { return mode ? elems * sizeof(double) : 0; }

}  // namespace

size_t small_scratch_elems(int n, int c) {
  const size_t e = std::max(chol_ws(n, std::max(n, c)), evd_elems(n));
  return e * sizeof(double) <= LDS_LIMIT ? 0 : e;
}

SmallWs small_ws(DBuf<double>& buf, int nb, int n, int c) {
  SmallWs w;
  w.n = n;
  w.c = c;
  w.stride = int64_t(small_scratch_elems(n, c));
  if (w.stride > 0) {
    buf.alloc(size_t(w.stride) * std::max(nb, 1));
    w.p = buf.p;
  }
  return w;
}

void small_chol_solve(Batch bt, int r, double* D, int64_t sD, const double* B, int64_t ldb, int64_t sB, double* X,
                      int64_t ldx, int64_t sX, int s, int s0, double alpha, int* flag, const SmallWs& ws,
                      hipStream_t st) {
  if (bt.nb <= 0 || (r <= 0 && s0 <= 0)) return;  // s == 0: factor only
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t el = chol_ws(r, s);
  const int mode = ws_mode(ws, el, r, s);
  k_small_chol_solve<<<bt.nb, NT, dyn_lds(mode, el), st>>>(r, bt.dims, D, sD, B, ldb, sB, X, ldx, sX, s, s0, alpha,
                                                           flag, 1, ws.p, ws.stride, mode);
  NS_LAUNCH_CHECK();
}

void small_chol_apply(Batch bt, int r, const double* L, int64_t sL, const double* B, int64_t ldb, int64_t sB,
                      double* X, int64_t ldx, int64_t sX, int s, int s0, double alpha, const SmallWs& ws,
                      hipStream_t st) {
  if (bt.nb <= 0 || (r <= 0 && s0 <= 0) || s <= 0) return;
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t el = chol_ws(r, s);
  const int mode = ws_mode(ws, el, r, s);
  k_small_chol_solve<<<bt.nb, NT, dyn_lds(mode, el), st>>>(r, bt.dims, const_cast<double*>(L), sL, B, ldb, sB, X,
                                                           ldx, sX, s, s0, alpha, nullptr, 0, ws.p, ws.stride, mode);
  NS_LAUNCH_CHECK();
}

void small_svqb(int nb, int s, const double* G, int64_t sG, double drop2, double* T, int64_t sT, int* out,
                const int* skip, const SmallWs& ws, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  const size_t el = evd_elems(s);
  const int mode = ws_mode(ws, el, s, s);
  k_small_svqb<<<nb, NT, dyn_lds(mode, el), st>>>(s, G, sG, drop2, T, sT, out, skip, ws.p, ws.stride, mode);
  NS_LAUNCH_CHECK();
}

void small_cholqr(Batch bt, int s, const double* G, int64_t sG, const double* shift, double* Rinv, double* Racc,
                  int init, int* flag, const SmallWs& ws, hipStream_t st, double certify, int* ok) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  const size_t el = chol_ws(s, s);
  const int mode = ws_mode(ws, el, s, s);
  k_small_cholqr<<<bt.nb, NT, dyn_lds(mode, el), st>>>(s, bt.dims, G, sG, shift, Rinv, Racc, init, flag, ws.p,
                                                       ws.stride, mode, certify, ok);
  NS_LAUNCH_CHECK();
}

void small_nystrom(int nb, int s, int k, const double* C, const double* R, double eps_rel, double* Wk, double* Ek,
                   int* out, const SmallWs& ws, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  const size_t el = chol_ws(s, s);
  const int mode = ws_mode(ws, el, s, s);
  k_small_nystrom<<<nb, NT, dyn_lds(mode, el), st>>>(s, k, C, R, eps_rel, Wk, Ek, out, ws.p, ws.stride, mode);
  NS_LAUNCH_CHECK();
}

void small_rowscale(int nb, int k, int ncols, const double* sigma, int64_t ssig, double* c, int64_t ldc, int64_t sc,
                    hipStream_t st) {
  if (k * ncols == 0 || nb == 0) return;
  k_small_rowscale<<<dim3((k * ncols + 255) / 256, nb), 256, 0, st>>>(k, ncols, sigma, ssig, c, ldc, sc);
  NS_LAUNCH_CHECK();
}

void small_gevd(int k, const double* A, const double* B, double* lam, double* C, double* Cl, int* flag, double* ws,
                const SmallWs& sw, hipStream_t st) {
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
  if (m > SMAX) fail(INVALID_ARG, "matrix too large for the small dense kernels (limit 256)");
  const size_t el = evd_elems(m);
  const int mode = ws_mode(ws, el, m, m);
  k_small_sym_evd<<<1, NT, dyn_lds(mode, el), st>>>(m, A, W, E, ws.p, mode);
  NS_LAUNCH_CHECK();
}

}  // namespace ns
