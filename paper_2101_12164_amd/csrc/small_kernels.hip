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
// global scratch per problem: two SMAX x (SMAX + 1) matrices or the Cholesky-solve layout
constexpr size_t scratch_evd = size_t(2) * SMAX * (SMAX + 1);
constexpr size_t scratch_cs = size_t(SMAX) * (SMAX + 1) + size_t(SMAX) * (4 * SMAX + 1);
constexpr size_t small_scratch_per_problem = scratch_evd > scratch_cs ? scratch_evd : scratch_cs;

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

// Dynamic LDS layout of the Cholesky-solve kernels: L (r x (r+1)) and X (r x (s+1)).
__host__ __device__ inline size_t cs_lds(int r, int s) {
  return (size_t(r) * (r + 1) + size_t(r) * (s + 1)) * sizeof(double);
}

// Problem b: D (r0 x r0, ld r0) at D + b sD, leading rb = dims[b] block used; B, X likewise.
__global__ __launch_bounds__(NT) void k_small_chol_solve(int r0, const int* __restrict__ dims, double* D, int64_t sD,
                                                         const double* B, int64_t ldb, int64_t sB, double* X,
                                                         int64_t ldx, int64_t sX, int s, int s0, double alpha,
                                                         int* flag, int factor, double* gw) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  const int b = blockIdx.x;
  const int r = dims ? dims[b] : r0;
  D += b * sD;
  B += b * sB;
  X += b * sX;
  gw += b * int64_t(small_scratch_per_problem);
  // rows r .. s0 - 1 of X are zero (directions this problem does not have)
  for (int e = threadIdx.x; e < (s0 - r) * s; e += NT) X[(r + e / s) * ldx + e % s] = 0.0;
  if (r == 0) return;
  const bool lds = cs_lds(r0, s) <= LDS_LIMIT;  // the launch's dynamic LDS is sized for r0 >= r
  double* Ls = lds ? sm : gw;
  const int ldl = r + 1, lx = s + 1;
  double* Xs = Ls + size_t(r) * ldl;
  for (int e = threadIdx.x; e < r * r; e += NT) Ls[(e / r) * ldl + e % r] = D[(e / r) * r0 + e % r];
  for (int e = threadIdx.x; e < r * s; e += NT) Xs[(e / s) * lx + e % s] = B[(e / s) * ldb + e % s];
  __syncthreads();
  if (factor) {
    const int info = chol_dev(Ls, r, ldl, &sinfo);
    if (info && threadIdx.x == 0) flag[0] = 1;
    for (int e = threadIdx.x; e < r * r; e += NT) D[(e / r) * r0 + e % r] = Ls[(e / r) * ldl + e % r];
    __syncthreads();
  }
  chol_solve_inplace(Ls, r, ldl, Xs, lx, s);
  for (int e = threadIdx.x; e < r * s; e += NT) X[(e / s) * ldx + e % s] = alpha * Xs[(e / s) * lx + e % s];
}

// Workspace for the Jacobi kernels: two n x (n+1) matrices + small arrays, in
// LDS when they fit, else in the caller's global scratch `gw`.
struct EvdSpace {
  double *A, *V, *cs, *d;
  int *pr, *ord;
  int ld;
};

__host__ __device__ inline size_t evd_bytes(int n) { return size_t(2) * n * (n + 1) * sizeof(double); }

__device__ EvdSpace evd_space(int n, double* sm, double* gw, double* small_d, int* small_i) {
  EvdSpace e;
  const bool lds = evd_bytes(n) <= LDS_LIMIT;
  double* base = lds ? sm : gw;
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
                                                   int64_t sT, int* out, const int* skip, double* gw) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  const int b = blockIdx.x;
  if (skip && skip[b]) return;
  G += b * sG;
  T += b * sT;
  gw += b * int64_t(small_scratch_per_problem);
  EvdSpace w = evd_space(s, sm, gw, sd, si);
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
                                                     int* flag, double* gw, double certify, int* ok) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  __shared__ double sshift, strace;
  __shared__ double red[NT];
  const int b = blockIdx.x;
  const int n = dims ? dims[b] : s;
  G += b * sG;
  Rinv += b * int64_t(s) * s;
  Racc += b * int64_t(s) * s;
  gw += b * int64_t(small_scratch_per_problem);
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
  const bool lds = evd_bytes(s) <= LDS_LIMIT;  // the launch's dynamic LDS is sized for s >= n
  const int ld = n + 1;
  double* A = lds ? sm : gw;
  double* X = A + size_t(n) * ld;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    A[i * ld + j] = 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift : 0.0);
    X[i * ld + j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  if (chol_dev(A, n, ld, &sinfo) && threadIdx.x == 0) flag[0] = 1;
  // X = L^{-1}: forward sweep on the identity (row m scaled, then the rows below updated)
  for (int m = 0; m < n; ++m) {
    const double inv = 1.0 / A[m * ld + m];
    for (int j = threadIdx.x; j <= m; j += NT) X[m * ld + j] *= inv;
    __syncthreads();
    for (int i = m + 1 + ty; i < n; i += 32) {
      const double l = A[i * ld + m];
      for (int j = tx; j <= m; j += 32) X[i * ld + j] -= l * X[m * ld + j];
    }
    __syncthreads();
  }
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
  // Racc <- R * Racc ; X reused for the product
  for (int e = threadIdx.x; e < n * n; e += NT) {
    const int i = e / n, j = e % n;
    double acc = 0.0;
    if (init) {
      acc = j >= i ? A[j * ld + i] : 0.0;
    } else {
      for (int m = i; m <= j; ++m) acc += A[m * ld + i] * Racc[m * s + j];
    }
    X[i * ld + j] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    Racc[e] = (i < n && j < n) ? X[i * ld + j] : 0.0;
  }
}

__global__ __launch_bounds__(NT) void k_small_nystrom(int s, int k, const double* C, const double* R, double eps_rel,
                                                      double* Wk, double* Ek, int* out, double* gw) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  __shared__ double dkeep[SMAX];
  __shared__ int ikeep[SMAX];
  __shared__ int nkeep;
  const int b = blockIdx.x;
  C += b * int64_t(s) * s;
  R += b * int64_t(s) * s;
  Wk += b * int64_t(s) * k;
  Ek += b * int64_t(k);
  out += 2 * b;
  gw += b * int64_t(small_scratch_per_problem);
  EvdSpace w = evd_space(s, sm, gw, sd, si);
  const int ld = w.ld;
  for (int e = threadIdx.x; e < s * s; e += NT) {  // symmetrised C
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
    int r = 0;
    if (dmax > 0.0)
      for (int i = 0; i < s; ++i)
        if (w.d[i] >= eps_rel * dmax) {
          ikeep[r] = i;
          dkeep[r] = w.d[i];
          ++r;
        }
    nkeep = r;
  }
  __syncthreads();
  const int r = nkeep;
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

__global__ __launch_bounds__(NT) void k_small_sym_evd(int m, const double* Ain, double* W, double* E, double* gw) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  EvdSpace w = evd_space(m, sm, gw, sd, si);
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

size_t evd_lds(int n) {
  const size_t b = evd_bytes(n);
  return b <= LDS_LIMIT ? b : 0;
}

}  // namespace

size_t small_scratch_elems() { return small_scratch_per_problem; }

void small_chol_solve(Batch bt, int r, double* D, int64_t sD, const double* B, int64_t ldb, int64_t sB, double* X,
                      int64_t ldx, int64_t sX, int s, int s0, double alpha, int* flag, double* gw, hipStream_t st) {
  if (bt.nb <= 0 || (r <= 0 && s0 <= 0)) return;  // s == 0: factor only
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t lb = cs_lds(r, s);
  k_small_chol_solve<<<bt.nb, NT, lb <= LDS_LIMIT ? lb : 0, st>>>(r, bt.dims, D, sD, B, ldb, sB, X, ldx, sX, s, s0,
                                                                   alpha, flag, 1, gw);
  NS_LAUNCH_CHECK();
}

void small_chol_apply(Batch bt, int r, const double* L, int64_t sL, const double* B, int64_t ldb, int64_t sB,
                      double* X, int64_t ldx, int64_t sX, int s, int s0, double alpha, double* gw, hipStream_t st) {
  if (bt.nb <= 0 || (r <= 0 && s0 <= 0) || s <= 0) return;
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t lb = cs_lds(r, s);
  k_small_chol_solve<<<bt.nb, NT, lb <= LDS_LIMIT ? lb : 0, st>>>(r, bt.dims, const_cast<double*>(L), sL, B, ldb, sB,
                                                                   X, ldx, sX, s, s0, alpha, nullptr, 0, gw);
  NS_LAUNCH_CHECK();
}

void small_svqb(int nb, int s, const double* G, int64_t sG, double drop2, double* T, int64_t sT, int* out,
                const int* skip, double* gw, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_svqb<<<nb, NT, evd_lds(s), st>>>(s, G, sG, drop2, T, sT, out, skip, gw);
  NS_LAUNCH_CHECK();
}

void small_cholqr(Batch bt, int s, const double* G, int64_t sG, const double* shift, double* Rinv, double* Racc,
                  int init, int* flag, double* gw, hipStream_t st, double certify, int* ok) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_cholqr<<<bt.nb, NT, evd_lds(s), st>>>(s, bt.dims, G, sG, shift, Rinv, Racc, init, flag, gw, certify, ok);
  NS_LAUNCH_CHECK();
}

void small_nystrom(int nb, int s, int k, const double* C, const double* R, double eps_rel, double* Wk, double* Ek,
                   int* out, double* gw, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_nystrom<<<nb, NT, evd_lds(s), st>>>(s, k, C, R, eps_rel, Wk, Ek, out, gw);
  NS_LAUNCH_CHECK();
}

void small_rowscale(int nb, int k, int ncols, const double* sigma, int64_t ssig, double* c, int64_t ldc, int64_t sc,
                    hipStream_t st) {
  if (k * ncols == 0 || nb == 0) return;
  k_small_rowscale<<<dim3((k * ncols + 255) / 256, nb), 256, 0, st>>>(k, ncols, sigma, ssig, c, ldc, sc);
  NS_LAUNCH_CHECK();
}

void small_gevd(int k, const double* A, const double* B, double* lam, double* C, double* Cl, int* flag, double* ws,
                double* gw, hipStream_t st) {
  if (k > SMAX) fail(INVALID_ARG, "matrix too large for the small dense kernels (limit 256)");
  double* L = ws;
  double* Linv = ws + size_t(k) * k;
  double* M = Linv + size_t(k) * k;
  double* W = M + size_t(k) * k;
  double* E = W + size_t(k) * k;
  k_gevd_reduce<<<1, NT, 0, st>>>(k, A, B, L, Linv, M, flag);
  NS_LAUNCH_CHECK();
  small_sym_evd(k, M, W, E, gw, st);
  k_gevd_back<<<1, 256, 0, st>>>(k, Linv, W, E, lam, C, Cl);
  NS_LAUNCH_CHECK();
}

void small_sym_evd(int m, const double* A, double* W, double* E, double* gw, hipStream_t st) {
  if (m > SMAX) fail(INVALID_ARG, "matrix too large for the small dense kernels (limit 256)");
  k_small_sym_evd<<<1, NT, evd_lds(m), st>>>(m, A, W, E, gw);
  NS_LAUNCH_CHECK();
}

}  // namespace ns
