// One-workgroup dense kernels on the s x s matrices of the method (s = k + p):
// Cholesky and solves for block CG, the eigen-decomposition based
// orthonormalisation of a block, shifted Cholesky-QR, and the Nystrom core of
// Algorithm alg:nystrom (EVD of C, threshold, T, EVD of T).  Symmetric
// eigen-decompositions use the cyclic two-sided Jacobi method with a
// round-robin ordering, so all rotations of a round are independent.
#include "ns_vec.h"

namespace ns {
namespace {

constexpr int NT = 1024;                  // threads per workgroup
constexpr size_t LDS_LIMIT = 136 * 1024;  // dynamic LDS used when the matrices fit

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

// Cyclic Jacobi: A (n x n, row-major, symmetric) is diagonalised in place; V
// receives the eigenvectors in its columns.  cs: 2*n doubles, pr: n ints.
__device__ void jacobi(double* A, double* V, int n, double* cs, int* pr, double* red) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += NT) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  if (n < 2) return;
  const int m = n + (n & 1);
  const int half = m / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += NT) {
      const double v = A[e] * A[e];
      tot += v;
      if (e / n != e % n) off += v;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (!(off > 1e-30 * tot)) break;
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
          const double apq = A[p * n + q];
          if (fabs(apq) > 1e-300) {
            const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        } else {
          p = -1;
        }
        pr[2 * tid] = p;
        pr[2 * tid + 1] = q;
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
      }
      __syncthreads();
      for (int t = tid; t < half * n; t += NT) {  // rows: A <- J^T A
        const int k = t / n, j = t % n;
        const int p = pr[2 * k];
        if (p < 0) continue;
        const int q = pr[2 * k + 1];
        const double c = cs[2 * k], s = cs[2 * k + 1];
        const double ap = A[p * n + j], aq = A[q * n + j];
        A[p * n + j] = c * ap - s * aq;
        A[q * n + j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int t = tid; t < half * n; t += NT) {  // columns: A <- A J, V <- V J
        const int k = t / n, i = t % n;
        const int p = pr[2 * k];
        if (p < 0) continue;
        const int q = pr[2 * k + 1];
        const double c = cs[2 * k], s = cs[2 * k + 1];
        const double ap = A[i * n + p], aq = A[i * n + q];
        A[i * n + p] = c * ap - s * aq;
        A[i * n + q] = s * ap + c * aq;
        const double vp = V[i * n + p], vq = V[i * n + q];
        V[i * n + p] = c * vp - s * vq;
        V[i * n + q] = s * vp + c * vq;
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

// In-place lower Cholesky of A (n x n, row-major, lda).  Returns 0 or the
// 1-based index of the first non-positive pivot (the pivot is then set to 1).
__device__ int chol_dev(double* A, int n, int lda, int* sinfo) {
  if (threadIdx.x == 0) *sinfo = 0;
  __syncthreads();
  for (int c = 0; c < n; ++c) {
    if (threadIdx.x == 0) {
      double d = A[c * lda + c];
      if (!(d > 0.0)) {
        if (*sinfo == 0) *sinfo = c + 1;
        d = 1.0;
      }
      A[c * lda + c] = sqrt(d);
    }
    __syncthreads();
    const double dinv = 1.0 / A[c * lda + c];
    for (int r = c + 1 + threadIdx.x; r < n; r += NT) A[r * lda + c] *= dinv;
    __syncthreads();
    const int m = n - 1 - c;
    for (int idx = threadIdx.x; idx < m * m; idx += NT) {
      const int q = c + 1 + idx / m, r = c + 1 + idx % m;
      if (r >= q) A[r * lda + q] -= A[r * lda + c] * A[q * lda + c];
    }
    __syncthreads();
  }
  const int info = *sinfo;
  __syncthreads();
  return info;
}

// X (r x s) = alpha * (L L^T)^{-1} B; one thread per column.
__device__ void chol_solve_dev(const double* L, int r, int ldl, const double* B, int64_t ldb, double* X, int64_t ldx,
                               int s, double alpha) {
  for (int j = threadIdx.x; j < s; j += NT) {
    for (int i = 0; i < r; ++i) {  // forward: L y = b
      double acc = B[i * ldb + j];
      for (int m = 0; m < i; ++m) acc -= L[i * ldl + m] * X[m * ldx + j];
      X[i * ldx + j] = acc / L[i * ldl + i];
    }
    for (int i = r - 1; i >= 0; --i) {  // backward: L^T x = y
      double acc = X[i * ldx + j];
      for (int m = i + 1; m < r; ++m) acc -= L[m * ldl + i] * X[m * ldx + j];
      X[i * ldx + j] = acc / L[i * ldl + i];
    }
    for (int i = 0; i < r; ++i) X[i * ldx + j] *= alpha;
  }
  __syncthreads();
}

__global__ __launch_bounds__(NT) void k_small_chol_solve(int r, double* D, const double* B, int64_t ldb, double* X,
                                                         int64_t ldx, int s, double alpha, int* flag) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  const bool lds = size_t(r) * r * sizeof(double) <= LDS_LIMIT;
  double* A = lds ? sm : D;
  if (lds)
    for (int e = threadIdx.x; e < r * r; e += NT) A[e] = D[e];
  __syncthreads();
  const int info = chol_dev(A, r, r, &sinfo);
  if (info && threadIdx.x == 0) flag[0] = 1;
  if (lds)
    for (int e = threadIdx.x; e < r * r; e += NT) D[e] = A[e];
  __syncthreads();
  chol_solve_dev(A, r, r, B, ldb, X, ldx, s, alpha);
}

__global__ __launch_bounds__(NT) void k_small_chol_apply(int r, const double* Lg, const double* B, int64_t ldb,
                                                         double* X, int64_t ldx, int s, double alpha) {
  extern __shared__ double sm[];
  const bool lds = size_t(r) * r * sizeof(double) <= LDS_LIMIT;
  const double* L = Lg;
  if (lds) {
    for (int e = threadIdx.x; e < r * r; e += NT) sm[e] = Lg[e];
    L = sm;
  }
  __syncthreads();
  chol_solve_dev(L, r, r, B, ldb, X, ldx, s, alpha);
}

// Workspace for the Jacobi kernels: two n x n matrices + small arrays, in LDS
// when they fit, else in the caller's global scratch `gw` (2 n^2 doubles).
struct EvdSpace {
  double *A, *V, *cs, *d;
  int *pr, *ord;
};

__device__ EvdSpace evd_space(int n, double* sm, double* gw, double* small_d, int* small_i) {
  EvdSpace e;
  const bool lds = size_t(2) * n * n * sizeof(double) <= LDS_LIMIT;
  double* base = lds ? sm : gw;
  e.A = base;
  e.V = base + size_t(n) * n;
  e.cs = small_d;
  e.d = small_d + 2 * n;
  e.pr = small_i;
  e.ord = small_i + 2 * n;
  return e;
}

constexpr int SMAX = 256;  // largest s supported by the small kernels

__global__ __launch_bounds__(NT) void k_small_svqb(int s, const double* G, double drop2, double* T, int* out,
                                                   double* gw) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  EvdSpace w = evd_space(s, sm, gw, sd, si);
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    w.A[e] = 0.5 * (G[i * s + j] + G[j * s + i]);
  }
  __syncthreads();
  jacobi(w.A, w.V, s, w.cs, w.pr, red);
  for (int i = threadIdx.x; i < s; i += NT) w.d[i] = w.A[i * s + i];
  __syncthreads();
  sort_desc(w.d, s, w.ord);
  const double lmax = w.d[w.ord[0]];
  int kept = 0;
  for (int c = 0; c < s; ++c) {
    const double l = w.d[w.ord[c]];
    if (l > 0.0 && l > drop2 * lmax) ++kept;
    else break;
  }
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, c = e % s;
    T[e] = c < kept ? w.V[i * s + w.ord[c]] / sqrt(w.d[w.ord[c]]) : 0.0;
  }
  if (threadIdx.x == 0) out[0] = kept;
}

__global__ __launch_bounds__(NT) void k_small_cholqr(int s, const double* G, double shift_coef, double* Rinv,
                                                     double* Racc, int init, int* flag, double* gw) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  __shared__ double sshift;
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < s; ++i) tr += G[i * s + i];
    sshift = shift_coef * tr;
  }
  __syncthreads();
  const double shift = sshift;
  const bool lds = size_t(2) * s * s * sizeof(double) <= LDS_LIMIT;
  double* A = lds ? sm : gw;
  double* X = A + size_t(s) * s;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    A[e] = 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift : 0.0);
  }
  __syncthreads();
  if (chol_dev(A, s, s, &sinfo) && threadIdx.x == 0) flag[0] = 1;
  // X = L^{-1} (lower), one thread per column
  for (int c = threadIdx.x; c < s; c += NT) {
    for (int r = 0; r < c; ++r) X[r * s + c] = 0.0;
    X[c * s + c] = 1.0 / A[c * s + c];
    for (int r = c + 1; r < s; ++r) {
      double acc = 0.0;
      for (int m = c; m < r; ++m) acc += A[r * s + m] * X[m * s + c];
      X[r * s + c] = -acc / A[r * s + r];
    }
  }
  __syncthreads();
  // Rinv = (L^{-1})^T (upper); R = L^T
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    Rinv[e] = X[j * s + i];
  }
  __syncthreads();
  // Racc <- R * Racc ; reuse X for the product
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    double acc = 0.0;
    if (init) {
      acc = j >= i ? A[j * s + i] : 0.0;
    } else {
      for (int m = i; m <= j; ++m) acc += A[m * s + i] * Racc[m * s + j];
    }
    X[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * s; e += NT) Racc[e] = X[e];
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
  EvdSpace w = evd_space(s, sm, gw, sd, si);
  for (int e = threadIdx.x; e < s * s; e += NT) {  // symmetrised C (step: EVD of C)
    const int i = e / s, j = e % s;
    w.A[e] = 0.5 * (C[i * s + j] + C[j * s + i]);
  }
  __syncthreads();
  jacobi(w.A, w.V, s, w.cs, w.pr, red);
  for (int i = threadIdx.x; i < s; i += NT) w.d[i] = w.A[i * s + i];
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
  // M = R V_1 (s x r) into A
  for (int e = threadIdx.x; e < s * r; e += NT) {
    const int i = e / r, c = e % r;
    double acc = 0.0;
    for (int m = i; m < s; ++m) acc += R[i * s + m] * w.V[m * s + ikeep[c]];
    w.A[i * r + c] = acc;
  }
  __syncthreads();
  // T = M D_1^{-1} M^T into V
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    double acc = 0.0;
    for (int c = 0; c < r; ++c) acc += w.A[i * r + c] * w.A[j * r + c] / dkeep[c];
    w.V[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * s; e += NT) {  // symmetrise T
    const int i = e / s, j = e % s;
    if (j > i) {
      const double a = 0.5 * (w.V[i * s + j] + w.V[j * s + i]);
      w.V[i * s + j] = a;
      w.V[j * s + i] = a;
    }
  }
  __syncthreads();
  jacobi(w.V, w.A, s, w.cs, w.pr, red);  // EVD of T: eigenvectors in A
  for (int i = threadIdx.x; i < s; i += NT) w.d[i] = w.V[i * s + i];
  __syncthreads();
  sort_desc(w.d, s, w.ord);
  const int kk = k < r ? k : r;
  for (int e = threadIdx.x; e < s * k; e += NT) {
    const int i = e / k, c = e % k;
    Wk[e] = c < kk ? w.A[i * s + w.ord[c]] : 0.0;
  }
  for (int c = threadIdx.x; c < k; c += NT) Ek[c] = c < kk ? w.d[w.ord[c]] : 0.0;
  if (threadIdx.x == 0) {
    out[0] = r;
    out[1] = kk;
  }
}

__global__ void k_small_rowscale(int k, int ncols, const double* sigma, double* c, int64_t ldc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * ncols) return;
  const int i = idx / ncols, j = idx % ncols;
  c[i * ldc + j] *= sigma[i];
}

__global__ __launch_bounds__(NT) void k_small_sym_evd(int m, const double* Ain, double* W, double* E, double* gw) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
  EvdSpace w = evd_space(m, sm, gw, sd, si);
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e / m, j = e % m;
    w.A[e] = 0.5 * (Ain[i * m + j] + Ain[j * m + i]);
  }
  __syncthreads();
  jacobi(w.A, w.V, m, w.cs, w.pr, red);
  for (int i = threadIdx.x; i < m; i += NT) w.d[i] = w.A[i * m + i];
  __syncthreads();
  sort_desc(w.d, m, w.ord);
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const int i = e / m, c = e % m;
    W[e] = w.V[i * m + w.ord[c]];
  }
  for (int c = threadIdx.x; c < m; c += NT) E[c] = w.d[w.ord[c]];
}

size_t evd_lds(int n) {
  const size_t b = size_t(2) * n * n * sizeof(double);
  return b <= LDS_LIMIT ? b : 0;
}

}  // namespace

void small_chol_solve(int r, double* D, const double* B, int64_t ldb, double* X, int64_t ldx, int s, double alpha,
                      int* flag, hipStream_t st) {
  if (r <= 0) return;
  const size_t b = size_t(r) * r * sizeof(double);
  k_small_chol_solve<<<1, NT, b <= LDS_LIMIT ? b : 0, st>>>(r, D, B, ldb, X, ldx, s, alpha, flag);
  NS_LAUNCH_CHECK();
}

void small_chol_apply(int r, const double* L, const double* B, int64_t ldb, double* X, int64_t ldx, int s,
                      double alpha, hipStream_t st) {
  if (r <= 0) return;
  const size_t b = size_t(r) * r * sizeof(double);
  k_small_chol_apply<<<1, NT, b <= LDS_LIMIT ? b : 0, st>>>(r, L, B, ldb, X, ldx, s, alpha);
  NS_LAUNCH_CHECK();
}

size_t small_scratch_elems() { return size_t(2) * SMAX * SMAX; }

void small_svqb(int s, const double* G, double drop2, double* T, int* out, double* gw, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_svqb<<<1, NT, evd_lds(s), st>>>(s, G, drop2, T, out, gw);
  NS_LAUNCH_CHECK();
}

void small_cholqr(int s, const double* G, double shift_coef, double* Rinv, double* Racc, int init, int* flag,
                  double* gw, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_cholqr<<<1, NT, evd_lds(s), st>>>(s, G, shift_coef, Rinv, Racc, init, flag, gw);
  NS_LAUNCH_CHECK();
}

void small_nystrom(int s, int k, const double* C, const double* R, double eps_rel, double* Wk, double* Ek, int* out,
                   double* gw, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_nystrom<<<1, NT, evd_lds(s), st>>>(s, k, C, R, eps_rel, Wk, Ek, out, gw);
  NS_LAUNCH_CHECK();
}

void small_rowscale(int k, int ncols, const double* sigma, double* c, int64_t ldc, hipStream_t st) {
  if (k * ncols == 0) return;
  k_small_rowscale<<<(k * ncols + 255) / 256, 256, 0, st>>>(k, ncols, sigma, c, ldc);
  NS_LAUNCH_CHECK();
}

void small_sym_evd(int m, const double* A, double* W, double* E, double* gw, hipStream_t st) {
  if (m > SMAX) fail(INVALID_ARG, "matrix too large for the small dense kernels (limit 256)");
  k_small_sym_evd<<<1, NT, evd_lds(m), st>>>(m, A, W, E, gw);
  NS_LAUNCH_CHECK();
}

}  // namespace ns
