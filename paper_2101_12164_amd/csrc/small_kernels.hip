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

// In-place lower Cholesky of A (n x n, stride lda).  Returns 0 or the 1-based
// index of the first non-positive pivot (the pivot is then taken as 1).
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

// X (r x s, stride ldx) <- (L L^T)^{-1} X, right-looking row sweeps, all
// columns and rows of a step in parallel.
__device__ void chol_solve_inplace(const double* L, int r, int ldl, double* X, int ldx, int s) {
  for (int m = 0; m < r; ++m) {  // forward: L y = x
    const double inv = 1.0 / L[m * ldl + m];
    for (int j = threadIdx.x; j < s; j += NT) X[m * ldx + j] *= inv;
    __syncthreads();
    const int rows = r - 1 - m;
    for (int t = threadIdx.x; t < rows * s; t += NT) {
      const int i = m + 1 + t / s, j = t % s;
      X[i * ldx + j] -= L[i * ldl + m] * X[m * ldx + j];
    }
    __syncthreads();
  }
  for (int m = r - 1; m >= 0; --m) {  // backward: L^T x = y
    const double inv = 1.0 / L[m * ldl + m];
    for (int j = threadIdx.x; j < s; j += NT) X[m * ldx + j] *= inv;
    __syncthreads();
    for (int t = threadIdx.x; t < m * s; t += NT) {
      const int i = t / s, j = t % s;
      X[i * ldx + j] -= L[m * ldl + i] * X[m * ldx + j];
    }
    __syncthreads();
  }
}

// Dynamic LDS layout of the Cholesky-solve kernels: L (r x (r+1)) and X (r x (s+1)).
__host__ __device__ inline size_t cs_lds(int r, int s) {
  return (size_t(r) * (r + 1) + size_t(r) * (s + 1)) * sizeof(double);
}

__global__ __launch_bounds__(NT) void k_small_chol_solve(int r, double* D, const double* B, int64_t ldb, double* X,
                                                         int64_t ldx, int s, double alpha, int* flag, int factor,
                                                         double* gw) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  const bool lds = cs_lds(r, s) <= LDS_LIMIT;
  double* Ls = lds ? sm : gw;
  const int ldl = r + 1, lx = s + 1;
  double* Xs = Ls + size_t(r) * ldl;
  for (int e = threadIdx.x; e < r * r; e += NT) Ls[(e / r) * ldl + e % r] = D[e];
  for (int e = threadIdx.x; e < r * s; e += NT) Xs[(e / s) * lx + e % s] = B[(e / s) * ldb + e % s];
  __syncthreads();
  if (factor) {
    const int info = chol_dev(Ls, r, ldl, &sinfo);
    if (info && threadIdx.x == 0) flag[0] = 1;
    for (int e = threadIdx.x; e < r * r; e += NT) D[e] = Ls[(e / r) * ldl + e % r];
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

__global__ __launch_bounds__(NT) void k_small_svqb(int s, const double* G, double drop2, double* T, int* out,
                                                   double* gw) {
  extern __shared__ double sm[];
  __shared__ double red[NT];
  __shared__ double sd[3 * SMAX];
  __shared__ int si[3 * SMAX];
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
  if (threadIdx.x == 0) out[0] = kept;
}

__global__ __launch_bounds__(NT) void k_small_cholqr(int s, const double* G, double shift_coef, double* Rinv,
                                                     double* Racc, int init, int* flag, double* gw, double certify,
                                                     int* ok) {
  extern __shared__ double sm[];
  __shared__ int sinfo;
  __shared__ double sshift, strace;
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < s; ++i) tr += G[i * s + i];
    sshift = shift_coef * tr;
    strace = tr;
  }
  __syncthreads();
  const double shift = sshift;
  const bool lds = evd_bytes(s) <= LDS_LIMIT;
  const int ld = s + 1;
  double* A = lds ? sm : gw;
  double* X = A + size_t(s) * ld;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    A[i * ld + j] = 0.5 * (G[i * s + j] + G[j * s + i]) + (i == j ? shift : 0.0);
    X[i * ld + j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  if (chol_dev(A, s, ld, &sinfo) && threadIdx.x == 0) flag[0] = 1;
  // X = L^{-1}: forward sweep on the identity
  for (int m = 0; m < s; ++m) {
    const double inv = 1.0 / A[m * ld + m];
    for (int j = threadIdx.x; j <= m; j += NT) X[m * ld + j] *= inv;
    __syncthreads();
    const int rows = s - 1 - m;
    for (int t = threadIdx.x; t < rows * (m + 1); t += NT) {
      const int i = m + 1 + t / (m + 1), j = t % (m + 1);
      X[i * ld + j] -= A[i * ld + m] * X[m * ld + j];
    }
    __syncthreads();
  }
  // Rinv = (L^{-1})^T (upper); R = L^T
  double fro = 0.0;
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    const double x = X[j * ld + i];
    Rinv[e] = x;
    fro += x * x;
  }
  if (ok) {
    // lambda_min(G) >= 1 / ||L^{-1}||_F^2 and lambda_max(G) <= trace(G): certify that no
    // singular value ratio of the block is at or below the drop tolerance
    __shared__ double red[NT];
    red[threadIdx.x] = fro;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double lmin_lb = 1.0 / red[0];
      ok[0] = (sinfo == 0 && lmin_lb > certify * strace) ? 1 : 0;
    }
  }
  __syncthreads();
  // Racc <- R * Racc ; X reused for the product
  for (int e = threadIdx.x; e < s * s; e += NT) {
    const int i = e / s, j = e % s;
    double acc = 0.0;
    if (init) {
      acc = j >= i ? A[j * ld + i] : 0.0;
    } else {
      for (int m = i; m <= j; ++m) acc += A[m * ld + i] * Racc[m * s + j];
    }
    X[i * ld + j] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < s * s; e += NT) Racc[e] = X[(e / s) * ld + e % s];
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

size_t evd_lds(int n) {
  const size_t b = evd_bytes(n);
  return b <= LDS_LIMIT ? b : 0;
}

}  // namespace

size_t small_scratch_elems() {
  const size_t evd = size_t(2) * SMAX * (SMAX + 1), cs = size_t(SMAX) * (SMAX + 1) + size_t(SMAX) * (4 * SMAX + 1);
  return evd > cs ? evd : cs;
}

void small_chol_solve(int r, double* D, const double* B, int64_t ldb, double* X, int64_t ldx, int s, double alpha,
                      int* flag, double* gw, hipStream_t st) {
  if (r <= 0) return;
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t b = cs_lds(r, s);
  k_small_chol_solve<<<1, NT, b <= LDS_LIMIT ? b : 0, st>>>(r, D, B, ldb, X, ldx, s, alpha, flag, 1, gw);
  NS_LAUNCH_CHECK();
}

void small_chol_apply(int r, const double* L, const double* B, int64_t ldb, double* X, int64_t ldx, int s,
                      double alpha, double* gw, hipStream_t st) {
  if (r <= 0 || s <= 0) return;
  if (r > SMAX || s > 4 * SMAX) fail(INVALID_ARG, "small Cholesky solve too large");
  const size_t b = cs_lds(r, s);
  k_small_chol_solve<<<1, NT, b <= LDS_LIMIT ? b : 0, st>>>(r, const_cast<double*>(L), B, ldb, X, ldx, s, alpha,
                                                            nullptr, 0, gw);
  NS_LAUNCH_CHECK();
}

void small_svqb(int s, const double* G, double drop2, double* T, int* out, double* gw, hipStream_t st) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_svqb<<<1, NT, evd_lds(s), st>>>(s, G, drop2, T, out, gw);
  NS_LAUNCH_CHECK();
}

void small_cholqr(int s, const double* G, double shift_coef, double* Rinv, double* Racc, int init, int* flag,
                  double* gw, hipStream_t st, double certify, int* ok) {
  if (s > SMAX) fail(INVALID_ARG, "k + p too large for the small dense kernels (limit 256)");
  k_small_cholqr<<<1, NT, evd_lds(s), st>>>(s, G, shift_coef, Rinv, Racc, init, flag, gw, certify, ok);
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
