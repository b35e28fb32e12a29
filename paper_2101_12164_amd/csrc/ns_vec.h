// Block-vector and small dense kernels (declarations).
#pragma once

#include "ns_internal.h"

namespace ns {

// G (ra x rb, row-major) = alpha * A^T B + beta * G; A: n x ra (ld lda), B: n x rb.
// work: at least gram_work_elems(max(ra, rb)) doubles.
template <class TA, class TB>
void gram(int64_t n, const TA* A, int64_t lda, int ra, const TB* B, int64_t ldb, int rb, double* G, double alpha,
          double beta, double* work, hipStream_t st);
size_t gram_work_elems(int maxw);

// Out = beta * Out + gamma * (X M + X2 M2); M: rm x ncols (ld ldm), FP64; X2 optional (rm2 = 0).
template <class T>
void ts_update(int64_t n, int ncols, T* Out, int64_t ldo, double beta, double gamma, const T* X, int64_t ldx, int rm,
               const double* M, int64_t ldm, const T* X2, int64_t ldx2, int rm2, const double* M2, int64_t ldm2,
               hipStream_t st);

template <class T, class U>
void convert_block(int64_t n, int ncols, const T* X, int64_t ldx, U* Y, int64_t ldy, hipStream_t st);

// out[c] = sum_r X[r, c]^2
template <class T>
void col_sumsq(int64_t n, int ncols, const T* X, int64_t ldx, double* out, double* work, hipStream_t st);

void dot(int64_t n, const double* x, const double* y, double* out, double* work, hipStream_t st);
void pcg_update_wr(int64_t n, const double* sc, int it, double* w, double* r, const double* p, const double* q,
                   double* rn2_out, double* work, hipStream_t st);
void pcg_update_p(int64_t n, const double* sc, int it, const double* z, double* p, hipStream_t st);
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);

// ---------------------------------------------------------------- small dense (one workgroup)
// All matrices row-major FP64 in device memory; gw: global scratch of
// small_scratch_elems() doubles, used when a matrix does not fit in LDS.

// L (in place of D, lower) = chol(D) for an r x r SPD D; X = alpha * D^{-1} B (B: r x s, ld ldb; X ld ldx).
// flag[0] is set to 1 when D is not numerically SPD.
void small_chol_solve(int r, double* D, const double* B, int64_t ldb, double* X, int64_t ldx, int s, double alpha,
                      int* flag, double* gw, hipStream_t st);
// X = alpha * (L L^T)^{-1} B with L from small_chol_solve.
void small_chol_apply(int r, const double* L, const double* B, int64_t ldb, double* X, int64_t ldx, int s,
                      double alpha, double* gw, hipStream_t st);
// Orthonormalising transform of a block with Gram matrix G (s x s): T[:, c] = u_c / sqrt(lambda_c)
// for the eigenpairs with lambda_c > drop2 * lambda_max, descending; out[0] = number kept.
void small_svqb(int s, const double* G, double drop2, double* T, int* out, double* gw, hipStream_t st);
// R = chol(G + shift_coef * trace(G) * I)^T (upper); Rinv = R^{-1}; Racc <- R * Racc (or R when init).
// With ok != NULL: ok[0] = 1 when the Cholesky succeeded and 1/||R^{-1}||_F^2 > certify * trace(G), which
// proves lambda_min(G) / lambda_max(G) > certify (so no direction falls below that ratio).
void small_cholqr(int s, const double* G, double shift_coef, double* Rinv, double* Racc, int init, int* flag,
                  double* gw, hipStream_t st, double certify = 0.0, int* ok = nullptr);
// Nystrom core: EVD of sym(C), keep eigenvalues >= eps_rel * max; T = (R V1) D1^{-1} (R V1)^T;
// EVD of T descending; Wk = first k' eigenvectors (s x k, ld k), Ek = eigenvalues; out = {r, k'}.
void small_nystrom(int s, int k, const double* C, const double* R, double eps_rel, double* Wk, double* Ek, int* out,
                   double* gw, hipStream_t st);
// c[i, j] *= sigma[i] for i < k, j < ncols (ld ldc)
void small_rowscale(int k, int ncols, const double* sigma, double* c, int64_t ldc, hipStream_t st);
// Symmetric EVD (descending) of an m x m matrix: W (m x m) eigenvectors in columns, E eigenvalues.
void small_sym_evd(int m, const double* A, double* W, double* E, double* gw, hipStream_t st);
// scratch (doubles) the small EVD kernels need in global memory when s is large
size_t small_scratch_elems();

}  // namespace ns
