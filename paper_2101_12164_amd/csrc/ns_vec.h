// Block-vector and small dense kernels (declarations).
//
// Block vectors are row-major n x c arrays over the interface rows.  The rows
// are split into segments, one per problem of a batch (a single problem is one
// segment): every reduction (Gram products, column norms, dot products) is
// taken per segment, over a fixed number of row chunks that depends only on
// the segment's row count, so a problem gives bitwise the same sums alone or
// inside a batch.  Per-segment small matrices are stacked with a stride.
#pragma once

#include "ns_internal.h"

namespace ns {

// Row segments (device arrays; host copies for sizing).
struct Seg {
  int n = 0;                     // segments
  int64_t rows = 0;              // total rows
  const int64_t* off = nullptr;  // [n + 1] first row of each segment
  const int* coff = nullptr;     // [n + 1] prefix of reduction chunks per segment
  const int* toff = nullptr;     // [n + 1] prefix of 64-row tiles per segment
  const int* rseg = nullptr;     // [rows] segment of each row
  int nchunk = 0, ntile = 0;     // totals
  int64_t first = 0;             // host copy of off[0]
  // [n] optional device flags: a segment flagged nonzero is passed over -- the Gram products leave its G_p as
  // it is, and the block updates copy X into Out (the orthonormalisation pass the flag makes unnecessary)
  const int* skip = nullptr;
};
// Owner of a segment description.
struct SegBuf {
  DBuf<int64_t> off;
  DBuf<int> coff, toff, rseg;
  std::vector<int64_t> h_off;
  Seg view;
  void build(const std::vector<int64_t>& offsets, hipStream_t st);
};
// reduction chunks of a segment with `rows` rows
int seg_chunks(int64_t rows);

// G_p (ra x rb, row-major, at G + p * gstride) = alpha * A_p^T B_p + beta * G_p for every segment p.
// work: at least gram_work_elems(seg, max(ra, rb)) doubles.
// With rscale, output row a of problem p is further scaled by rscale[p * rsstride + a].  symmetric: the caller
// knows A_p^T B_p to be symmetric (ra = rb, e.g. P^T S P): FP64 blocks then form its lower tiles only and mirror
// them (the result is exactly symmetric).
template <class TA, class TB>
void gram(const Seg& sg, const TA* A, int64_t lda, int ra, const TB* B, int64_t ldb, int rb, double* G,
          int64_t gstride, double alpha, double beta, double* work, hipStream_t st, const double* rscale = nullptr,
          int64_t rsstride = 0, bool symmetric = false);
size_t gram_work_elems(const Seg& sg, int maxw);

// Out_p = beta * Out_p + gamma * (X_p M_p + X2_p M2_p) on the rows of every segment p;
// M_p: rm x ncols (ld ldm) at M + p * mstride, FP64; X2 optional (rm2 = 0).  A skipped segment (sg.skip) gets
// Out = X.  Out may be X itself (same leading dimension, at most 256 columns, no X2): every workgroup reads
// only the rows it writes, all of them before its first store, and a skipped segment is left as it is.
template <class T>
void ts_update(const Seg& sg, int ncols, T* Out, int64_t ldo, double beta, double gamma, const T* X, int64_t ldx,
               int rm, const double* M, int64_t ldm, int64_t mstride, const T* X2 = nullptr, int64_t ldx2 = 0,
               int rm2 = 0, const double* M2 = nullptr, int64_t ldm2 = 0, int64_t m2stride = 0,
               hipStream_t st = nullptr);

template <class T, class U>
void convert_block(int64_t n, int ncols, const T* X, int64_t ldx, U* Y, int64_t ldy, hipStream_t st);

// out[p * ncols + c] = sum over the rows r of segment p of X[r, c]^2
template <class T>
void col_sumsq(const Seg& sg, int ncols, const T* X, int64_t ldx, double* out, double* work, hipStream_t st);

// out[p * ostride] = x_p^T y_p
void dot(const Seg& sg, const double* x, const double* y, double* out, int64_t ostride, double* work,
         hipStream_t st);
// y = a x + b y (no reduction)
void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);

// ---------------------------------------------------------------- PCG with per-problem state
// Scalars of problem p live at ps + p * PS: rho_j, rho_{j+1}, p^T q, ||r||^2, ||f||.  The iteration
// index j is a device counter, so one captured iteration body serves every iteration.
// done[p] freezes problem p's iterate once it met the tolerance (1) or its residual is not a number (2);
// it[p] is its iteration count; hist[p * hstride + j] the relative residual after iteration j (j = 0:
// initial).  Iterations j >= maxit change nothing.
constexpr int PS = 8;
constexpr int PS_RHO = 0, PS_RHO_NEW = 1, PS_PQ = 2, PS_RN2 = 3, PS_NF = 4;
struct PcgState {
  double* ps;
  int* done;
  int* it;
  int* ndone;  // number of problems done (device counter)
  int* j;      // current iteration (device counter)
  double* hist;
  int64_t hstride;
  double rtol;
  int maxit;
};
// part[c] = x^T y over the rows of reduction chunk c (one value per chunk of every segment)
void dot_partials(const Seg& sg, const double* x, const double* y, double* part, hipStream_t st);
// w += alpha_p p, r -= alpha_p q for problems not done (alpha_p = rho_j / (p^T q)_p, (p^T q)_p summed from the
// chunk partials pq_part of dot_partials), then ||r||^2 per problem (chunk partials in work), the stopping test,
// it and hist.
void pcg_update_wr(const Seg& sg, const PcgState& s, double* w, double* r, const double* p, const double* q,
                   const double* pq_part, double* work, hipStream_t st);
// p = z + beta_p p with beta_p = rho_{j+1} / rho_j, rho_{j+1} = (r^T z)_p summed from the chunk partials rz_part.
void pcg_update_p(const Seg& sg, const PcgState& s, const double* z, double* p, const double* rz_part,
                  hipStream_t st);
// rho_j <- rho_{j+1} for every problem; j <- j + 1.
void pcg_advance(int nseg, const PcgState& s, hipStream_t st);
// hist[., 0] and done for the initial residual: rel = sqrt(rn2) / nf; j <- 0.
void pcg_init_check(int nseg, const PcgState& s, hipStream_t st);

// ---------------------------------------------------------------- small dense (one workgroup per problem)
// Problem b (0 <= b < nb) of a batch uses the matrices at base + b * stride (row-major FP64, device) and
// dimension dim[b] (dims == nullptr: the uniform value r); a problem of dimension 0 gets zero outputs.
struct Batch {
  int nb = 1;
  const int* dims = nullptr;
};
// Global scratch for launches whose matrices do not fit in LDS: `stride` doubles per problem, valid for
// dimensions <= n and column counts <= c; p == nullptr when every such launch fits in LDS.  A launch that
// needs more than the scratch provides fails with INVALID_ARG.
struct SmallWs {
  double* p = nullptr;
  int64_t stride = 0;
  int n = 0, c = 0;
  // eigen-decompositions of n x n matrices past the LDS limit: per problem, a rotation log of jstride doubles
  // and a status word (nullptr when not needed or not provided)
  double* jlog = nullptr;
  int64_t jstride = 0;
  int* jstat = nullptr;
};
// doubles per problem for dimensions <= n and column counts <= c (0 when everything fits in LDS)
size_t small_scratch_elems(int n, int c);
// doubles per problem of the Cholesky solve / apply kernels for an r x r factor and c columns (0: in LDS)
size_t small_chol_scratch_elems(int r, int c);
// a scratch for nb problems (buf is allocated only when needed); evd: also the rotation logs of the
// eigen-decompositions (the setup's Nystrom core and block-CG orthonormalisation)
SmallWs small_ws(DBuf<double>& buf, int nb, int n, int c, bool evd = false);

// L (in place of D, lower) = chol(D) for an r x r SPD D; X = alpha * D^{-1} B (B: r x s, ld ldb; X ld ldx).
// Rows r..s0-1 of X are set to zero (s0 = rows of the stacked X, pass r when unused).  s = 0: factor only.
// flag[0] is set to 1 when some D is not numerically SPD.
void small_chol_solve(Batch bt, int r, double* D, int64_t sD, const double* B, int64_t ldb, int64_t sB, double* X,
                      int64_t ldx, int64_t sX, int s, int s0, double alpha, int* flag, const SmallWs& ws,
                      hipStream_t st);
// X = alpha * (L L^T)^{-1} B with L from small_chol_solve.
void small_chol_apply(Batch bt, int r, const double* L, int64_t sL, const double* B, int64_t ldb, int64_t sB,
                      double* X, int64_t ldx, int64_t sX, int s, int s0, double alpha, const SmallWs& ws,
                      hipStream_t st);
// Orthonormalising transform of a block with Gram matrix G (s x s): T[:, c] = u_c / sqrt(lambda_c)
// for the eigenpairs with lambda_c > drop2 * lambda_max, descending, zero columns after them;
// out[b] = number kept.  Problems with skip[b] != 0 are left untouched.
void small_svqb(int nb, int s, const double* G, int64_t sG, double drop2, double* T, int64_t sT, int* out,
                const int* skip, const SmallWs& ws, hipStream_t st);
// R = chol(G + shift_b * trace(G) * I)^T (upper) on the leading dim_b block (zero elsewhere);
// Rinv = R^{-1}; Racc <- R * Racc (or R when init).  shift_b = shift[b] when shift != nullptr.
// With ok != nullptr: ok[b] = 1 when the Cholesky succeeded and a guaranteed lower bound of lambda_min(G)
// exceeds certify times an upper bound of lambda_max(G) (no direction falls below that ratio); single[b] = 1
// when the same bounds for the column-equilibrated D G D (unit diagonal) certify a condition number below
// 1 / single_thr, small enough for one Cholesky-QR pass (its rounding depends on that scaled condition).
void small_cholqr(Batch bt, int s, const double* G, int64_t sG, const double* shift, double* Rinv, double* Racc,
                  int init, int* flag, const SmallWs& ws, hipStream_t st, double certify = 0.0, int* ok = nullptr,
                  double single_thr = 0.0, int* single = nullptr);
// Nystrom core: EVD of sym(C), keep eigenvalues >= eps_rel * max; T = (R V1) D1^{-1} (R V1)^T;
// EVD of T descending; Wk = first k' eigenvectors (s x k, ld k), Ek = eigenvalues; out[2b..] = {r, k'}.
// (A Cholesky of C that certifies every eigenvalue above the threshold replaces the first EVD.)
void small_nystrom(int nb, int s, int k, const double* C, const double* R, double eps_rel, double* Wk, double* Ek,
                   int* out, const SmallWs& ws, hipStream_t st);
// Symmetric EVD (descending) of an m x m matrix: W (m x m) eigenvectors in columns, E eigenvalues.
void small_sym_evd(int m, const double* A, double* W, double* E, const SmallWs& ws, hipStream_t st);
// Generalised symmetric EVD A c = lambda B c (B SPD), ascending: lam (k), C (k x k, C^T B C = I),
// Cl = -C diag(lambda); ws: 4 k^2 + k doubles; flag[0] = 1 when B is not numerically SPD.
void small_gevd(int k, const double* A, const double* B, double* lam, double* C, double* Cl, int* flag, double* ws,
                const SmallWs& sw, hipStream_t st);

}  // namespace ns
