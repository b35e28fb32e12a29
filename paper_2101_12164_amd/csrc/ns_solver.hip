// Host orchestration and the C ABI: Algorithm alg:prec1 (setup), the
// preconditioner application (eq. left_prec_mat or the adapted deflation form)
// and the block LDL^T solve with PCG on the Schur complement (eqs. A_LDLT,
// Sx=b).  Every numerical step runs in the library's HIP kernels; the host only
// sequences launches and reads back convergence scalars.
#include <cmath>
#include <cstring>

#include "ns_handle.h"
#include "ns_vec.h"

namespace ns {

[[noreturn]] void fail(int status, const std::string& msg) { throw Error{status, msg}; }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  const char* base = strrchr(file, '/');
  fail(HIP, std::string(what) + ": " + hipGetErrorString(e) + " (" + (base ? base + 1 : file) + ":" +
                std::to_string(line) + ")");
}

namespace {

thread_local std::string g_last_error = "no error";

struct Events {
  hipEvent_t e[8];
  hipStream_t st;
  explicit Events(hipStream_t s) : st(s) {
    for (auto& x : e) NS_HIP(hipEventCreate(&x));
  }
  ~Events() {
    for (auto& x : e) (void)hipEventDestroy(x);
  }
  void rec(int i) { NS_HIP(hipEventRecord(e[i], st)); }
  double sec(int a, int b) {
    float ms = 0.f;
    NS_HIP(hipEventSynchronize(e[b]));
    NS_HIP(hipEventElapsedTime(&ms, e[a], e[b]));
    return ms * 1e-3;
  }
};

// Small FP64 matrices of one setup, carved from a single allocation.
struct SmallMats {
  DBuf<double> buf;
  double *Delta, *G1, *alpha, *G2, *beta, *Gorth, *Torth, *Rinv, *Racc, *C, *Wk, *Ek, *colsq, *nF2;
  DBuf<int> ibuf;
  int *flag, *rank;
  void init(int s) {
    const size_t m = size_t(s) * s;
    buf.alloc(12 * m + 3 * s + 8);
    double* p = buf.p;
    for (double** q : {&Delta, &G1, &alpha, &G2, &beta, &Gorth, &Torth, &Rinv, &Racc, &C, &Wk}) {
      *q = p;
      p += m;
    }
    Ek = p;
    p += s;
    colsq = p;
    p += s;
    nF2 = p;
    ibuf.alloc(8);
    NS_HIP(hipMemset(ibuf.p, 0, 8 * sizeof(int)));
    flag = ibuf.p;
    rank = ibuf.p + 4;
  }
};

template <class T>
void read_back(Handle& h, T* host, const T* dev, size_t count) {
  NS_HIP(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, h.stream));
  NS_HIP(hipStreamSynchronize(h.stream));
}

void check_chol(Handle& h, int level, ns_setup_info* info) {
  int e[3];
  read_back(h, e, h.dflags.p + 8, 3);
  if (!e[0]) return;
  int blk = e[1];
  if (level == 2) blk = -2 - blk;
  if (level == 3) blk = -1;
  if (info) {
    info->bad_block = blk;
    info->bad_col = e[2];
  }
  fail(NOT_SPD, "Cholesky pivot <= 0 in block " + std::to_string(blk) + ", column " + std::to_string(e[2]));
}

// Orthonormal basis of the columns of V (n_G x s, ld s) into P, dropping
// directions with singular value <= drop * sigma_max.  When a Cholesky of the
// Gram matrix certifies that every singular value ratio exceeds the drop
// tolerance, nothing is dropped and Cholesky-QR2 yields a basis of the same
// span; otherwise the Gram matrix is eigen-decomposed (SVQB: keep the
// eigenpairs above drop^2 * lambda_max) followed by one Cholesky-QR pass.
// Returns the number of columns kept.  Q is used as scratch.
template <class T>
int orth(Handle& h, SmallMats& sm, DBuf<double>& work, const T* V, T*& P, T*& Q, int s) {
  hipStream_t st = h.stream;
  const int64_t nG = h.nG;
  const double drop2 = h.drop_rel * h.drop_rel;
  gram<T, T>(nG, V, s, s, V, s, s, sm.Gorth, 1.0, 0.0, work, st);
  small_cholqr(s, sm.Gorth, 0.0, sm.Rinv, sm.Racc, 1, sm.flag + 1, h.small.p, st, drop2, sm.rank + 2);
  int okv = 0;
  read_back(h, &okv, sm.rank + 2, 1);
  int r = s;
  if (okv) {
    ts_update<T>(nG, s, P, s, 0.0, 1.0, V, s, s, sm.Rinv, s, nullptr, 0, 0, nullptr, 0, st);
  } else {
    small_svqb(s, sm.Gorth, drop2, sm.Torth, sm.rank, h.small.p, st);
    read_back(h, &r, sm.rank, 1);
    if (r == 0) return 0;
    ts_update<T>(nG, r, P, s, 0.0, 1.0, V, s, s, sm.Torth, s, nullptr, 0, 0, nullptr, 0, st);
  }
  gram<T, T>(nG, P, s, r, P, s, r, sm.Gorth, 1.0, 0.0, work, st);
  small_cholqr(r, sm.Gorth, 0.0, sm.Rinv, sm.Racc, 1, sm.flag + 1, h.small.p, st);
  ts_update<T>(nG, r, Q, s, 0.0, 1.0, P, s, r, sm.Rinv, r, nullptr, 0, 0, nullptr, 0, st);
  std::swap(P, Q);
  return r;
}

// Breakdown-free block PCG on S_Gamma D = W Omega, preconditioned by
// A_Gamma^{-1}, from D = 0 (the inner solve of Algorithm alg:prec1, steps 2-4,
// in the shifted Schur form: A_Gamma D = A_GammaI S_I^{-1} A_IGamma Omega by
// eq. S-1).  Writes D (FP64, n_G x s) and returns the iteration count.
template <class T>
int block_pcg(Handle& h, SmallMats& sm, const double* Omega, double* D, double& relres, bool& converged) {
  hipStream_t st = h.stream;
  const int s = h.s;
  const int64_t nG = h.nG;
  DBuf<T> Om, X, R, Pb, Qb, Z;
  for (DBuf<T>* b : {&X, &R, &Pb, &Qb, &Z}) b->alloc(nG * s);
  DBuf<double> work;
  work.alloc(gram_work_elems(s));
  const T* Omt;
  if constexpr (sizeof(T) == 8) {
    Omt = Omega;
  } else {
    Om.alloc(nG * s);
    convert_block<double, float>(nG, s, Omega, s, Om.p, s, st);
    Omt = Om.p;
  }
  T* P = Pb.p;
  T* Q = Qb.p;
  op_schur<T>(h, Omt, s, R.p, s, s, /*w_only=*/true);  // F = W Omega
  NS_HIP(hipMemsetAsync(X.p, 0, nG * s * sizeof(T), st));
  col_sumsq<T>(nG, s, R.p, s, sm.nF2, work, st);
  std::vector<double> nF2(s), nr2(s);
  read_back(h, nF2.data(), sm.nF2, s);
  auto max_rel = [&](const std::vector<double>& r2) {
    double m = 0.0;
    for (int j = 0; j < s; ++j)
      if (nF2[j] > 0.0) m = std::max(m, std::sqrt(r2[j] / nF2[j]));
    return m;
  };
  relres = max_rel(nF2);
  converged = relres <= h.tol_inner;
  int it = 0;
  if (!converged) {
    op_gamma_solve<T>(h, R.p, s, Z.p, s, s);
    int r = orth<T>(h, sm, work, Z.p, P, Q, s);
    while (r > 0 && it < h.max_inner) {
      ++it;
      op_schur<T>(h, P, s, Q, s, r, false);                                   // Q = S P
      gram<T, T>(nG, P, s, r, Q, s, r, sm.Delta, 1.0, 0.0, work, st);       // Delta = P^T Q
      gram<T, T>(nG, P, s, r, R.p, s, s, sm.G1, 1.0, 0.0, work, st);        // P^T R
      small_chol_solve(r, sm.Delta, sm.G1, s, sm.alpha, s, s, 1.0, sm.flag, h.small.p, st);  // alpha
      ts_update<T>(nG, s, X.p, s, 1.0, 1.0, P, s, r, sm.alpha, s, nullptr, 0, 0, nullptr, 0, st);
      ts_update<T>(nG, s, R.p, s, 1.0, -1.0, Q, s, r, sm.alpha, s, nullptr, 0, 0, nullptr, 0, st);
      col_sumsq<T>(nG, s, R.p, s, sm.colsq, work, st);
      read_back(h, nr2.data(), sm.colsq, s);
      int fl = 0;
      read_back(h, &fl, sm.flag, 1);
      if (fl) fail(BREAKDOWN, "block CG: P^T S P is not positive definite");
      relres = max_rel(nr2);
      if (relres <= h.tol_inner) {
        converged = true;
        break;
      }
      op_gamma_solve<T>(h, R.p, s, Z.p, s, s);                            // Z = A_G^{-1} R
      gram<T, T>(nG, Q, s, r, Z.p, s, s, sm.G2, 1.0, 0.0, work, st);       // Q^T Z
      small_chol_apply(r, sm.Delta, sm.G2, s, sm.beta, s, s, -1.0, h.small.p, st);    // beta
      ts_update<T>(nG, s, Z.p, s, 1.0, 1.0, P, s, r, sm.beta, s, nullptr, 0, 0, nullptr, 0, st);  // Z + P beta
      r = orth<T>(h, sm, work, Z.p, P, Q, s);
    }
  }
  if constexpr (sizeof(T) == 8)
    NS_HIP(hipMemcpyAsync(D, X.p, nG * s * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    convert_block<float, double>(nG, s, X.p, s, D, s, st);
  NS_HIP(hipStreamSynchronize(st));
  return it;
}

// Nystrom core (Algorithm alg:prec1 steps 5-11): QR of Y by shifted
// Cholesky-QR (three passes), C = Omega^T Y, EVDs, U = Q W(:, 1:k'), Z = A_G^{-1} U.
void nystrom(Handle& h, SmallMats& sm, const double* Omega, double* Y) {
  hipStream_t st = h.stream;
  const int s = h.s, k = h.k;
  const int64_t nG = h.nG;
  DBuf<double> Qb, U, work;
  Qb.alloc(nG * s);
  work.alloc(gram_work_elems(s));
  gram<double, double>(nG, Omega, s, s, Y, s, s, sm.C, 1.0, 0.0, work, st);  // C = Omega^T Y
  const double u = std::ldexp(1.0, -53);
  const double coef = 11.0 * (double(nG) * s + double(s) * (s + 1)) * u;
  double* A = Y;
  double* B = Qb.p;
  for (int pass = 0; pass < 3; ++pass) {
    gram<double, double>(nG, A, s, s, A, s, s, sm.Gorth, 1.0, 0.0, work, st);
    small_cholqr(s, sm.Gorth, pass == 0 ? coef : 0.0, sm.Rinv, sm.Racc, pass == 0, sm.flag + 2, h.small.p, st);
    ts_update<double>(nG, s, B, s, 0.0, 1.0, A, s, s, sm.Rinv, s, nullptr, 0, 0, nullptr, 0, st);
    std::swap(A, B);
  }
  // A now holds Q (orthonormal), sm.Racc holds R
  small_nystrom(s, k, sm.C, sm.Racc, h.eig_rel, sm.Wk, sm.Ek, sm.rank, h.small.p, st);
  int out[2];
  read_back(h, out, sm.rank, 2);
  h.k_eff = out[1];
  h.Z.alloc(nG * (k > 0 ? k : 1));
  h.Sigma.alloc(k > 0 ? k : 1);
  if (h.k_eff == 0) return;
  U.alloc(nG * k);
  ts_update<double>(nG, h.k_eff, U.p, k, 0.0, 1.0, A, s, s, sm.Wk, k, nullptr, 0, 0, nullptr, 0, st);
  op_gamma_solve<double>(h, U.p, k, h.Z.p, k, h.k_eff);
  NS_HIP(hipMemcpyAsync(h.Sigma.p, sm.Ek, h.k_eff * sizeof(double), hipMemcpyDeviceToDevice, st));
  NS_HIP(hipStreamSynchronize(st));
}

// Adapted deflation: SZ = S Z, E = Z^T S Z, chol(E).
void setup_adef2(Handle& h) {
  hipStream_t st = h.stream;
  const int k = h.k, ke = h.k_eff;
  const int64_t nG = h.nG;
  if (ke == 0) return;
  h.SZ.alloc(nG * k);
  h.Echol.alloc(size_t(k) * k);
  op_schur<double>(h, h.Z.p, k, h.SZ.p, k, ke, false);
  DBuf<double> work;
  work.alloc(gram_work_elems(k));
  gram<double, double>(nG, h.Z.p, k, ke, h.SZ.p, k, ke, h.Echol.p, 1.0, 0.0, work, st);
  small_chol_solve(ke, h.Echol.p, nullptr, 0, nullptr, 0, 0, 1.0, h.dflags.p + 12, h.small.p, st);
  int fl = 0;
  read_back(h, &fl, h.dflags.p + 12, 1);
  if (fl) fail(BREAKDOWN, "Z^T S Z is not positive definite");
}

// z = M r for ncols vectors (FP64, interface order, row-major).
void apply_prec(Handle& h, const double* r, int64_t ldr, double* z, int64_t ldz, int ncols, double* work,
                double* c1, double* c2) {
  hipStream_t st = h.stream;
  const int64_t nG = h.nG;
  const int k = h.k, ke = h.k_eff;
  op_gamma_solve<double>(h, r, ldr, z, ldz, ncols);  // t = A_Gamma^{-1} r
  if (ke == 0) return;
  if (h.apply_mode == NS_APPLY_M2) {
    gram<double, double>(nG, h.Z.p, k, ke, r, ldr, ncols, c1, 1.0, 0.0, work, st);  // Z^T r
    small_rowscale(ke, ncols, h.Sigma.p, c1, ncols, st);
    ts_update<double>(nG, ncols, z, ldz, 1.0, 1.0, h.Z.p, k, ke, c1, ncols, nullptr, 0, 0, nullptr, 0, st);
  } else {
    gram<double, double>(nG, h.Z.p, k, ke, r, ldr, ncols, c1, 1.0, 0.0, work, st);   // Z^T r
    gram<double, double>(nG, h.SZ.p, k, ke, z, ldz, ncols, c1, -1.0, 1.0, work, st);  // - (SZ)^T t
    small_chol_apply(ke, h.Echol.p, c1, ncols, c2, ncols, ncols, 1.0, h.small.p, st);           // E^{-1} (...)
    ts_update<double>(nG, ncols, z, ldz, 1.0, 1.0, h.Z.p, k, ke, c2, ncols, nullptr, 0, 0, nullptr, 0, st);
  }
}

__global__ void k_finite_check(int64_t n, const double* __restrict__ x, int* flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  if (!(v == v) || v - v != 0.0) flag[0] = 1;
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) c[i] = a[i] - b[i];
}

ns_status finish(Handle* h, const Error& e) {
  g_last_error = e.msg;
  if (h) h->last_error = e.msg;
  return ns_status(e.status);
}

}  // namespace
}  // namespace ns

using namespace ns;

ns_handle_s::~ns_handle_s() {
  if (hflags) (void)hipHostFree(hflags);
  if (hscal) (void)hipHostFree(hscal);
}

extern "C" {

ns_status nystrom_schur_setup(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                              const double* val, const int32_t* part, const ns_options* opt, ns_handle* out,
                              ns_setup_info* info) {
  if (out) *out = nullptr;
  Handle* h = nullptr;
  try {
    if (!out || !opt) fail(INVALID_ARG, "out and opt must not be NULL");
    if (n <= 0 || nnz < n || !row_ptr || !col_idx || !val || !part)
      fail(INVALID_ARG, "need n > 0, nnz >= n and non-NULL CSR/part pointers");
    if (opt->k < 0 || opt->p < 0) fail(INVALID_ARG, "k and p must be >= 0");
    if (opt->k > 0 && !opt->omega) fail(INVALID_ARG, "omega (the sketch) is required when k > 0");
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->bad_block = info->bad_col = -1;
    }
    h = new Handle();
    h->stream = static_cast<hipStream_t>(opt->stream);
    h->k = opt->k;
    h->p = opt->p;
    h->s = opt->k + opt->p;
    h->tol_inner = opt->tol_inner > 0 ? opt->tol_inner : 0.1;
    h->eig_rel = opt->eig_thresh_rel > 0 ? opt->eig_thresh_rel : 1e-10;
    h->prec_inner = opt->prec_inner == NS_FP32 ? 1 : 0;
    h->drop_rel = opt->orth_drop_rel > 0 ? opt->orth_drop_rel : (h->prec_inner ? 1e-5 : 1e-6);
    h->max_inner = opt->max_inner_iters > 0 ? opt->max_inner_iters : 500;
    h->apply_mode = opt->apply_mode == NS_APPLY_ADEF2 ? 1 : 0;
    h->trsm_cols = opt->trsm_cols;
    h->schur_mode = opt->schur_mode;
    if (h->schur_mode < 0 || h->schur_mode > 2) fail(INVALID_ARG, "schur_mode must be 0, 1 or 2");
    if (h->trsm_cols != 0 && h->trsm_cols != 16 && h->trsm_cols != 32 && h->trsm_cols != 64)
      fail(INVALID_ARG, "trsm_cols must be 0, 16, 32 or 64");
    h->dflags.alloc(16);
    NS_HIP(hipMemset(h->dflags.p, 0, 16 * sizeof(int)));
    NS_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->hflags), 16 * sizeof(int), hipHostMallocDefault));
    NS_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->hscal), 64 * sizeof(double), hipHostMallocDefault));
    h->small.alloc(small_scratch_elems());
    Events ev(h->stream);
    ev.rec(0);
    extract_dbbd(*h, n, nnz, row_ptr, col_idx, val, part);
    if (h->s > h->nG) fail(INVALID_ARG, "k + p exceeds the interface size n_gamma");
    ev.rec(1);
    tile_cholesky(h->L1, h->dflags.p + 8, h->stream);
    check_chol(*h, 1, info);
    if (h->schur_mode != SCHUR_TRIANGULAR) local_schur_build(*h);
    tile_cholesky(h->L2, h->dflags.p + 8, h->stream);
    check_chol(*h, 2, info);
    assemble_junction(*h);
    tile_cholesky(h->LJ, h->dflags.p + 8, h->stream);
    check_chol(*h, 3, info);
    tile_make_transposed(h->L1, h->stream);
    for (ns::TileLevel* lv : {&h->L2, &h->LJ})
      if (lv->nblk && lv->max_nt * TILE <= 4096 && lv->nrows_pad * lv->max_nt * TILE <= (int64_t(1) << 28))
        tile_make_inverse(*lv, h->prec_inner != 0, h->stream);
    if (h->prec_inner) {
      if (!h->LS.built) tile_make_fp32(h->L1, h->stream);
      tile_make_fp32(h->L2, h->stream);
      tile_make_fp32(h->LJ, h->stream);
    }
    ev.rec(2);
    int it = 0;
    double relres = 0.0;
    bool conv = true;
    if (h->k > 0) {
      SmallMats sm;
      sm.init(h->s);
      DBuf<double> D;
      D.alloc(h->nG * h->s);
      if (h->prec_inner)
        it = block_pcg<float>(*h, sm, opt->omega, D.p, relres, conv);
      else
        it = block_pcg<double>(*h, sm, opt->omega, D.p, relres, conv);
      ev.rec(3);
      DBuf<double> Y;
      Y.alloc(h->nG * h->s);
      csr_mult<double>(h->AGG, D.p, h->s, Y.p, h->s, h->s, h->stream);  // Y = A_Gamma D
      nystrom(*h, sm, opt->omega, Y.p);
      if (h->apply_mode == NS_APPLY_ADEF2) setup_adef2(*h);
    } else {
      ev.rec(3);
    }
    ev.rec(4);
    NS_HIP(hipStreamSynchronize(h->stream));
    if (info) {
      info->n = h->n;
      info->n_interior = h->nI;
      info->n_gamma = h->nG;
      info->n_junction = h->nJ;
      info->n_sub = h->nsub;
      info->n_level2_blocks = h->nl2;
      info->k_eff = h->k_eff;
      info->it_inner = it;
      info->inner_converged = conv ? 1 : 0;
      info->inner_relres = relres;
      info->t_extract = ev.sec(0, 1);
      info->t_factor = ev.sec(1, 2);
      info->t_inner = ev.sec(2, 3);
      info->t_nystrom = ev.sec(3, 4);
      info->t_total = ev.sec(0, 4);
    }
    *out = h;
    return NS_OK;
  } catch (const Error& e) {
    ns_status st = finish(h, e);
    delete h;
    return st;
  }
}

ns_status nystrom_schur_apply(ns_handle h, const double* r_gamma, double* z_gamma, int32_t ncols) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    if (ncols < 1 || ncols > 1024 || !r_gamma || !z_gamma) fail(INVALID_ARG, "bad apply arguments");
    DBuf<double> work, c1, c2;
    work.alloc(gram_work_elems(std::max(h->k, ncols)));
    c1.alloc(size_t(std::max(h->k, 1)) * ncols);
    c2.alloc(size_t(std::max(h->k, 1)) * ncols);
    apply_prec(*h, r_gamma, ncols, z_gamma, ncols, ncols, work, c1, c2);
    NS_HIP(hipStreamSynchronize(h->stream));
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_pcg_solve(ns_handle h, const double* b, double* x, double rtol, int32_t maxit,
                                  ns_solve_info* info) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    if (!b || !x || maxit < 0 || !(rtol > 0.0)) fail(INVALID_ARG, "bad pcg_solve arguments");
    hipStream_t st = h->stream;
    const int64_t n = h->n, nG = h->nG, nIp = h->L1.nrows_pad;
    Events ev(st);
    ev.rec(0);
    NS_HIP(hipMemsetAsync(h->dflags.p + 14, 0, sizeof(int), st));
    k_finite_check<<<unsigned((n + 255) / 256), 256, 0, st>>>(n, b, h->dflags.p + 14);
    NS_LAUNCH_CHECK();
    int bad = 0;
    read_back(*h, &bad, h->dflags.p + 14, 1);
    if (bad) fail(INVALID_ARG, "b contains NaN or Inf");
    DBuf<double> bI, f, w, r, z, p, q, sc, work, c1, c2, tmp;
    bI.alloc(nIp);
    for (DBuf<double>* v : {&f, &w, &r, &z, &p, &q}) v->alloc(nG);
    sc.alloc(4 * (size_t(maxit) + 2));
    work.alloc(std::max<size_t>(gram_work_elems(std::max(h->k, 1)), 4096));
    c1.alloc(std::max(h->k, 1));
    c2.alloc(std::max(h->k, 1));
    tmp.alloc(n);
    // f = b_Gamma - A_GammaI A_I^{-1} b_I
    gather_rows<double>(nIp, h->iperm, b, 1, bI.p, 1, 1, st);
    tile_solve<double>(h->L1, bI.p, 1, 1, h->trsm_cols, st);
    {
      // f[g] = b[gperm[g]] - sum A_GI(g, :) bI
      DBuf<double> bG;
      bG.alloc(nG);
      gather_rows<double>(nG, h->gperm, b, 1, bG.p, 1, 1, st);
      csr_mult<double>(h->AGI, bI.p, 1, f.p, 1, 1, st);
      axpby(nG, 1.0, bG.p, -1.0, f.p, st);
      NS_HIP(hipStreamSynchronize(st));
    }
    dot(nG, f.p, f.p, sc.p + 3, work, st);
    double nf2 = 0.0;
    read_back(*h, &nf2, sc.p + 3, 1);
    const double nf = std::sqrt(nf2);
    NS_HIP(hipMemsetAsync(w.p, 0, nG * sizeof(double), st));
    NS_HIP(hipMemcpyAsync(r.p, f.p, nG * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (h->apply_mode == NS_APPLY_ADEF2 && h->k_eff > 0 && nf > 0.0) {
      // w0 = Z E^{-1} Z^T f ; r = f - S w0
      const int k = h->k, ke = h->k_eff;
      gram<double, double>(nG, h->Z.p, k, ke, f.p, 1, 1, c1.p, 1.0, 0.0, work, st);
      small_chol_apply(ke, h->Echol.p, c1.p, 1, c2.p, 1, 1, 1.0, h->small.p, st);
      ts_update<double>(nG, 1, w.p, 1, 0.0, 1.0, h->Z.p, k, ke, c2.p, 1, nullptr, 0, 0, nullptr, 0, st);
      op_schur<double>(*h, w.p, 1, q.p, 1, 1, false);
      axpby(nG, 1.0, f.p, -1.0, q.p, st);
      NS_HIP(hipMemcpyAsync(r.p, q.p, nG * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    int it = 0;
    bool conv = false;
    double rel = 0.0;
    std::vector<double> hist;
    if (nf == 0.0) {
      conv = true;
      hist.push_back(0.0);
    } else {
      dot(nG, r.p, r.p, sc.p + 2, work, st);
      double rn2 = 0.0;
      read_back(*h, &rn2, sc.p + 2, 1);
      rel = std::sqrt(rn2) / nf;
      hist.push_back(rel);
      conv = rel <= rtol;
      if (!conv) {
        apply_prec(*h, r.p, 1, z.p, 1, 1, work, c1, c2);
        dot(nG, r.p, z.p, sc.p + 0, work, st);
        NS_HIP(hipMemcpyAsync(p.p, z.p, nG * sizeof(double), hipMemcpyDeviceToDevice, st));
        for (int j = 0; j < maxit; ++j) {
          op_schur<double>(*h, p.p, 1, q.p, 1, 1, false);                 // q = S p
          dot(nG, p.p, q.p, sc.p + 4 * j + 1, work, st);                 // p^T q
          pcg_update_wr(nG, sc.p, j, w.p, r.p, p.p, q.p, sc.p + 4 * j + 2, work, st);
          read_back(*h, h->hscal, sc.p + 4 * j + 2, 1);
          rel = std::sqrt(h->hscal[0]) / nf;
          hist.push_back(rel);
          it = j + 1;
          if (!(rel > rtol)) {
            conv = rel <= rtol;
            break;
          }
          apply_prec(*h, r.p, 1, z.p, 1, 1, work, c1, c2);              // z = M r
          dot(nG, r.p, z.p, sc.p + 4 * (j + 1), work, st);               // rho_{j+1}
          pcg_update_p(nG, sc.p, j, z.p, p.p, st);
        }
      }
    }
    // back-substitution: x_I = A_I^{-1} (b_I - A_IGamma w), x_Gamma = w
    {
      DBuf<double> rhs;
      rhs.alloc(nIp);
      gather_rows<double>(nIp, h->iperm, b, 1, rhs.p, 1, 1, st);
      csr_mult<double>(h->AIG, w.p, 1, bI.p, 1, 1, st);
      axpby(nIp, 1.0, rhs.p, -1.0, bI.p, st);
      tile_solve<double>(h->L1, bI.p, 1, 1, h->trsm_cols, st);
      scatter_rows<double, double>(nIp, h->iperm, bI.p, 1, x, 1, 1, st);
      scatter_rows<double, double>(nG, h->gperm, w.p, 1, x, 1, 1, st);
      // true residual ||b - A x|| / ||b||
      csr_mult<double>(h->Aorig, x, 1, tmp.p, 1, 1, st);
      k_sub<<<unsigned((n + 255) / 256), 256, 0, st>>>(n, b, tmp.p, tmp.p);
      NS_LAUNCH_CHECK();
      dot(n, tmp.p, tmp.p, sc.p + 1, work, st);
      dot(n, b, b, sc.p + 2, work, st);
      double rr[2];
      read_back(*h, rr, sc.p + 1, 2);
      ev.rec(1);
      if (info) {
        info->it_pcg = it;
        info->converged = conv ? 1 : 0;
        info->relres_schur = rel;
        info->relres_true = rr[1] > 0 ? std::sqrt(rr[0] / rr[1]) : 0.0;
        info->t_solve = ev.sec(0, 1);
        if (info->res_hist && info->res_hist_cap > 0) {
          const size_t m = std::min<size_t>(hist.size(), size_t(info->res_hist_cap));
          std::memcpy(info->res_hist, hist.data(), m * sizeof(double));
        }
      }
    }
    if (!conv) fail(NOT_CONVERGED, "PCG did not reach rtol within maxit iterations");
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_schur_apply(ns_handle h, const double* X, double* Y, int32_t ncols, int32_t prec) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    if (ncols < 1 || ncols > 1024 || !X || !Y) fail(INVALID_ARG, "bad arguments");
    if (prec == NS_FP32) {
      if (!h->prec_inner) fail(INVALID_ARG, "FP32 operators exist only with prec_inner = NS_FP32");
      DBuf<float> x32, y32;
      x32.alloc(h->nG * ncols);
      y32.alloc(h->nG * ncols);
      convert_block<double, float>(h->nG, ncols, X, ncols, x32.p, ncols, h->stream);
      op_schur<float>(*h, x32.p, ncols, y32.p, ncols, ncols, false);
      convert_block<float, double>(h->nG, ncols, y32.p, ncols, Y, ncols, h->stream);
      NS_HIP(hipStreamSynchronize(h->stream));
    } else {
      op_schur<double>(*h, X, ncols, Y, ncols, ncols, false);
      NS_HIP(hipStreamSynchronize(h->stream));
    }
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_interface_solve(ns_handle h, const double* X, double* Y, int32_t ncols, int32_t prec) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    if (ncols < 1 || ncols > 1024 || !X || !Y) fail(INVALID_ARG, "bad arguments");
    if (prec == NS_FP32) {
      if (!h->prec_inner) fail(INVALID_ARG, "FP32 operators exist only with prec_inner = NS_FP32");
      DBuf<float> x32, y32;
      x32.alloc(h->nG * ncols);
      y32.alloc(h->nG * ncols);
      convert_block<double, float>(h->nG, ncols, X, ncols, x32.p, ncols, h->stream);
      op_gamma_solve<float>(*h, x32.p, ncols, y32.p, ncols, ncols);
      convert_block<float, double>(h->nG, ncols, y32.p, ncols, Y, ncols, h->stream);
    } else {
      op_gamma_solve<double>(*h, X, ncols, Y, ncols, ncols);
    }
    NS_HIP(hipStreamSynchronize(h->stream));
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_interior_solve(ns_handle h, const double* X, double* Y, int32_t ncols, int32_t prec) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    if (ncols < 1 || ncols > 1024 || !X || !Y) fail(INVALID_ARG, "bad arguments");
    if (prec == NS_FP32) {
      if (!h->prec_inner) fail(INVALID_ARG, "FP32 operators exist only with prec_inner = NS_FP32");
      DBuf<float> x32, y32;
      x32.alloc(h->nI * ncols);
      y32.alloc(h->nI * ncols);
      convert_block<double, float>(h->nI, ncols, X, ncols, x32.p, ncols, h->stream);
      op_interior_solve<float>(*h, x32.p, y32.p, ncols);
      convert_block<float, double>(h->nI, ncols, y32.p, ncols, Y, ncols, h->stream);
    } else {
      op_interior_solve<double>(*h, X, Y, ncols);
    }
    NS_HIP(hipStreamSynchronize(h->stream));
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_export_factor(ns_handle h, int32_t block, double* L) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    if (block < 0 || block >= h->nsub || !L) fail(INVALID_ARG, "bad block index");
    tile_export(h->L1, block, L, h->stream);
    NS_HIP(hipStreamSynchronize(h->stream));
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_get_sizes(ns_handle h, int64_t* out) {
  if (!h || !out) return finish(h, Error{INVALID_ARG, "NULL argument"});
  out[0] = h->n;
  out[1] = h->nI;
  out[2] = h->nG;
  out[3] = h->nsub;
  out[4] = h->nJ;
  out[5] = h->nl2;
  out[6] = h->k_eff;
  out[7] = h->nsub ? h->L1.h_nb[0] : 0;
  return NS_OK;
}

ns_status nystrom_schur_get_lowrank(ns_handle h, double* Z, double* Sigma) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    if (h->k_eff > 0) {
      if (Z)
        NS_HIP(hipMemcpy2DAsync(Z, h->k_eff * sizeof(double), h->Z.p, h->k * sizeof(double),
                                h->k_eff * sizeof(double), h->nG, hipMemcpyDeviceToDevice, h->stream));
      if (Sigma)
        NS_HIP(hipMemcpyAsync(Sigma, h->Sigma.p, h->k_eff * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
      NS_HIP(hipStreamSynchronize(h->stream));
    }
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

void nystrom_schur_destroy(ns_handle h) { delete h; }

const char* nystrom_schur_last_error(ns_handle h) {
  if (h) return h->last_error.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
