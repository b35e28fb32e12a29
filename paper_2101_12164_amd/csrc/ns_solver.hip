// Host orchestration and the C ABI: Algorithm alg:prec1 (setup), the
// preconditioner application (eq. left_prec_mat or the adapted deflation form)
// and the block LDL^T solve with PCG on the Schur complement (eqs. A_LDLT,
// Sx=b).  Every numerical step runs in the library's HIP kernels; the host only
// sequences launches and reads back convergence scalars.
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

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

// Small FP64 matrices of one setup, stacked per problem (s x s each unless noted).
struct SmallMats {
  DBuf<double> buf;
  double *Delta, *G1, *alpha, *G2, *beta, *Gorth, *Torth, *Rinv, *Racc, *C;
  double *Wk, *Ek, *colsq, *nF2, *coef, *relres;  // Wk s x k, Ek k, colsq / nF2 s, coef / relres 1
  DBuf<int> ibuf;
  int* flag;   // [4] breakdown / factorisation flags
  int* ctr;    // [4] ctr[0]: problems no longer active in the inner solve
  int *active, *rank, *ok, *skip, *svr, *dimA, *itp, *conv, *single, *dimB, *skip2, *dimC, *nys;  // (nys: 2)
  int np = 0;
  void init(int nprob, int s, int k) {
    np = nprob;
    const size_t m = size_t(s) * s * np;
    buf.alloc(10 * m + size_t(s) * std::max(k, 1) * np + size_t(std::max(k, 1)) * np + 2 * size_t(s) * np + 2 * np);
    double* p = buf.p;
    for (double** q : {&Delta, &G1, &alpha, &G2, &beta, &Gorth, &Torth, &Rinv, &Racc, &C}) {
      *q = p;
      p += m;
    }
    Wk = p;
    p += size_t(s) * std::max(k, 1) * np;
    Ek = p;
    p += size_t(std::max(k, 1)) * np;
    colsq = p;
    p += size_t(s) * np;
    nF2 = p;
    p += size_t(s) * np;
    coef = p;
    p += np;
    relres = p;
    ibuf.alloc(8 + 14 * size_t(np));
    NS_HIP(hipMemsetAsync(ibuf.p, 0, ibuf.n * sizeof(int), alloc_stream()));
    flag = ibuf.p;
    ctr = ibuf.p + 4;
    int* q = ibuf.p + 8;
    for (int** d : {&active, &rank, &ok, &skip, &svr, &dimA, &itp, &conv, &single, &dimB, &skip2, &dimC}) {
      *d = q;
      q += np;
    }
    nys = q;
  }
};

// An event without timing, destroyed with its owner.
struct Event {
  hipEvent_t e = nullptr;
  Event() { NS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
  ~Event() {
    if (e) (void)hipEventDestroy(e);
  }
  Event(const Event&) = delete;
  Event& operator=(const Event&) = delete;
};

// Issues the handle's work on another stream (allocations included) until the end of the scope.
struct StreamSwap {
  Handle& h;
  hipStream_t prev;
  StreamScope ss;
  StreamSwap(Handle& hh, hipStream_t s) : h(hh), prev(hh.stream), ss(s) { h.stream = s; }
  ~StreamSwap() { h.stream = prev; }
  StreamSwap(const StreamSwap&) = delete;
  StreamSwap& operator=(const StreamSwap&) = delete;
};

template <class T>
void read_back(Handle& h, T* host, const T* dev, size_t count) {
  NS_HIP(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, h.stream));
  NS_HIP(hipStreamSynchronize(h.stream));
  stream_idle(h.stream);
}

// Pivot flags of the three factorisation levels (subdomains, interface blocks, junction), read once after
// all of them: a failed level only leaves meaningless values in the later ones, whose launches do not depend
// on them, and the first failing level is reported.
constexpr int CHOL_FLAGS = 16;  // dflags[16 + 3 (level - 1) ..]: (flag, block, column)
void check_chol(Handle& h, ns_setup_info* info) {
  int e[9];
  read_back(h, e, h.dflags.p + CHOL_FLAGS, 9);
  for (int level = 1; level <= 3; ++level) {
    const int* f = e + 3 * (level - 1);
    if (!f[0]) continue;
    int blk = f[1];
    if (level == 2) blk = -2 - blk;
    if (level == 3) blk = -1;
    if (info) {
      info->bad_block = blk;
      info->bad_col = f[2];
    }
    fail(NOT_SPD, "Cholesky pivot <= 0 in block " + std::to_string(blk) + ", column " + std::to_string(f[2]));
  }
}

// ------------------------------------------------------------------ inner-solve control (per problem)
// Stopping test of block CG: rel_p = max_j ||R_p(:, j)|| / ||F_p(:, j)||; an active problem with
// rel_p <= tol stops (converged) at iteration it.
__global__ void k_iter(int* it) { *it += 1; }

// it: the iteration index, or, with itd != nullptr, read from the device (graph-replayed iterations)
// One wave per problem: the largest relative column residual sqrt(colsq / nF2) over the s columns, lanes over
// columns (four per lane in flight together, from clamped positions), a butterfly for the maximum.
// A problem that converges here also gets dims[p] = 0 (the dimension the small solves take, active ? rank : 0).
__global__ __launch_bounds__(64) void k_bcg_check(int np, int s, const double* __restrict__ colsq,
                                                  const double* __restrict__ nF2, double tol, int it, int* active,
                                                  int* itp, int* conv, double* relres, int* ndone, const int* itd,
                                                  int* dims) {
  const int p = blockIdx.x, lane = threadIdx.x;
  if (p >= np || !active[p]) return;  // uniform over the wave
  if (itd) it = *itd;
  double m = 0.0;
  for (int j0 = 0; j0 < s; j0 += 4 * 64) {
    double f[4], c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = min(j0 + 64 * k + lane, s - 1);
      f[k] = nF2[int64_t(p) * s + j];
      c[k] = colsq[int64_t(p) * s + j];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (j0 + 64 * k + lane < s && f[k] > 0.0) m = fmax(m, sqrt(c[k] / f[k]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane == 0) {
    relres[p] = m;
    itp[p] = it;
    if (m <= tol) {
      conv[p] = 1;
      active[p] = 0;
      dims[p] = 0;
      atomicAdd(ndone, 1);
    }
  }
}

// dims[p] = active[p] ? (rank ? rank[p] : s) : 0; skip[p] for the eigen-decomposition fallback
__global__ void k_dims(int np, int s, const int* active, const int* rank, int* dims) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) dims[p] = active[p] ? (rank ? rank[p] : s) : 0;
}
// dims of the second Cholesky-QR pass: 0 where the first pass was certified to suffice
__global__ void k_dims2(int np, const int* rank, const int* single, int* dims) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) dims[p] = single[p] ? 0 : rank[p];
}
// The second Cholesky-QR pass measured before it runs: skip2[p] = 1 where it has nothing to do (dims 0) or where
// the Gram matrix G of the first pass's basis is already within eta of the identity in the Frobenius norm over
// its leading dims x dims block (the basis then has condition number at most sqrt((1 + eta) / (1 - eta)));
// dimC[p] = skip2[p] ? 0 : dims[p].  One workgroup per problem.
__global__ __launch_bounds__(1024) void k_near_identity(int np, int s, const int* dims, const double* G, int64_t sG,
                                                        double eta, int* skip2, int* dimC) {
  __shared__ double red[16];
  const int p = blockIdx.x;
  const int n = dims[p];
  const double* Gp = G + int64_t(p) * sG;
  double e2 = 0.0;
  for (int e0 = threadIdx.x; e0 < n * n; e0 += 4 * 1024) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(e0 + 1024 * u, n * n - 1), i = e / n, j = e - i * n;
      v[u] = Gp[int64_t(i) * s + j] - (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + 1024 * u < n * n) e2 += v[u] * v[u];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double f2 = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) f2 += red[w];
    const int sk = (n == 0 || f2 <= eta * eta) ? 1 : 0;
    skip2[p] = sk;
    dimC[p] = sk ? 0 : n;
  }
}

__global__ void k_svqb_mask(int np, const int* active, const int* ok, int* skip) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < np) skip[p] = !(active[p] && !ok[p]);
}
// Transform per problem: the Cholesky-QR inverse when certified, else the eigen-decomposition based one
// (copied into Rinv); rank: s, the number of directions kept, or 0 when inactive.  An active problem
// left without directions stops (not converged).  dims[p] = active ? rank : 0 afterwards (the dimension of the
// next small solves).
__global__ void k_orth_select(int np, int s, int* active, const int* ok, const int* svr, const double* Torth,
                              double* Rinv, int* rank, int it, int* itp, int* ndone, const int* itd, int* dims) {
  const int p = blockIdx.x;
  if (itd) it = *itd;
  const bool use_svqb = active[p] && !ok[p];
  if (use_svqb)
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) Rinv[int64_t(p) * s * s + e] = Torth[int64_t(p) * s * s + e];
  if (threadIdx.x == 0) {
    const int r = !active[p] ? 0 : (ok[p] ? s : svr[p]);
    rank[p] = r;
    if (active[p] && r == 0) {
      active[p] = 0;
      itp[p] = it;
      atomicAdd(ndone, 1);
    }
    dims[p] = active[p] ? r : 0;
  }
}

// Orthonormal basis of the columns of every active problem's block of V (n_G x s, ld s) into P, dropping
// directions with singular value <= drop * sigma_max.  When a Cholesky of the Gram matrix certifies
// that every singular value ratio exceeds the drop tolerance, nothing is dropped and Cholesky-QR2
// yields a basis of the same span; otherwise the Gram matrix is eigen-decomposed (SVQB: keep the
// eigenpairs above drop^2 * lambda_max) followed by one Cholesky-QR pass.  The second pass runs in place,
// and only where the first pass's basis B is measurably short of orthonormal: ||B^T B - I||_F > ORTH_ETA (a
// basis within ORTH_ETA has condition number below 1 + ORTH_ETA, and the block CG's recurrences only need a
// well-conditioned basis of the span).  Inactive problems get zero columns; dropped directions are zero
// columns at the end.  P and Q trade places (the old P is scratch).
constexpr double ORTH_ETA = 1e-4;
template <class T>
void orth(Handle& h, const Seg& sg, SmallMats& sm, double* work, const T* V, T*& P, T*& Q, int s, int it,
          const int* itd = nullptr) {
  hipStream_t st = h.stream;
  const int np = h.nprob;
  const int64_t ss = int64_t(s) * s;
  const double drop2 = h.drop_rel * h.drop_rel;
  const int pb = (np + 255) / 256;
  gram<T, T>(sg, V, s, s, V, s, s, sm.Gorth, ss, 1.0, 0.0, work, st);
  k_dims<<<pb, 256, 0, st>>>(np, s, sm.active, nullptr, sm.dimA);
  NS_LAUNCH_CHECK();
  // FP64 blocks: when the bounds certify that the column-equilibrated Gram matrix has a condition number below
  // 1e6, the first pass already leaves an orthonormality error of order 1e6 times its rounding (1e-9 or less),
  // and the second pass is passed over on the device (its block update becomes a copy, so the result lands
  // where the graph expects it); FP32 blocks always take both passes
  int* single = sizeof(T) == 8 ? sm.single : nullptr;
  small_cholqr(Batch{np, sm.dimA}, s, sm.Gorth, ss, nullptr, sm.Rinv, sm.Racc, 1, sm.flag + 1, h.sws, st, drop2,
               sm.ok, 1e-6, single);
  k_svqb_mask<<<pb, 256, 0, st>>>(np, sm.active, sm.ok, sm.skip);
  NS_LAUNCH_CHECK();
  small_svqb(np, s, sm.Gorth, ss, drop2, sm.Torth, ss, sm.svr, sm.skip, h.sws, st);
  k_orth_select<<<np, 256, 0, st>>>(np, s, sm.active, sm.ok, sm.svr, sm.Torth, sm.Rinv, sm.rank, it, sm.itp,
                                    sm.ctr, itd, sm.dimA);
  NS_LAUNCH_CHECK();
  ts_update<T>(sg, s, Q, s, 0.0, 1.0, V, s, s, sm.Rinv, s, ss, nullptr, 0, 0, nullptr, 0, 0, st);
  Seg sg2 = sg;
  const int* dims2 = sm.rank;
  if (single) {
    sg2.skip = single;
    k_dims2<<<pb, 256, 0, st>>>(np, sm.rank, single, sm.dimB);
    NS_LAUNCH_CHECK();
    dims2 = sm.dimB;
  }
  gram<T, T>(sg2, Q, s, s, Q, s, s, sm.Gorth, ss, 1.0, 0.0, work, st);
  k_near_identity<<<np, 1024, 0, st>>>(np, s, dims2, sm.Gorth, ss, ORTH_ETA, sm.skip2, sm.dimC);
  NS_LAUNCH_CHECK();
  sg2.skip = sm.skip2;
  small_cholqr(Batch{np, sm.dimC}, s, sm.Gorth, ss, nullptr, sm.Rinv, sm.Racc, 1, sm.flag + 1, h.sws, st);
  ts_update<T>(sg2, s, Q, s, 0.0, 1.0, Q, s, s, sm.Rinv, s, ss, nullptr, 0, 0, nullptr, 0, 0, st);  // in place
  std::swap(P, Q);
}

// Breakdown-free block PCG on S_Gamma D = F, preconditioned by A_Gamma^{-1}, from D = 0 (the inner solve of
// Algorithm alg:prec1, steps 2-4, in the shifted Schur form: with F = W Omega, A_Gamma D = A_GammaI S_I^{-1}
// A_IGamma Omega by eq. S-1), for every problem of the batch at once.  rhs(T* R) writes F into R.  Writes D
// (FP64, n_G x s) and adds the per-problem iteration counts to h.it_inner (convergence and final column-max
// relative residuals are those of this solve).
// The operators of the shifted form: rows = interface rows, S = S_Gamma, preconditioner A_Gamma^{-1}.
template <class T>
struct SchurOps {
  Handle& h;
  const Seg& seg() const { return h.segG.view; }
  int64_t rows() const { return h.nG; }
  void S(const T* P, T* Q) { op_schur<T>(h, P, h.s, Q, h.s, h.s, false); }
  void M(const T* R, T* Z) { op_gamma_solve<T>(h, R, h.s, Z, h.s, h.s); }
};

template <class T, class Ops, class Rhs>
void block_pcg(Handle& h, SmallMats& sm, Ops& ops, Rhs rhs, double* D) {
  hipStream_t st = h.stream;
  const Seg& sg = ops.seg();
  const int s = h.s, np = h.nprob;
  const int64_t nG = ops.rows(), ss = int64_t(s) * s;
  DBuf<T> X, R, Pb, Qb, Z;
  for (DBuf<T>* b : {&X, &R, &Pb, &Qb, &Z}) b->alloc(nG * s);
  DBuf<double> work;
  work.alloc(gram_work_elems(sg, s));
  T* P = Pb.p;
  T* Q = Qb.p;
  std::vector<int> ones(np, 1);
  upload(sm.active, ones.data(), np * sizeof(int), st);
  NS_HIP(hipMemsetAsync(sm.conv, 0, np * sizeof(int), st));
  NS_HIP(hipMemsetAsync(sm.ctr, 0, 4 * sizeof(int), st));
  rhs(R.p);  // F (n_G x s, precision T)
  NS_HIP(hipMemsetAsync(X.p, 0, nG * s * sizeof(T), st));
  col_sumsq<T>(sg, s, R.p, s, sm.nF2, work, st);
  NS_HIP(hipMemcpyAsync(sm.colsq, sm.nF2, size_t(np) * s * sizeof(double), hipMemcpyDeviceToDevice, st));
  k_bcg_check<<<np, 64, 0, st>>>(np, s, sm.colsq, sm.nF2, h.tol_inner, 0, sm.active, sm.itp, sm.conv, sm.relres,
                                  sm.ctr, nullptr, sm.dimA);
  NS_LAUNCH_CHECK();
  int hc[2] = {0, 0};
  read_back(h, hc, sm.ctr, 1);
  if (hc[0] < np) {
    // the iteration index lives on the device, so that the same launches, recorded once into a HIP graph, serve
    // every iteration: k_iter advances it, the stopping test and the orthonormalisation read it
    DBuf<int> itd;
    itd.alloc(1);
    NS_HIP(hipMemsetAsync(itd.p, 0, sizeof(int), st));
    // first half: Q = S P, alpha, X and R, the stopping test; second half: Z = M R, beta, P = orth(Z + P beta)
    auto half1 = [&](hipStream_t q) {
      k_iter<<<1, 1, 0, q>>>(itd.p);
      ops.S(P, Q);                                                            // Q = S P
      gram<T, T>(sg, P, s, s, Q, s, s, sm.Delta, ss, 1.0, 0.0, work, q, nullptr, 0, true);  // Delta = P^T S P
      gram<T, T>(sg, P, s, s, R.p, s, s, sm.G1, ss, 1.0, 0.0, work, q);       // P^T R
      // sm.dimA = active ? rank : 0, kept by the orthonormalisation's selection and the stopping test
      small_chol_solve(Batch{np, sm.dimA}, s, sm.Delta, ss, sm.G1, s, ss, sm.alpha, s, ss, s, s, 1.0, sm.flag,
                       h.sws, q);  // alpha
      ts_update<T>(sg, s, X.p, s, 1.0, 1.0, P, s, s, sm.alpha, s, ss, nullptr, 0, 0, nullptr, 0, 0, q);
      ts_update<T>(sg, s, R.p, s, 1.0, -1.0, Q, s, s, sm.alpha, s, ss, nullptr, 0, 0, nullptr, 0, 0, q);
      col_sumsq<T>(sg, s, R.p, s, sm.colsq, work, q);
      k_bcg_check<<<np, 64, 0, q>>>(np, s, sm.colsq, sm.nF2, h.tol_inner, 0, sm.active, sm.itp, sm.conv,
                                     sm.relres, sm.ctr, itd.p, sm.dimA);
      NS_LAUNCH_CHECK();
    };
    auto half2 = [&](hipStream_t q) {
      ops.M(R.p, Z.p);                                                        // Z = M R
      gram<T, T>(sg, Q, s, s, Z.p, s, s, sm.G2, ss, 1.0, 0.0, work, q);       // Q^T Z
      small_chol_apply(Batch{np, sm.dimA}, s, sm.Delta, ss, sm.G2, s, ss, sm.beta, s, ss, s, s, -1.0, h.sws,
                       q);  // beta
      ts_update<T>(sg, s, Z.p, s, 1.0, 1.0, P, s, s, sm.beta, s, ss, nullptr, 0, 0, nullptr, 0, 0, q);  // Z + P beta
      orth<T>(h, sg, sm, work, Z.p, P, Q, s, 0, itd.p);
    };
    auto done = [&]() {  // breakdown flag and problems finished, from the device
      NS_HIP(hipMemcpyAsync(hc + 1, sm.flag, sizeof(int), hipMemcpyDeviceToHost, st));
      read_back(h, hc, sm.ctr, 1);
      if (hc[1]) fail(BREAKDOWN, "block CG: P^T S P is not positive definite");
      return hc[0] >= np;
    };
    ops.M(R.p, Z.p);
    orth<T>(h, sg, sm, work, Z.p, P, Q, s, 0, itd.p);
    int it = 1;
    half1(st);  // the first iteration runs with plain launches: it also sizes every workspace the body uses
    bool fin = done();
    if (!fin && it < h.max_inner) half2(st);
    // m iterations per graph (an even count, so that the two search-direction buffers P and Q, which swap
    // roles every iteration, are where the recording found them at every replay); iterations a replay runs
    // after every problem has finished change nothing (finished problems are frozen)
    const int mb = h.bcg_graph == 0 ? tuned("bcg_graph_iters", h.bf16 ? "bf16" : (sizeof(T) == 8 ? "f64" : "f32"),
                                            nG, 2)
                                    : h.bcg_graph;
    const int m = mb <= 0 || kernel_timing_in_loops(false) ? 0 : 2 * ((mb + 1) / 2);
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    if (!fin && m > 0 && it + m <= h.max_inner) {
      NS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipGraph_t graph = nullptr;
      h.stream = cap;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          for (int t = 0; t < m; ++t) {
            half1(cap);
            half2(cap);
          }
        } catch (...) {
          (void)hipStreamEndCapture(cap, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          h.stream = st;
          (void)hipStreamDestroy(cap);
          throw;
        }
        e = hipStreamEndCapture(cap, &graph);
      }
      h.stream = st;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(cap);
        fail(HIP, std::string("block-CG graph capture failed: ") + hipGetErrorString(e));
      }
      while (!fin && it + m <= h.max_inner) {
        NS_HIP(hipGraphLaunch(exec, st));
        it += m;
        fin = done();
      }
    }
    while (!fin && it < h.max_inner) {  // plain launches (no graph, or the last iterations before the cap)
      ++it;
      half1(st);
      fin = done();
      if (!fin && it < h.max_inner) half2(st);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cap) (void)hipStreamDestroy(cap);
  }
  if constexpr (sizeof(T) == 8)
    NS_HIP(hipMemcpyAsync(D, X.p, nG * s * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    convert_block<float, double>(nG, s, X.p, s, D, s, st);
  std::vector<int> its(np), conv(np);
  h.relres_inner.resize(np);
  NS_HIP(hipMemcpyAsync(its.data(), sm.itp, np * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(conv.data(), sm.conv, np * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(h.relres_inner.data(), sm.relres, np * sizeof(double), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  h.it_inner.resize(np, 0);
  h.conv_inner.resize(np, 1);
  for (int q = 0; q < np; ++q) {
    h.it_inner[q] += its[q];
    h.conv_inner[q] = h.conv_inner[q] && conv[q];
  }
}

// While alive, FP32 operator applications of the handle use the BF16 operand copies (NS_BF16).
struct BF16Scope {
  Handle& h;
  int prev;
  explicit BF16Scope(Handle& hh, bool on = true) : h(hh), prev(hh.op_bf16) { h.op_bf16 = on && h.bf16; }
  ~BF16Scope() { h.op_bf16 = prev; }
};

// Three Cholesky-QR passes per problem over the rows of sg: X (rows x s) <- X R^{-1} with R^T R = X^T M X,
// where MX holds M X for an SPD M (MX == nullptr: M = I, the QR of X); MX is updated alongside.  The first
// pass is shifted by 11 (m s + s (s + 1)) u (m the problem's rows, u = 2^-53).  On return X (and MX) point at
// the orthonormalised blocks (one of the two given buffers each) and sm.Racc holds R.
void chol_qr3(Handle& h, SmallMats& sm, const Seg& sg, const std::vector<int64_t>& prow, int s, double*& X,
              double*& Xs, double*& MX, double*& MXs, double* work) {
  hipStream_t st = h.stream;
  const int np = h.nprob;
  const int64_t ss = int64_t(s) * s;
  {
    const double u = std::ldexp(1.0, -53);
    std::vector<double> coef(np);
    for (int q = 0; q < np; ++q) coef[q] = 11.0 * (double(prow[q]) * s + double(s) * (s + 1)) * u;
    upload(sm.coef, coef.data(), np * sizeof(double), st);
  }
  for (int pass = 0; pass < 3; ++pass) {
    gram<double, double>(sg, X, s, s, MX ? MX : X, s, s, sm.Gorth, ss, 1.0, 0.0, work, st);
    small_cholqr(Batch{np, nullptr}, s, sm.Gorth, ss, pass == 0 ? sm.coef : nullptr, sm.Rinv, sm.Racc, pass == 0,
                 sm.flag + 2, h.sws, st);
    ts_update<double>(sg, s, Xs, s, 0.0, 1.0, X, s, s, sm.Rinv, s, ss, nullptr, 0, 0, nullptr, 0, 0, st);
    std::swap(X, Xs);
    if (MX) {
      ts_update<double>(sg, s, MXs, s, 0.0, 1.0, MX, s, s, sm.Rinv, s, ss, nullptr, 0, 0, nullptr, 0, 0, st);
      std::swap(MX, MXs);
    }
  }
}

// Nystrom core (Algorithm alg:nystrom steps 3-8, Algorithm alg:prec1 steps 5-10) per problem on the rows of sg:
// C = G^T BG with G the sketch and BG = B G; an orthonormal basis Q of the sketched range with BG = Q R (the
// QR of BG; with D given, BG = A_Gamma D and the basis is D orthonormalised in the A_Gamma inner product, which
// is R_Gamma^{-1} times the QR basis of R_Gamma D: the variant M_1); EVDs of C and T; out = Q W(:, 1:k')
// (rows x k).  Sets k_eff and Sigma; BG and D are overwritten.
void nystrom_factor(Handle& h, SmallMats& sm, const Seg& sg, const std::vector<int64_t>& prow, int64_t rows,
                    const double* G, double* BG, double* D, double* out) {
  hipStream_t st = h.stream;
  const int s = h.s, k = h.k, np = h.nprob;
  const int64_t ss = int64_t(s) * s;
  DBuf<double> s1, s2, work;
  s1.alloc(rows * s);
  work.alloc(gram_work_elems(sg, s));
  gram<double, double>(sg, G, s, s, BG, s, s, sm.C, ss, 1.0, 0.0, work, st);  // C = G^T B G
  double* X = D ? D : BG;
  double* Xs = s1.p;
  double* MX = D ? BG : nullptr;
  double* MXs = nullptr;
  if (D) {
    s2.alloc(rows * s);
    MXs = s2.p;
  }
  chol_qr3(h, sm, sg, prow, s, X, Xs, MX, MXs, work);
  small_nystrom(np, s, k, sm.C, sm.Racc, h.eig_rel, sm.Wk, sm.Ek, sm.nys, h.sws, st);
  std::vector<int> o(2 * np);
  read_back(h, o.data(), sm.nys, 2 * np);
  h.h_keff.resize(np);
  h.k_eff = 0;
  for (int q = 0; q < np; ++q) {
    h.h_keff[q] = o[2 * q + 1];
    h.k_eff = std::max(h.k_eff, h.h_keff[q]);
  }
  h.keff_d.alloc(np);
  upload(h.keff_d.p, h.h_keff.data(), np * sizeof(int), st);
  h.Sigma.alloc(size_t(k > 0 ? k : 1) * np);
  NS_HIP(hipMemcpyAsync(h.Sigma.p, sm.Ek, size_t(k) * np * sizeof(double), hipMemcpyDeviceToDevice, st));
  NS_HIP(hipMemsetAsync(out, 0, rows * k * sizeof(double), st));
  if (h.k_eff > 0)
    ts_update<double>(sg, k, out, k, 0.0, 1.0, X, s, s, sm.Wk, k, int64_t(s) * k, nullptr, 0, 0, nullptr, 0, 0, st);
}

// R_Gamma^{-1} X (FP64, n_G x ncols, interface order) for A_Gamma = R_Gamma^T R_Gamma, R_Gamma = L^T P with L the
// Cholesky factor of A_Gamma in the order of the interface split: [A_s A_sJ; A_Js A_J] = L L^T with
// L = [L_s 0; A_Js L_s^{-T} L_J] and L_J L_J^T = S_J, so u_J = L_J^{-T} x_J and
// u_s = L_s^{-T} (x_s - L_s^{-1} A_sJ u_J).
void gamma_rinv(Handle& h, const double* X, double* Out, int ncols) {
  hipStream_t st = h.stream;
  const int64_t n2pad = h.L2.nrows_pad, nJpad = h.LJ.nrows_pad;
  DBuf<double> Bs, Bt, Gj;
  if (nJpad) {
    Gj.alloc(nJpad * ncols);
    gather_rows<double>(nJpad, h.jsrc, X, ncols, Gj.p, ncols, ncols, st);
    tile_solve_bwd<double>(h.LJ, Gj.p, ncols, ncols, 0, st);  // u_J
    scatter_rows<double, double>(nJpad, h.jsrc, Gj.p, ncols, Out, ncols, ncols, st);
  }
  if (n2pad) {
    Bs.alloc(n2pad * ncols);
    gather_rows<double>(n2pad, h.l2src, X, ncols, Bs.p, ncols, ncols, st);
    if (nJpad && h.AsJ.nnz) {
      Bt.alloc(n2pad * ncols);
      csr_mult<double>(h.AsJ, Gj.p, ncols, Bt.p, ncols, ncols, st);                // A_sJ u_J
      tile_solve_fwd<double>(h.L2, Bt.p, ncols, ncols, 64, st);                    // L_s^{-1} A_sJ u_J
      axpby(n2pad * ncols, -1.0, Bt.p, 1.0, Bs.p, st);
    }
    tile_solve_bwd<double>(h.L2, Bs.p, ncols, ncols, 0, st);  // u_s
    scatter_rows<double, double>(n2pad, h.l2src, Bs.p, ncols, Out, ncols, ncols, st);
  }
}

// The block CG in the inner precision.  NS_BF16: the operators on BF16 operands; a breakdown there (P^T S P
// not positive definite: the BF16 rounding of S_j is larger than S_Gamma's small eigenvalues) is the measured
// gate -- the solve is run again with FP32 Schur operands, the preconditioner keeping its BF16 operands.
template <class Rhs>
void run_inner(Handle& h, SmallMats& sm, Rhs rhs, double* D) {
  if (!h.prec_inner) {
    SchurOps<double> ops{h};
    block_pcg<double>(h, sm, ops, rhs, D);
    return;
  }
  BF16Scope b16(h);
  SchurOps<float> ops{h};
  if (h.bf16 && h.bf16_schur) {
    try {
      block_pcg<float>(h, sm, ops, rhs, D);
      return;
    } catch (const Error& e) {
      if (e.status != BREAKDOWN) throw;
      (void)hipGetLastError();
      NS_HIP(hipMemsetAsync(sm.flag, 0, 4 * sizeof(int), h.stream));
      h.bf16_schur = 0;
    }
  }
  block_pcg<float>(h, sm, ops, rhs, D);
}

// The operators of the inner system exactly as Algorithm alg:prec1 step 3 prints it: rows = padded interior rows
// (zero on the padding), S = S_I = A_I - A_IGamma A_Gamma^{-1} A_GammaI (eq. SI), preconditioner A_I^{-1}.  A_I P
// is the interior part of A [P; 0] (the original matrix times P with the interface rows zero).  FP64, one problem.
struct FormAOps {
  Handle& h;
  DBuf<double> full, fullA, g1, g2, tI;
  explicit FormAOps(Handle& hh) : h(hh) {
    const int64_t s = h.s;
    full.alloc(h.n * s);
    fullA.alloc(h.n * s);
    g1.alloc(h.nG * s);
    g2.alloc(h.nG * s);
    tI.alloc(h.L1.nrows_pad * s);
    NS_HIP(hipMemsetAsync(full.p, 0, h.n * s * sizeof(double), h.stream));  // its interface rows stay zero
  }
  const Seg& seg() const { return h.segI.view; }
  int64_t rows() const { return h.L1.nrows_pad; }
  void S(const double* P, double* Q) {
    hipStream_t st = h.stream;
    const int s = h.s;
    const int64_t nIp = h.L1.nrows_pad;
    scatter_rows<double, double>(nIp, h.iperm, P, s, full.p, s, s, st);  // [P; 0] in the original order
    csr_mult<double>(h.Aorig, full.p, s, fullA.p, s, s, st);              // A [P; 0]
    gather_rows<double>(nIp, h.iperm, fullA.p, s, Q, s, s, st);           // A_I P (zero on the padding)
    csr_mult<double>(h.AGI, P, s, g1.p, s, s, st);                        // A_GammaI P
    op_gamma_solve<double>(h, g1.p, s, g2.p, s, s);                       // A_Gamma^{-1} A_GammaI P
    csr_mult<double>(h.AIG, g2.p, s, tI.p, s, s, st);                     // A_IGamma (...)
    axpby(nIp * s, -1.0, tI.p, 1.0, Q, st);                                // S_I P
  }
  void M(const double* R, double* Z) {
    NS_HIP(hipMemcpyAsync(Z, R, h.L1.nrows_pad * h.s * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
    tile_solve<double>(h.L1, Z, h.s, h.s, h.trsm_cols, h.stream);        // A_I^{-1} R
  }
};

// Block CG on S_I X = F (F, X: padded interior rows x s, FP64), preconditioned by A_I^{-1}.
void inner_solve_forma(Handle& h, SmallMats& sm, const double* F, double* X) {
  FormAOps ops(h);
  const int64_t n = h.L1.nrows_pad * h.s;
  auto rhs = [&](double* R) { NS_HIP(hipMemcpyAsync(R, F, n * sizeof(double), hipMemcpyDeviceToDevice, h.stream)); };
  block_pcg<double>(h, sm, ops, rhs, X);
}

// Block CG on the shifted system with right-hand side F = W G (G: n_G x s, FP64) in the inner precision.
void inner_solve_w(Handle& h, SmallMats& sm, const double* G, double* D) {
  const int s = h.s;
  const int64_t nG = h.nG;
  auto rhs = [&](auto* R) {
    using T = std::remove_pointer_t<decltype(R)>;
    if constexpr (sizeof(T) == 8) {
      op_schur<double>(h, G, s, R, s, s, /*w_only=*/true);
    } else {
      DBuf<float> Gf;
      Gf.alloc(nG * s);
      convert_block<double, float>(nG, s, G, s, Gf.p, s, h.stream);
      op_schur<float>(h, Gf.p, s, R, s, s, /*w_only=*/true);
    }
  };
  run_inner(h, sm, rhs, D);
}

// Block CG on the shifted system with a given right-hand side F (FP64, n_G x s).
void inner_solve_f(Handle& h, SmallMats& sm, const double* F, double* D) {
  const int s = h.s;
  const int64_t nG = h.nG;
  auto rhs = [&](auto* R) {
    using T = std::remove_pointer_t<decltype(R)>;
    if constexpr (sizeof(T) == 8)
      NS_HIP(hipMemcpyAsync(R, F, nG * s * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
    else
      convert_block<double, float>(nG, s, F, s, R, s, h.stream);
  };
  run_inner(h, sm, rhs, D);
}

// The low-rank term of the chosen variant (Algorithm alg:prec1 and its analogues for M_1 and M_3) with q power
// iterations (eq. power): products B G through the inner block solves, the sketch orthonormalised after every
// product but the last, the Nystrom core on the last one, then Z.  mark() is called after the last inner solve.
template <class Mark>
void lowrank_setup(Handle& h, SmallMats& sm, const double* omega, Mark mark) {
  hipStream_t st = h.stream;
  const int s = h.s, k = h.k, np = h.nprob;
  const int64_t nG = h.nG, nIp = h.L1.nrows_pad;
  const bool m3 = h.variant == NS_VARIANT_M3, m1 = h.variant == NS_VARIANT_M1;
  const bool forma = h.inner_form == NS_INNER_FORM_A;
  std::vector<int64_t> prow(np);
  for (int q = 0; q < np; ++q) prow[q] = h.h_goff[q + 1] - h.h_goff[q];
  const int64_t rows = m3 ? nIp : nG;  // rows of the sketch and of B G
  if (m3 || forma) h.segI.build({0, nIp}, st);
  if (m3) prow.assign(1, nIp);
  DBuf<double> FI, XI;  // form A: right-hand side and solution on the padded interior rows
  if (forma && !m3) {
    FI.alloc(nIp * s);
    XI.alloc(nIp * s);
  }
  const Seg& sg = m3 ? h.segI.view : h.segG.view;
  DBuf<double> Gb, BGb, BGs, Db, Ds, F, work;
  for (DBuf<double>* b : {&Gb, &BGb}) b->alloc(rows * s);
  Db.alloc(nG * s);
  if (m3) F.alloc(nG * s);
  work.alloc(gram_work_elems(sg, s));
  double* G = Gb.p;   // current sketch (M_1: in the coordinates of R_Gamma^{-1})
  double* BG = BGb.p;
  double* D = Db.p;
  // the first sketch
  if (m3)
    gather_rows<double>(nIp, h.icomp, omega, s, G, s, s, st);  // padded interior rows, zero on the padding
  else if (m1)
    gamma_rinv(h, omega, G, s);
  else
    NS_HIP(hipMemcpyAsync(G, omega, nG * s * sizeof(double), hipMemcpyDeviceToDevice, st));
  h.it_inner.assign(np, 0);
  h.conv_inner.assign(np, 1);
  for (int it = 0; it <= h.power; ++it) {
    if (forma && m3) {
      inner_solve_forma(h, sm, G, BG);                    // S_I^{-1} G, the literal inner system
    } else if (forma) {
      csr_mult<double>(h.AIG, G, s, FI.p, s, s, st);      // F = A_IGamma G
      inner_solve_forma(h, sm, FI.p, XI.p);               // S_I X = F
      csr_mult<double>(h.AGI, XI.p, s, BG, s, s, st);     // B G = A_GammaI X
    } else if (m3) {
      // S_I^{-1} G = A_I^{-1} (G + A_IGamma D) with S_Gamma D = A_GammaI A_I^{-1} G (Sherman-Morrison-Woodbury)
      NS_HIP(hipMemcpyAsync(BG, G, rows * s * sizeof(double), hipMemcpyDeviceToDevice, st));
      tile_solve<double>(h.L1, BG, s, s, h.trsm_cols, st);
      csr_mult<double>(h.AGI, BG, s, F.p, s, s, st);
      inner_solve_f(h, sm, F.p, D);
      csr_mult<double>(h.AIG, D, s, BG, s, s, st);
      axpby(rows * s, 1.0, G, 1.0, BG, st);
      tile_solve<double>(h.L1, BG, s, s, h.trsm_cols, st);
    } else {
      inner_solve_w(h, sm, G, D);                          // S_Gamma D = W G
      csr_mult<double>(h.AGG, D, s, BG, s, s, st);         // B G = A_Gamma D (M_1: R_Gamma^T times R_Gamma D)
    }
    if (it == h.power) break;
    // next sketch: the orthonormalised product (M_1: D in the A_Gamma inner product, i.e. R_Gamma^{-1} times
    // the orthonormal basis of R_Gamma D)
    double* X = m1 ? D : BG;
    double* MX = m1 ? BG : nullptr;
    if (!Ds.p) Ds.alloc(nG * s);
    if (!BGs.p) BGs.alloc(rows * s);
    double* Xs = m1 ? Ds.p : BGs.p;
    double* MXs = m1 ? BGs.p : nullptr;
    chol_qr3(h, sm, sg, prow, s, X, Xs, MX, MXs, work);
    NS_HIP(hipMemcpyAsync(G, X, rows * s * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  mark();
  DBuf<double> out;
  out.alloc(rows * std::max(k, 1));
  nystrom_factor(h, sm, sg, prow, rows, G, BG, m1 ? D : nullptr, out.p);
  h.Z.alloc(nG * (k > 0 ? k : 1));
  NS_HIP(hipMemsetAsync(h.Z.p, 0, h.Z.n * sizeof(double), st));
  if (h.k_eff > 0) {
    if (m1) {
      // Z = R_Gamma^{-1} U = (D orthonormalised in the A_Gamma inner product) W(:, 1:k')
      NS_HIP(hipMemcpyAsync(h.Z.p, out.p, nG * k * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else if (m3) {
      // Z = A_Gamma^{-1} A_GammaI V (V: padded interior rows)
      DBuf<double> t;
      t.alloc(nG * k);
      csr_mult<double>(h.AGI, out.p, k, t.p, k, k, st);
      op_gamma_solve<double>(h, t.p, k, h.Z.p, k, k);
    } else {
      h.U.alloc(nG * k);
      NS_HIP(hipMemcpyAsync(h.U.p, out.p, nG * k * sizeof(double), hipMemcpyDeviceToDevice, st));
      op_gamma_solve<double>(h, h.U.p, k, h.Z.p, k, k);
    }
  }
  NS_HIP(hipStreamSynchronize(st));
}

// Judge a proposed starting subspace Z0 (n_G x k, one problem): Z = A_Gamma^{-1} Z0, Rayleigh-Ritz on the
// pencil (S_Gamma, A_Gamma) over span(Z) (Ritz values ascending, Ritz vectors Y = Z C with Y^T A_Gamma Y = I),
// eigen-residuals rho_i = ||S y_i - lambda_i A_Gamma y_i|| / ||A_Gamma y_i||; accepted when the ceil(k/2) smallest
// Ritz values have rho_i <= accept_tol.  Accepted: Z <- Y (the deflation space of the adapted deflation).
bool judge_proposal(Handle& h) {
  hipStream_t st = h.stream;
  const Seg& sg = h.segG.view;
  const int k = h.k;
  const int64_t nG = h.nG, kk = int64_t(k) * k;
  DBuf<double> Zp, SZ, AZ, Y, R, work, sm, colsq;
  for (DBuf<double>* b : {&Zp, &SZ, &AZ, &Y, &R}) b->alloc(nG * k);
  work.alloc(gram_work_elems(sg, k));
  sm.alloc(10 * kk + 4 * size_t(k) + 16);
  colsq.alloc(2 * size_t(k));
  double* Ar = sm.p;
  double* Br = Ar + kk;
  double* C = Br + kk;
  double* Cl = C + kk;
  double* lam = Cl + kk;
  double* ws = lam + k;
  DBuf<int> flag;
  flag.alloc(1);
  NS_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  op_gamma_solve<double>(h, h.proposal, k, Zp.p, k, k);                // Z = A_Gamma^{-1} Z0
  op_schur<double>(h, Zp.p, k, SZ.p, k, k, false);                      // S Z
  csr_mult<double>(h.AGG, Zp.p, k, AZ.p, k, k, st);                     // A_Gamma Z
  gram<double, double>(sg, Zp.p, k, k, SZ.p, k, k, Ar, kk, 1.0, 0.0, work, st);
  gram<double, double>(sg, Zp.p, k, k, AZ.p, k, k, Br, kk, 1.0, 0.0, work, st);
  small_gevd(k, Ar, Br, lam, C, Cl, flag, ws, h.sws, st);
  ts_update<double>(sg, k, Y.p, k, 0.0, 1.0, Zp.p, k, k, C, k, 0, nullptr, 0, 0, nullptr, 0, 0, st);   // Y = Z C
  ts_update<double>(sg, k, R.p, k, 0.0, 1.0, SZ.p, k, k, C, k, 0, AZ.p, k, k, Cl, k, 0, st);           // S Y - A Y L
  col_sumsq<double>(sg, k, R.p, k, colsq.p, work, st);
  ts_update<double>(sg, k, SZ.p, k, 0.0, 1.0, AZ.p, k, k, C, k, 0, nullptr, 0, 0, nullptr, 0, 0, st);  // A Y
  col_sumsq<double>(sg, k, SZ.p, k, colsq.p + k, work, st);
  std::vector<double> cs(2 * k);
  int fl = 0;
  NS_HIP(hipMemcpyAsync(&fl, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  read_back(h, cs.data(), colsq.p, 2 * k);
  if (fl) {  // Z^T A_Gamma Z singular: the proposal is rank deficient
    h.proposal_rho = INFINITY;
    return false;
  }
  double rmax = 0.0;
  for (int i = 0; i < (k + 1) / 2; ++i) {
    const double rho = cs[k + i] > 0.0 ? std::sqrt(cs[i] / cs[k + i]) : INFINITY;
    rmax = (rho > rmax || !(rho == rho)) ? rho : rmax;
  }
  h.proposal_rho = rmax;
  if (!(rmax <= h.accept_tol)) return false;
  h.Z.alloc(nG * k);
  NS_HIP(hipMemcpyAsync(h.Z.p, Y.p, nG * k * sizeof(double), hipMemcpyDeviceToDevice, st));
  h.Sigma.alloc(k);
  NS_HIP(hipMemsetAsync(h.Sigma.p, 0, k * sizeof(double), st));
  h.k_eff = k;
  h.h_keff.assign(1, k);
  h.keff_d.alloc(1);
  upload(h.keff_d.p, h.h_keff.data(), sizeof(int), st);
  NS_HIP(hipStreamSynchronize(st));
  return true;
}

// Adapted deflation: SZ = S Z, E = Z^T S Z and chol(E), per problem.
void setup_adef2(Handle& h) {
  hipStream_t st = h.stream;
  const Seg& sg = h.segG.view;
  const int k = h.k, np = h.nprob;
  const int64_t nG = h.nG, kk = int64_t(k) * k;
  if (h.k_eff == 0) return;
  h.SZ.alloc(nG * k);
  h.Echol.alloc(size_t(kk) * np);
  op_schur<double>(h, h.Z.p, k, h.SZ.p, k, k, false);
  DBuf<double> work;
  work.alloc(gram_work_elems(sg, k));
  gram<double, double>(sg, h.Z.p, k, k, h.SZ.p, k, k, h.Echol.p, kk, 1.0, 0.0, work, st);
  NS_HIP(hipMemsetAsync(h.dflags.p + 12, 0, sizeof(int), st));
  small_chol_solve(Batch{np, h.keff_d}, k, h.Echol.p, kk, nullptr, 0, 0, nullptr, 0, 0, 0, 0, 1.0, h.dflags.p + 12,
                   h.sws, st);
  int fl = 0;
  read_back(h, &fl, h.dflags.p + 12, 1);
  if (fl) fail(BREAKDOWN, "Z^T S Z is not positive definite");
}

// z = M r for ncols vectors (FP64, interface order, row-major), every problem with its own low-rank term.
// c1, c2: k x ncols per problem.
void apply_prec(Handle& h, const double* r, int64_t ldr, double* z, int64_t ldz, int ncols, double* work,
                double* c1, double* c2, const SmallWs& ws) {
  hipStream_t st = h.stream;
  const Seg& sg = h.segG.view;
  const int k = h.k, np = h.nprob;
  const int64_t cs = int64_t(k) * ncols;
  op_gamma_solve<double>(h, r, ldr, z, ldz, ncols);  // t = A_Gamma^{-1} r
  if (h.k_eff == 0) return;
  if (h.apply_mode == NS_APPLY_M2) {
    gram<double, double>(sg, h.Z.p, k, k, r, ldr, ncols, c1, cs, 1.0, 0.0, work, st, h.Sigma.p, k);  // Sigma Z^T r
    ts_update<double>(sg, ncols, z, ldz, 1.0, 1.0, h.Z.p, k, k, c1, ncols, cs, nullptr, 0, 0, nullptr, 0, 0, st);
  } else {
    gram<double, double>(sg, h.Z.p, k, k, r, ldr, ncols, c1, cs, 1.0, 0.0, work, st);    // Z^T r
    gram<double, double>(sg, h.SZ.p, k, k, z, ldz, ncols, c1, cs, -1.0, 1.0, work, st);  // - (SZ)^T t
    small_chol_apply(Batch{np, h.keff_d}, k, h.Echol.p, int64_t(k) * k, c1, ncols, cs, c2, ncols, cs, ncols, k, 1.0,
                     ws, st);  // E^{-1} (...)
    ts_update<double>(sg, ncols, z, ldz, 1.0, 1.0, h.Z.p, k, k, c2, ncols, cs, nullptr, 0, 0, nullptr, 0, 0, st);
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

__global__ void k_sqrt_inplace(int n, double* x, int stride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[int64_t(i) * stride] = sqrt(x[int64_t(i) * stride]);
}

// PCG iterations for every problem until all are done or maxit iterations ran.  head(s): q = A p, alpha,
// w and r, the stopping test; tail(s): z = M r, beta, p.  The iteration index lives on the device, so the same
// launches, recorded once into a HIP graph, serve every iteration (m per replay); the first iteration runs
// with plain launches (it also sizes every workspace the body uses).  hc: problems done, iterations run.
template <class Head, class Tail>
void pcg_loop(Handle& h, int np, const PcgState& S, int maxit, int hc[2], Head head, Tail tail) {
  hipStream_t st = h.stream;
  int m = h.pcg_graph == 0 ? tuned("pcg_graph_iters", "f64", h.nG, np > 1 ? 4 : 1) : h.pcg_graph;
  if (kernel_timing_in_loops(true)) m = 0;  // every launch timed
  head(st);
  read_back(h, hc, S.ndone, 2);
  if (hc[0] < np && hc[1] < maxit) tail(st);
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  if (m > 0 && hc[0] < np && hc[1] < maxit) {
    // record m iterations on a private stream (the handle's stream may be the null stream)
    NS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    h.stream = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        for (int t = 0; t < m; ++t) {
          head(cap);
          tail(cap);
        }
      } catch (...) {
        (void)hipStreamEndCapture(cap, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        h.stream = st;
        (void)hipStreamDestroy(cap);
        throw;
      }
      e = hipStreamEndCapture(cap, &graph);
    }
    h.stream = st;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamDestroy(cap);
      fail(HIP, std::string("PCG graph capture failed: ") + hipGetErrorString(e));
    }
  }
  if (exec && hc[0] < np && hc[1] < maxit) {
    // One replay ahead: replay g + 1 is queued before the host reads the counters left by replay g, so the
    // device never waits for the host's test.  Replays after convergence change nothing (finished problems
    // are frozen, iterations past maxit are no-ops).
    int* hp = static_cast<int*>(pinned_scratch(4 * sizeof(int)));
    Event ev[2];
    int64_t issued = hc[1];
    auto issue = [&](int s) {
      NS_HIP(hipGraphLaunch(exec, st));
      NS_HIP(hipMemcpyAsync(hp + 2 * s, S.ndone, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      NS_HIP(hipEventRecord(ev[s].e, st));
      issued += m;
    };
    int slot = 0;
    issue(0);
    for (;;) {
      const bool more = issued < maxit;
      if (more) issue(slot ^ 1);
      NS_HIP(hipEventSynchronize(ev[slot].e));
      hc[0] = hp[2 * slot];
      hc[1] = hp[2 * slot + 1];
      if (hc[0] >= np || hc[1] >= maxit || !more) break;
      slot ^= 1;
    }
    NS_HIP(hipStreamSynchronize(st));  // the replay queued ahead has finished too
    stream_idle(st);
  }
  while (!exec && hc[0] < np && hc[1] < maxit) {
    head(st);
    read_back(h, hc, S.ndone, 2);
    if (hc[0] >= np || hc[1] >= maxit) break;
    tail(st);
    read_back(h, hc, S.ndone, 2);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (cap) (void)hipStreamDestroy(cap);
}

// Results of one problem's solve.
struct SolveOut {
  int it = 0, converged = 0;
  double relres_schur = 0.0, relres_true = 0.0;
  std::vector<double> hist;
};

// True residual ||b - A x|| / ||b|| and the recurrence history of every problem after a PCG run.
// tmp: n doubles of scratch; ist: [done per problem, iterations per problem]; hist: hs values per problem.
void pcg_results(Handle& h, const double* b, const double* x, double* tmp, const int* ist, const double* hist,
                 int64_t hs, int maxit, int iters, std::vector<SolveOut>& res) {
  hipStream_t st = h.stream;
  const int np = h.nprob;
  const int64_t n = h.n;
  csr_mult<double>(h.Aorig, x, 1, tmp, 1, 1, st);
  k_sub<<<unsigned((n + 255) / 256), 256, 0, st>>>(n, b, tmp, tmp);
  NS_LAUNCH_CHECK();
  const Seg& sn = h.segN.view;
  DBuf<double> rr, work2;
  rr.alloc(2 * size_t(np));
  work2.alloc(size_t(sn.nchunk) + 16);
  dot(sn, tmp, tmp, rr.p, 2, work2, st);
  dot(sn, b, b, rr.p + 1, 2, work2, st);
  std::vector<double> hrr(2 * np), hh(size_t(hs) * np);
  std::vector<int> hi(2 * np);
  NS_HIP(hipMemcpyAsync(hrr.data(), rr.p, 2 * np * sizeof(double), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(hi.data(), ist, 2 * np * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(hh.data(), hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  res.assign(np, SolveOut{});
  for (int g = 0; g < np; ++g) {
    SolveOut& o = res[g];
    const int done = hi[g];
    o.it = done ? hi[np + g] : iters;
    if (!done) o.it = std::min(o.it, maxit);
    o.converged = done == 1;
    o.hist.assign(hh.begin() + size_t(g) * hs, hh.begin() + size_t(g) * hs + o.it + 1);
    o.relres_schur = o.hist.back();
    o.relres_true = hrr[2 * g + 1] > 0 ? std::sqrt(hrr[2 * g] / hrr[2 * g + 1]) : 0.0;
  }
}

// f = b_Gamma - A_GammaI A_I^{-1} b_I; PCG on S_Gamma w = f with M (w0 = Q f for the adapted deflation);
// x_I = A_I^{-1} (b_I - A_IGamma w), x_Gamma = w (eqs. A_LDLT and Sx=b), for every problem at once.
// b, x: the batch's right-hand side and solution (original order of the block-diagonal matrix).
void pcg_core(Handle& h, const double* b, double* x, double rtol, int maxit, std::vector<SolveOut>& res) {
  hipStream_t st = h.stream;
  const Seg& sg = h.segG.view;
  const int np = h.nprob;
  const int64_t n = h.n, nG = h.nG, nIp = h.L1.nrows_pad;
  const int k = std::max(h.k, 1);
  DBuf<double> bI, f, w, r, z, p, q, work, c1, c2, tmp, psd, hist;
  DBuf<int> ist;
  bI.alloc(nIp);
  for (DBuf<double>* v : {&f, &w, &r, &z, &p, &q}) v->alloc(nG);
  work.alloc(std::max<size_t>(gram_work_elems(sg, k), 2 * size_t(sg.nchunk) + 32));
  c1.alloc(size_t(k) * np);
  c2.alloc(size_t(k) * np);
  tmp.alloc(std::max(n, nIp));  // gathers of the padded interior rows (n_I padded can exceed n)
  psd.alloc(size_t(PS) * np);
  const int64_t hs = int64_t(maxit) + 1;
  hist.alloc(size_t(hs) * np);
  ist.alloc(2 * size_t(np) + 4);
  NS_HIP(hipMemsetAsync(psd.p, 0, psd.n * sizeof(double), st));
  NS_HIP(hipMemsetAsync(ist.p, 0, ist.n * sizeof(int), st));
  PcgState S{psd.p, ist.p, ist.p + np, ist.p + 2 * np, ist.p + 2 * np + 1, hist.p, hs, rtol, maxit};
  // f = b_Gamma - A_GammaI A_I^{-1} b_I
  gather_rows<double>(nIp, h.iperm, b, 1, bI.p, 1, 1, st);
  tile_solve<double>(h.L1, bI.p, 1, 1, h.trsm_cols, st);
  gather_rows<double>(nG, h.gperm, b, 1, tmp.p, 1, 1, st);
  csr_mult<double>(h.AGI, bI.p, 1, f.p, 1, 1, st);
  axpby(nG, 1.0, tmp.p, -1.0, f.p, st);
  dot(sg, f.p, f.p, psd.p + PS_NF, PS, work, st);
  k_sqrt_inplace<<<(np + 255) / 256, 256, 0, st>>>(np, psd.p + PS_NF, PS);
  NS_LAUNCH_CHECK();
  NS_HIP(hipMemsetAsync(w.p, 0, nG * sizeof(double), st));
  NS_HIP(hipMemcpyAsync(r.p, f.p, nG * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (h.apply_mode == NS_APPLY_ADEF2 && h.k_eff > 0) {
    // w0 = Z E^{-1} Z^T f ; r = f - S w0
    const int kk = h.k;
    gram<double, double>(sg, h.Z.p, kk, kk, f.p, 1, 1, c1.p, kk, 1.0, 0.0, work, st);
    small_chol_apply(Batch{np, h.keff_d}, kk, h.Echol.p, int64_t(kk) * kk, c1.p, 1, kk, c2.p, 1, kk, 1, kk, 1.0,
                     h.sws, st);
    ts_update<double>(sg, 1, w.p, 1, 0.0, 1.0, h.Z.p, kk, kk, c2.p, 1, kk, nullptr, 0, 0, nullptr, 0, 0, st);
    op_schur<double>(h, w.p, 1, q.p, 1, 1, false);
    axpby(nG, 1.0, f.p, -1.0, q.p, st);
    NS_HIP(hipMemcpyAsync(r.p, q.p, nG * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  dot(sg, r.p, r.p, psd.p + PS_RN2, PS, work, st);
  pcg_init_check(np, S, st);
  int hc[2] = {0, 0};  // problems done, iterations run
  read_back(h, hc, S.ndone, 2);
  // One PCG iteration for every problem; the iteration index lives on the device, so the same launches
  // (recorded once into a graph) serve every iteration.
  double* dpart = work.p + sg.nchunk + 16;  // chunk partials of p^T q and r^T z (work itself takes ||r||^2)
  auto head = [&](hipStream_t s) {
    op_schur<double>(h, p.p, 1, q.p, 1, 1, false);            // q = S p
    dot_partials(sg, p.p, q.p, dpart, s);                       // p^T q per chunk
    pcg_update_wr(sg, S, w.p, r.p, p.p, q.p, dpart, work, s);  // alpha, w, r, ||r||, stopping test
  };
  auto tail = [&](hipStream_t s) {
    apply_prec(h, r.p, 1, z.p, 1, 1, work, c1, c2, h.sws);  // z = M r
    dot_partials(sg, r.p, z.p, dpart, s);                    // r^T z per chunk
    pcg_update_p(sg, S, z.p, p.p, dpart, s);                 // rho_{j+1}, p = z + beta p
    pcg_advance(np, S, s);
  };
  if (hc[0] < np && maxit > 0) {
    apply_prec(h, r.p, 1, z.p, 1, 1, work, c1, c2, h.sws);
    dot(sg, r.p, z.p, psd.p + PS_RHO, PS, work, st);  // rho_0
    NS_HIP(hipMemcpyAsync(p.p, z.p, nG * sizeof(double), hipMemcpyDeviceToDevice, st));
    pcg_loop(h, np, S, maxit, hc, head, tail);
  }
  const int iters = std::min(hc[1], maxit);
  // back-substitution: x_I = A_I^{-1} (b_I - A_IGamma w), x_Gamma = w
  gather_rows<double>(nIp, h.iperm, b, 1, tmp.p, 1, 1, st);
  csr_mult<double>(h.AIG, w.p, 1, bI.p, 1, 1, st);
  axpby(nIp, 1.0, tmp.p, -1.0, bI.p, st);
  tile_solve<double>(h.L1, bI.p, 1, 1, h.trsm_cols, st);
  scatter_rows<double, double>(nIp, h.iperm, bI.p, 1, x, 1, 1, st);
  scatter_rows<double, double>(nG, h.gperm, w.p, 1, x, 1, 1, st);
  pcg_results(h, b, x, tmp.p, ist.p, hist.p, hs, maxit, iters, res);
}

// PCG on A x = b for every problem at once, preconditioned by the approximate block LDL^T factorisation with
// S~^{-1} = M (eq. M_inv_A): z_I = u_I - A_I^{-1} A_IGamma y_G, z_G = y_G, with u_I = A_I^{-1} r_I and
// y_G = M (r_G - A_GammaI u_I).  Vectors in the original order; x_0 = 0; stops on ||r_j|| / ||b|| <= rtol.
void pcg_full_core(Handle& h, const double* b, double* x, double rtol, int maxit, std::vector<SolveOut>& res) {
  hipStream_t st = h.stream;
  const Seg& sg = h.segG.view;
  const Seg& sn = h.segN.view;
  const int np = h.nprob;
  const int64_t n = h.n, nG = h.nG, nIp = h.L1.nrows_pad;
  const int k = std::max(h.k, 1);
  DBuf<double> r, z, p, q, uI, vI, rg, yg, work, workN, c1, c2, tmp, psd, hist;
  DBuf<int> ist;
  for (DBuf<double>* v : {&r, &z, &p, &q}) v->alloc(n);
  for (DBuf<double>* v : {&uI, &vI}) v->alloc(nIp);
  for (DBuf<double>* v : {&rg, &yg}) v->alloc(nG);
  work.alloc(std::max<size_t>(gram_work_elems(sg, k), 2 * size_t(sg.nchunk) + 32));
  workN.alloc(2 * size_t(sn.nchunk) + 32);
  c1.alloc(size_t(k) * np);
  c2.alloc(size_t(k) * np);
  tmp.alloc(std::max(n, nIp));
  psd.alloc(size_t(PS) * np);
  const int64_t hs = int64_t(maxit) + 1;
  hist.alloc(size_t(hs) * np);
  ist.alloc(2 * size_t(np) + 4);
  NS_HIP(hipMemsetAsync(psd.p, 0, psd.n * sizeof(double), st));
  NS_HIP(hipMemsetAsync(ist.p, 0, ist.n * sizeof(int), st));
  PcgState S{psd.p, ist.p, ist.p + np, ist.p + 2 * np, ist.p + 2 * np + 1, hist.p, hs, rtol, maxit};
  double* dpart = workN.p + sn.nchunk + 16;  // chunk partials of p^T q and r^T z
  auto prec = [&](hipStream_t s) {
    gather_rows<double>(nIp, h.iperm, r.p, 1, uI.p, 1, 1, s);
    tile_solve<double>(h.L1, uI.p, 1, 1, h.trsm_cols, s);     // u_I = A_I^{-1} r_I
    gather_rows<double>(nG, h.gperm, r.p, 1, rg.p, 1, 1, s);
    csr_mult<double>(h.AGI, uI.p, 1, yg.p, 1, 1, s);
    axpby(nG, 1.0, rg.p, -1.0, yg.p, s);                       // r_G - A_GammaI u_I
    apply_prec(h, yg.p, 1, rg.p, 1, 1, work, c1, c2, h.sws);  // y_G = M (r_G - A_GammaI u_I)
    csr_mult<double>(h.AIG, rg.p, 1, vI.p, 1, 1, s);
    tile_solve<double>(h.L1, vI.p, 1, 1, h.trsm_cols, s);
    axpby(nIp, -1.0, vI.p, 1.0, uI.p, s);                      // z_I = u_I - A_I^{-1} A_IGamma y_G
    scatter_rows<double, double>(nIp, h.iperm, uI.p, 1, z.p, 1, 1, s);
    scatter_rows<double, double>(nG, h.gperm, rg.p, 1, z.p, 1, 1, s);
  };
  auto head = [&](hipStream_t s) {
    csr_mult<double>(h.Aorig, p.p, 1, q.p, 1, 1, s);           // q = A p
    dot_partials(sn, p.p, q.p, dpart, s);
    pcg_update_wr(sn, S, x, r.p, p.p, q.p, dpart, workN, s);   // alpha, x, r, ||r||, stopping test
  };
  auto tail = [&](hipStream_t s) {
    prec(s);
    dot_partials(sn, r.p, z.p, dpart, s);
    pcg_update_p(sn, S, z.p, p.p, dpart, s);
    pcg_advance(np, S, s);
  };
  NS_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
  NS_HIP(hipMemcpyAsync(r.p, b, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  dot(sn, b, b, psd.p + PS_NF, PS, workN, st);
  k_sqrt_inplace<<<(np + 255) / 256, 256, 0, st>>>(np, psd.p + PS_NF, PS);
  NS_LAUNCH_CHECK();
  dot(sn, r.p, r.p, psd.p + PS_RN2, PS, workN, st);
  pcg_init_check(np, S, st);
  int hc[2] = {0, 0};
  read_back(h, hc, S.ndone, 2);
  if (hc[0] < np && maxit > 0) {
    prec(st);
    dot(sn, r.p, z.p, psd.p + PS_RHO, PS, workN, st);  // rho_0
    NS_HIP(hipMemcpyAsync(p.p, z.p, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    pcg_loop(h, np, S, maxit, hc, head, tail);
  }
  pcg_results(h, b, x, tmp.p, ist.p, hist.p, hs, maxit, std::min(hc[1], maxit), res);
}

ns_status finish(Handle* h, const Error& e) {
  g_last_error = e.msg;
  if (h) h->last_error = e.msg;
  return ns_status(e.status);
}

Handle* new_handle(const ns_options* opt) {
  if (!opt) fail(INVALID_ARG, "opt must not be NULL");
  if (opt->k < 0 || opt->p < 0) fail(INVALID_ARG, "k and p must be >= 0");
  Handle* h = new Handle();
  h->stream = static_cast<hipStream_t>(opt->stream);
  h->k = opt->k;
  h->p = opt->p;
  h->s = opt->k + opt->p;
  h->tol_inner = opt->tol_inner > 0 ? opt->tol_inner : 0.1;
  h->eig_rel = opt->eig_thresh_rel > 0 ? opt->eig_thresh_rel : 1e-10;
  if (opt->prec_inner < NS_FP64 || opt->prec_inner > NS_BF16) fail(INVALID_ARG, "prec_inner must be 0, 1 or 2");
  h->prec_inner = opt->prec_inner == NS_FP64 ? 0 : 1;  // FP32 block vectors for NS_FP32 and NS_BF16
  h->bf16 = opt->prec_inner == NS_BF16 ? 1 : 0;
  h->drop_rel = opt->orth_drop_rel > 0 ? opt->orth_drop_rel : (h->prec_inner ? 1e-5 : 1e-6);
  h->max_inner = opt->max_inner_iters > 0 ? opt->max_inner_iters : 500;
  h->apply_mode = opt->apply_mode == NS_APPLY_ADEF2 ? 1 : 0;
  h->trsm_cols = opt->trsm_cols;
  h->schur_mode = opt->schur_mode;
  h->pcg_graph = opt->pcg_graph_iters;
  h->bcg_graph = opt->bcg_graph_iters;
  h->proposal = opt->proposal;
  h->accept_tol = opt->accept_tol > 0 ? opt->accept_tol : 0.2;
  h->variant = opt->variant;
  h->power = opt->power_iters;
  h->outer = opt->outer;
  h->inner_form = opt->inner_form;
  h->level2 = opt->level2;
  h->level2_k = opt->level2_k;
  h->level2_p = opt->level2_p;
  h->level2_tol = opt->level2_tol_inner;
  h->level2_omega = opt->level2_omega;
  return h;
}

void check_options(Handle* h) {
  if (h->schur_mode < 0 || h->schur_mode > 2) fail(INVALID_ARG, "schur_mode must be 0, 1 or 2");
  if (h->variant < NS_VARIANT_M2 || h->variant > NS_VARIANT_M3) fail(INVALID_ARG, "variant must be 0, 1 or 2");
  if (h->power < 0 || h->power > 32) fail(INVALID_ARG, "power_iters must be in [0, 32]");
  if (h->outer != NS_OUTER_SCHUR && h->outer != NS_OUTER_FULL) fail(INVALID_ARG, "outer must be 0 or 1");
  if (h->outer == NS_OUTER_FULL && h->apply_mode != NS_APPLY_M2)
    fail(INVALID_ARG, "the full-system outer iteration needs the symmetric additive form (NS_APPLY_M2)");
  if (h->trsm_cols != 0 && h->trsm_cols != 16 && h->trsm_cols != 32 && h->trsm_cols != 64)
    fail(INVALID_ARG, "trsm_cols must be 0, 16, 32 or 64");
  if (h->inner_form != NS_INNER_SHIFTED && h->inner_form != NS_INNER_FORM_A) fail(INVALID_ARG, "inner_form must be 0 or 1");
  if (h->inner_form == NS_INNER_FORM_A) {
    if (h->prec_inner || h->bf16) fail(INVALID_ARG, "the literal inner form runs with FP64 inner work only");
    if (h->variant == NS_VARIANT_M1) fail(INVALID_ARG, "the literal inner form serves the variants M_2 and M_3");
  }
  if (h->level2 != NS_LEVEL2_EXACT && h->level2 != NS_LEVEL2_NYSTROM) fail(INVALID_ARG, "level2 must be 0 or 1");
  if (h->level2 == NS_LEVEL2_NYSTROM) {
    if (h->prec_inner || h->bf16) fail(INVALID_ARG, "the recursive level runs with FP64 inner work only");
    if (h->variant == NS_VARIANT_M1) fail(INVALID_ARG, "variant M1 needs an exact factor of A_Gamma");
    if (h->proposal) fail(INVALID_ARG, "a learned proposal is not combined with the recursive level");
    if (h->level2_k < 0 || h->level2_p < 0) fail(INVALID_ARG, "level2_k and level2_p must be >= 0");
    if (h->level2_k > 0 && !h->level2_omega) fail(INVALID_ARG, "level2_omega is required when level2_k > 0");
  }
  h->dflags.alloc(32);
  NS_HIP(hipMemsetAsync(h->dflags.p, 0, 32 * sizeof(int), h->stream));
}

void build_recursive_level(Handle* h, const int32_t* part);

// Setup after the matrix is in place: extraction, factorisations, inner solve, Nystrom.
// omega: n_G x s row-major (the problems' sketches stacked in interface order).
void setup_core(Handle* h, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                const int32_t* part, const Pieces* pieces, const double* const* omegas, ns_setup_info* info) {
  Events ev(h->stream);
  ev.rec(0);
  extract_dbbd(*h, n, nnz, row_ptr, col_idx, val, part, pieces);
  for (int q = 0; q < h->nprob; ++q)
    if (h->s > h->h_goff[q + 1] - h->h_goff[q]) fail(INVALID_ARG, "k + p exceeds the interface size n_gamma");
  h->segG.build(h->h_goff, h->stream);
  h->segN.build(h->h_noff, h->stream);
  h->sws = small_ws(h->small, h->nprob, h->s, h->s, true);
  ev.rec(1);
  // The interface levels (patch factorisation, junction complement, explicit inverses) do not depend on the
  // interior factorisation and the local Schur formation: they run on a second stream, joined before the pivot
  // check, so the two latency-bound chains fill the device together.
  if (!h->aux) NS_HIP(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
  Event fork, join, l1done, planned;
  NS_HIP(hipEventRecord(fork.e, h->stream));
  NS_HIP(hipStreamWaitEvent(h->aux, fork.e, 0));
  // the interior factorisation is queued first; the symbolic part of the local Schur formation (which reads
  // sizes back) then runs on the second stream while the host waits and the device factorises, and the
  // interface levels follow it there (they overlap the formation's start: measured faster overall than
  // finishing them before the formation, whose event-timed launches then share the device)
  tile_cholesky(h->L1, h->dflags.p + CHOL_FLAGS, h->stream);
  NS_HIP(hipEventRecord(l1done.e, h->stream));
  {
    StreamSwap sw(*h, h->aux);
    if (h->schur_mode != SCHUR_TRIANGULAR) local_schur_plan(*h);
    NS_HIP(hipEventRecord(planned.e, h->stream));
    if (h->level2 == NS_LEVEL2_NYSTROM) {
      build_recursive_level(h, part);  // A_Gamma preconditioned one level down instead of factorised
    } else {
      tile_cholesky(h->L2, h->dflags.p + CHOL_FLAGS + 3, h->stream);
      assemble_junction(*h);
      tile_cholesky(h->LJ, h->dflags.p + CHOL_FLAGS + 6, h->stream);
      for (ns::TileLevel* lv : {&h->L2, &h->LJ})
        if (lv->nblk && lv->max_nt * TILE <= 4096 && lv->nrows_pad * lv->max_nt * TILE <= (int64_t(1) << 28))
          tile_make_inverse(*lv, h->prec_inner != 0, h->stream);
      if (h->prec_inner) {
        tile_make_fp32(h->L2, h->stream);
        tile_make_fp32(h->LJ, h->stream);
      }
      make_l2_coefs(*h);
      if (h->bf16) {
        tile_make_bf16_inverse(h->L2, h->stream);
        tile_make_bf16_inverse(h->LJ, h->stream);
      }
    }
    NS_HIP(hipEventRecord(join.e, h->stream));
  }
  NS_HIP(hipStreamWaitEvent(h->stream, planned.e, 0));  // the plan's last uploads and sorts
  if (h->schur_mode != SCHUR_TRIANGULAR) local_schur_form(*h);
  if (h->bf16) local_schur_make_bf16(*h);
  if (h->prec_inner && !h->LS.built) tile_make_fp32(h->L1, h->stream);
  // the tile-transposed interior factor is only read by the solve's single-column backward sweeps: it is made
  // on the second stream while this one runs the inner solve (after the formation, so the two do not share the
  // device), and joined at the end of the setup
  Event formed, transposed;
  NS_HIP(hipEventRecord(formed.e, h->stream));
  {
    StreamSwap sw(*h, h->aux);
    NS_HIP(hipStreamWaitEvent(h->stream, l1done.e, 0));
    NS_HIP(hipStreamWaitEvent(h->stream, formed.e, 0));
    if (trsv1_supported_size(h->L1)) tile_make_transposed(h->L1, h->stream);
    NS_HIP(hipEventRecord(transposed.e, h->stream));
  }
  NS_HIP(hipStreamWaitEvent(h->stream, join.e, 0));
  check_chol(*h, info);
  ev.rec(2);
  const int np = h->nprob;
  h->it_inner.assign(np, 0);
  h->conv_inner.assign(np, 1);
  h->relres_inner.assign(np, 0.0);
  h->h_keff.assign(np, 0);
  h->proposal_accepted = 0;
  if (h->k > 0 && h->proposal) {
    if (np != 1) fail(INVALID_ARG, "a proposal applies to one problem (not a batch)");
    if (judge_proposal(*h)) {
      h->proposal_accepted = 1;
      h->apply_mode = NS_APPLY_ADEF2;
      h->conv_inner.assign(1, 1);
      ev.rec(3);
      setup_adef2(*h);
    }
  }
  if (h->proposal_accepted) {
    // the accepted subspace replaces the inner solve and the Nystrom core
  } else if (h->k > 0) {
    SmallMats sm;
    sm.init(np, h->s, h->k);
    DBuf<double> Om;
    const double* omega = omegas[0];
    if (np > 1) {
      Om.alloc(h->nG * h->s);
      for (int q = 0; q < np; ++q)
        NS_HIP(hipMemcpyAsync(Om.p + h->h_goff[q] * h->s, omegas[q],
                              (h->h_goff[q + 1] - h->h_goff[q]) * h->s * sizeof(double), hipMemcpyDeviceToDevice,
                              h->stream));
      omega = Om.p;
    }
    lowrank_setup(*h, sm, omega, [&] { ev.rec(3); });
    if (h->apply_mode == NS_APPLY_ADEF2) setup_adef2(*h);
  } else {
    h->keff_d.alloc(np);
    NS_HIP(hipMemsetAsync(h->keff_d.p, 0, np * sizeof(int), h->stream));
    ev.rec(3);
  }
  NS_HIP(hipStreamWaitEvent(h->stream, transposed.e, 0));
  ev.rec(4);
  NS_HIP(hipStreamSynchronize(h->stream));
  if (info) {
    for (int q = 0; q < np; ++q) {
      ns_setup_info& o = info[q];
      o.n = h->h_noff[q + 1] - h->h_noff[q];
      o.n_gamma = h->h_goff[q + 1] - h->h_goff[q];
      o.n_interior = o.n - o.n_gamma;
      o.n_junction = h->LJ.nblk ? h->LJ.h_nb[q] : 0;
      o.n_sub = pieces ? pieces->sub[q + 1] - pieces->sub[q] : h->nsub;
      o.n_level2_blocks = pieces ? pieces->l2[q + 1] - pieces->l2[q] : h->nl2;
      o.k_eff = h->h_keff[q];
      o.proposal_accepted = h->proposal_accepted;
      o.it_inner = h->it_inner[q];
      o.inner_converged = h->conv_inner[q];
      o.inner_relres = h->relres_inner[q];
      o.t_extract = ev.sec(0, 1);
      o.t_factor = ev.sec(1, 2);
      o.t_inner = ev.sec(2, 3);
      o.t_nystrom = ev.sec(3, 4);
      o.t_total = ev.sec(0, 4);
      o.inner_bf16_schur = h->bf16 && h->bf16_schur ? 1 : 0;
      o.level2_it_inner = h->sub ? h->sub->it_inner[0] : 0;
      o.level2_k_eff = h->sub ? h->sub->h_keff[0] : 0;
    }
  }
}

__global__ void k_level2_labels(int64_t nG, const int32_t* __restrict__ gperm, const int32_t* __restrict__ part,
                                int32_t* __restrict__ out) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= nG) return;
  const int lab = part[gperm[g]];
  out[g] = lab <= -2 ? -2 - lab : -1;
}

// The level below of the recursive construction: A_Gamma (this handle's interface rows and their couplings,
// in interface order) set up as a problem of its own, with the interface blocks as its subdomains and the
// junction nodes as its interface, on this handle's current stream.  The handle owns it from then on.
void build_recursive_level(Handle* h, const int32_t* part) {
  if (h->nprob != 1) fail(INVALID_ARG, "the recursive level applies to one problem (not a batch)");
  if (h->nl2 == 0 || h->nJ == 0)
    fail(INVALID_ARG, "the recursive level needs at least one interface block and one junction node");
  if (h->level2_k > 0 && int64_t(h->level2_k) + h->level2_p > h->nJ)
    fail(INVALID_ARG, "level2_k + level2_p exceeds the number of junction nodes");
  DBuf<int32_t> part2;
  part2.alloc(h->nG);
  k_level2_labels<<<unsigned((h->nG + 255) / 256), 256, 0, h->stream>>>(h->nG, h->gperm, part, part2);
  NS_LAUNCH_CHECK();
  ns_options o{};
  o.k = h->level2_k;
  o.p = h->level2_k > 0 ? h->level2_p : 0;
  o.tol_inner = h->level2_tol > 0 ? h->level2_tol : h->tol_inner;
  o.eig_thresh_rel = h->eig_rel;
  o.orth_drop_rel = h->drop_rel;
  o.max_inner_iters = h->max_inner;
  o.prec_inner = NS_FP64;
  o.apply_mode = NS_APPLY_M2;
  o.trsm_cols = h->trsm_cols;
  o.schur_mode = h->schur_mode;
  o.omega = h->level2_omega;
  o.stream = h->stream;
  o.pcg_graph_iters = -1;
  o.bcg_graph_iters = h->bcg_graph;
  Handle* g = new_handle(&o);
  h->sub = g;  // freed with h, also when its setup fails
  check_options(g);
  const double* om = h->level2_k > 0 ? h->level2_omega : nullptr;
  setup_core(g, h->nG, h->AGG.nnz, h->AGG.ptr.p, h->AGG.col.p, h->AGG.val64.p, part2.p, nullptr, &om, nullptr);
}

// Batch layout: part labels of every problem shifted into one numbering.
__global__ void k_part_minmax(int64_t n, const int32_t* __restrict__ part, int* mm) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int pmax = INT32_MIN, pmin = INT32_MAX;
  if (i < n) pmax = pmin = part[i];
  for (int o = 32; o > 0; o >>= 1) {  // one atomic per wave
    pmax = max(pmax, __shfl_xor(pmax, o));
    pmin = min(pmin, __shfl_xor(pmin, o));
  }
  if ((threadIdx.x & 63) == 0) {
    if (pmax != INT32_MIN) atomicMax(&mm[0], pmax);
    if (pmin != INT32_MAX) atomicMin(&mm[1], pmin);
  }
}
__global__ void k_concat(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ part, int64_t e0,
                         int64_t a, int sub0, int l20, int64_t* __restrict__ rpu, int32_t* __restrict__ partu) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  rpu[a + i] = rp[i] + e0;
  const int p = part[i];
  partu[a + i] = p >= 0 ? p + sub0 : (p <= -2 ? p - l20 : -1);
}
__global__ void k_check_rows(int64_t n, int64_t nnz, const int64_t* __restrict__ rp, int* bad) {
  if (rp[0] != 0 || rp[n] != nnz) bad[0] = 1;
}
__global__ void k_cols_in_range(int64_t m, const int32_t* __restrict__ c, int64_t n, int* bad) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m && (c[e] < 0 || c[e] >= n)) bad[0] = 1;
}
__global__ void k_shift_cols(int64_t m, const int32_t* __restrict__ c, int64_t a, int32_t* __restrict__ cu) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < m) cu[e] = int32_t(c[e] + a);
}

}  // namespace

void sub_apply(Handle& g, const double* r, int64_t ldr, double* z, int64_t ldz, int ncols) {
  const int k = std::max(g.k, 1);
  if (ncols > g.sub_cols) {
    g.subW.alloc(gram_work_elems(g.segG.view, std::max(k, ncols)));
    g.subC1.alloc(size_t(k) * ncols * g.nprob);
    g.subC2.alloc(size_t(k) * ncols * g.nprob);
    g.sub_cols = ncols;
  }
  apply_prec(g, r, ldr, z, ldz, ncols, g.subW.p, g.subC1.p, g.subC2.p, g.sws);
}

}  // namespace ns

// ---------------------------------------------------------------------------------------------------------
// Allocation-free apply.  Its scratch -- the Gram partials of Z^T r (and of (S Z)^T t), the k x ncols
// coefficient blocks and the small dense kernels' workspace -- is this file-scope device array, of which every
// GPU the library runs on holds one copy until the process ends.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in symbol): the device address is looked up once per device, with
// that device current, and used from then on.
constexpr size_t kScratchDoubles = size_t(1) << 19;  // 4 MiB per device
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace ns {
namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxScratchDevices] = {};

double* scratch_address() {
  int dev = 0;
  NS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) fail(HIP, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      fail(HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch[dev] = static_cast<double*>(p);
  }
  return g_scratch[dev];
}

size_t round256(size_t n) { return (n + 31) / 32 * 32; }  // doubles, keeping 256-byte alignment
}  // namespace
}  // namespace ns

using namespace ns;

namespace ns {
namespace {
// Frees the handle's buffers in order behind the work queued on its stream.
void destroy_handle(Handle* h) {
  if (!h) return;
  if (h->sub) {
    h->sub->stream = h->stream;  // the level below may still name a stream a graph capture used
    destroy_handle(h->sub);
    h->sub = nullptr;
  }
  if (h->aux) (void)hipStreamSynchronize(h->aux);  // a failed setup may leave work queued there
  {
    StreamScope ss(h->stream);
    hipStream_t aux = h->aux;
    delete h;
    if (aux) (void)hipStreamDestroy(aux);
  }
}
}  // namespace
}  // namespace ns

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
    h = new_handle(opt);
    StreamScope ss(h->stream);
    check_options(h);
    const double* om[1] = {opt->omega};
    setup_core(h, n, nnz, row_ptr, col_idx, val, part, nullptr, om, info);
    *out = h;
    return NS_OK;
  } catch (const Error& e) {
    ns_status st = finish(h, e);
    destroy_handle(h);
    return st;
  }
}

ns_status nystrom_schur_setup_batched(int32_t nprob, const int64_t* n, const int64_t* nnz,
                                      const int64_t* const* row_ptr, const int32_t* const* col_idx,
                                      const double* const* val, const int32_t* const* part,
                                      const double* const* omega, const ns_options* opt, ns_handle* out,
                                      ns_setup_info* info) {
  if (out) *out = nullptr;
  Handle* h = nullptr;
  try {
    if (!out || !opt || !n || !nnz || !row_ptr || !col_idx || !val || !part)
      fail(INVALID_ARG, "out, opt and the per-problem arrays must not be NULL");
    if (nprob < 1 || nprob > 65535) fail(INVALID_ARG, "nprob must be in 1..65535");
    if (opt->k > 0 && !omega) fail(INVALID_ARG, "omega (the sketches) is required when k > 0");
    if (info)
      for (int q = 0; q < nprob; ++q) {
        std::memset(info + q, 0, sizeof(*info));
        info[q].bad_block = info[q].bad_col = -1;
      }
    h = new_handle(opt);
    StreamScope ss(h->stream);
    if (h->inner_form != NS_INNER_SHIFTED) fail(INVALID_ARG, "the literal inner form applies to one problem (not a batch)");
    if (h->level2 != NS_LEVEL2_EXACT) fail(INVALID_ARG, "the recursive level applies to one problem (not a batch)");
    check_options(h);
    if (h->variant == NS_VARIANT_M3 && nprob > 1)
      fail(INVALID_ARG, "the variant M_3 (sketch on the interior space) takes one problem per handle");
    hipStream_t st = h->stream;
    Pieces pc;
    pc.node.assign(nprob + 1, 0);
    pc.sub.assign(nprob + 1, 0);
    pc.l2.assign(nprob + 1, 0);
    std::vector<int64_t> eoff(nprob + 1, 0);
    DBuf<int> mm;
    mm.alloc(2 * size_t(nprob));
    std::vector<int> hmm(2 * nprob);
    for (int q = 0; q < nprob; ++q) {
      hmm[2 * q] = INT32_MIN;
      hmm[2 * q + 1] = INT32_MAX;
    }
    upload(mm.p, hmm.data(), hmm.size() * sizeof(int), st);
    for (int q = 0; q < nprob; ++q) {
      if (n[q] <= 0 || nnz[q] < n[q] || !row_ptr[q] || !col_idx[q] || !val[q] || !part[q])
        fail(INVALID_ARG, "problem " + std::to_string(q) + ": need n > 0, nnz >= n and non-NULL arrays");
      if (opt->k > 0 && !omega[q]) fail(INVALID_ARG, "problem " + std::to_string(q) + ": omega is NULL");
      if (pc.node[q] + n[q] > INT32_MAX) fail(INVALID_ARG, "batch too large (more than 2^31 - 1 unknowns)");
      pc.node[q + 1] = pc.node[q] + n[q];
      eoff[q + 1] = eoff[q] + nnz[q];
      k_part_minmax<<<unsigned((n[q] + 255) / 256), 256, 0, st>>>(n[q], part[q], mm.p + 2 * q);
      NS_LAUNCH_CHECK();
    }
    NS_HIP(hipMemcpyAsync(hmm.data(), mm.p, hmm.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    NS_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < nprob; ++q) {
      pc.sub[q + 1] = pc.sub[q] + (hmm[2 * q] >= 0 ? hmm[2 * q] + 1 : 0);
      pc.l2[q + 1] = pc.l2[q] + (hmm[2 * q + 1] <= -2 ? -hmm[2 * q + 1] - 1 : 0);
    }
    // the batch as one block-diagonal matrix (each problem's CSR is validated as part of it: its
    // columns stay inside its own rows only if they were in range)
    const int64_t nu = pc.node[nprob], nnzu = eoff[nprob];
    DBuf<int64_t> rpu;
    DBuf<int32_t> colu, partu;
    DBuf<double> valu;
    rpu.alloc(nu + 1);
    colu.alloc(nnzu);
    partu.alloc(nu);
    valu.alloc(nnzu);
    DBuf<int> bad;
    bad.alloc(1);
    NS_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
    for (int q = 0; q < nprob; ++q) {
      // per-problem CSR structure: row_ptr[0] == 0, row_ptr[n] == nnz, columns in [0, n)
      k_check_rows<<<1, 1, 0, st>>>(n[q], nnz[q], row_ptr[q], bad.p);
      NS_LAUNCH_CHECK();
      k_concat<<<unsigned((n[q] + 255) / 256), 256, 0, st>>>(n[q], row_ptr[q], part[q], eoff[q], pc.node[q],
                                                              pc.sub[q], pc.l2[q], rpu.p, partu.p);
      NS_LAUNCH_CHECK();
      k_cols_in_range<<<unsigned((nnz[q] + 255) / 256), 256, 0, st>>>(nnz[q], col_idx[q], n[q], bad.p);
      NS_LAUNCH_CHECK();
      k_shift_cols<<<unsigned((nnz[q] + 255) / 256), 256, 0, st>>>(nnz[q], col_idx[q], pc.node[q], colu.p + eoff[q]);
      NS_LAUNCH_CHECK();
      NS_HIP(hipMemcpyAsync(valu.p + eoff[q], val[q], nnz[q] * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    upload(rpu.p + nu, &nnzu, sizeof(int64_t), st);
    int hb = 0;
    read_back(*h, &hb, bad.p, 1);
    if (hb) fail(INVALID_ARG, "CSR structure invalid (row_ptr/col_idx out of range) in some problem");
    setup_core(h, nu, nnzu, rpu.p, colu.p, valu.p, partu.p, &pc, omega, info);
    *out = h;
    return NS_OK;
  } catch (const Error& e) {
    ns_status st = finish(h, e);
    destroy_handle(h);
    return st;
  }
}

ns_status nystrom_schur_apply(ns_handle h, const double* r_gamma, double* z_gamma, int32_t ncols) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    StreamScope ss(h->stream);
    if (ncols < 1 || ncols > 1024 || !r_gamma || !z_gamma) fail(INVALID_ARG, "bad apply arguments");
    DBuf<double> work, c1, c2;
    work.alloc(gram_work_elems(h->segG.view, std::max(h->k, ncols)));
    c1.alloc(size_t(std::max(h->k, 1)) * ncols * h->nprob);
    c2.alloc(size_t(std::max(h->k, 1)) * ncols * h->nprob);
    DBuf<double> gs;
    const SmallWs ws = small_ws(gs, h->nprob, std::max(h->s, 1), ncols);
    apply_prec(*h, r_gamma, ncols, z_gamma, ncols, ncols, work, c1, c2, ws);
    NS_HIP(hipStreamSynchronize(h->stream));
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_get_tuning(ns_handle h, int32_t* out) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    StreamScope ss(h->stream);
    if (!out) fail(INVALID_ARG, "out must not be NULL");
    const char* pi = h->bf16 ? "bf16" : (h->prec_inner ? "f32" : "f64");
    const int s = std::max(h->s, 1);
    out[0] = h->trsm_cols ? h->trsm_cols : tuned("trsm_cols", h->prec_inner ? "f32" : "f64", s, s <= 16 ? 16 : 32);
    out[1] = h->pcg_graph ? h->pcg_graph : tuned("pcg_graph_iters", "f64", h->nG, h->nprob > 1 ? 4 : 1);
    out[2] = h->bcg_graph ? h->bcg_graph : tuned("bcg_graph_iters", pi, h->nG, 2);
    out[3] = tuned("ls_gemm_cols", h->prec_inner ? "f32" : "f64", s, 80);
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_apply_noalloc(ns_handle h, const double* r_gamma, double* z_gamma, int32_t ncols) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    StreamScope ss(h->stream);
    if (ncols < 1 || ncols > 1024 || !r_gamma || !z_gamma) fail(INVALID_ARG, "bad apply arguments");
    if (h->sub) fail(INVALID_ARG, "nystrom_schur_apply_noalloc: not available with the recursive level");
    // the operator workspaces of the handle (made at setup for k + p columns, or by an earlier apply) must
    // already hold ncols columns: growing them would allocate
    if (ncols > h->ws_cols)
      fail(INVALID_ARG, "nystrom_schur_apply_noalloc: " + std::to_string(ncols) +
                            " columns exceed the handle's workspaces (" + std::to_string(h->ws_cols) + ")");
    const Seg& sg = h->segG.view;
    const int k = std::max(h->k, 1), np = h->nprob;
    const size_t nwork = round256(std::max<size_t>(size_t(sg.nchunk) * size_t(k) * size_t(ncols), 2 * sg.nchunk + 32));
    const size_t ncoef = round256(size_t(k) * ncols * np);
    const size_t stride = h->apply_mode == NS_APPLY_ADEF2 ? small_chol_scratch_elems(k, ncols) : 0;
    const size_t need = nwork + 2 * ncoef + round256(stride * size_t(np));
    if (need > kScratchDoubles)
      fail(INVALID_ARG, "nystrom_schur_apply_noalloc: needs " + std::to_string(need * sizeof(double)) +
                            " bytes of scratch, the limit is " + std::to_string(kScratchDoubles * sizeof(double)) +
                            " per device (fewer columns, or nystrom_schur_apply)");
    double* base = scratch_address();
    double* work = base;
    double* c1 = work + nwork;
    double* c2 = c1 + ncoef;
    SmallWs ws;
    ws.n = k;
    ws.c = ncols;
    ws.stride = int64_t(stride);
    ws.p = stride ? c2 + ncoef : nullptr;
    apply_prec(*h, r_gamma, ncols, z_gamma, ncols, ncols, work, c1, c2, ws);
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
    StreamScope ss(h->stream);
    if (!b || !x || maxit < 0 || !(rtol > 0.0)) fail(INVALID_ARG, "bad pcg_solve arguments");
    if (h->nprob != 1) fail(INVALID_ARG, "batched handle: use nystrom_schur_pcg_solve_batched");
    hipStream_t st = h->stream;
    Events ev(st);
    ev.rec(0);
    NS_HIP(hipMemsetAsync(h->dflags.p + 14, 0, sizeof(int), st));
    k_finite_check<<<unsigned((h->n + 255) / 256), 256, 0, st>>>(h->n, b, h->dflags.p + 14);
    NS_LAUNCH_CHECK();
    int bad = 0;
    read_back(*h, &bad, h->dflags.p + 14, 1);
    if (bad) fail(INVALID_ARG, "b contains NaN or Inf");
    std::vector<SolveOut> res;
    if (h->outer == NS_OUTER_FULL)
      pcg_full_core(*h, b, x, rtol, maxit, res);
    else
      pcg_core(*h, b, x, rtol, maxit, res);
    ev.rec(1);
    if (info) {
      info->it_pcg = res[0].it;
      info->converged = res[0].converged;
      info->relres_schur = res[0].relres_schur;
      info->relres_true = res[0].relres_true;
      info->t_solve = ev.sec(0, 1);
      if (info->res_hist && info->res_hist_cap > 0) {
        const size_t m = std::min<size_t>(res[0].hist.size(), size_t(info->res_hist_cap));
        std::memcpy(info->res_hist, res[0].hist.data(), m * sizeof(double));
      }
    }
    if (!res[0].converged) fail(NOT_CONVERGED, "PCG did not reach rtol within maxit iterations");
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_pcg_solve_batched(ns_handle h, const double* const* b, double* const* x, double rtol,
                                          int32_t maxit, ns_solve_info* info) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    StreamScope ss(h->stream);
    if (!b || !x || maxit < 0 || !(rtol > 0.0)) fail(INVALID_ARG, "bad pcg_solve_batched arguments");
    hipStream_t st = h->stream;
    const int np = h->nprob;
    Events ev(st);
    ev.rec(0);
    DBuf<double> bu, xu;
    bu.alloc(h->n);
    xu.alloc(h->n);
    for (int q = 0; q < np; ++q) {
      if (!b[q] || !x[q]) fail(INVALID_ARG, "NULL right-hand side or solution pointer");
      NS_HIP(hipMemcpyAsync(bu.p + h->h_noff[q], b[q], (h->h_noff[q + 1] - h->h_noff[q]) * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    }
    NS_HIP(hipMemsetAsync(h->dflags.p + 14, 0, sizeof(int), st));
    k_finite_check<<<unsigned((h->n + 255) / 256), 256, 0, st>>>(h->n, bu.p, h->dflags.p + 14);
    NS_LAUNCH_CHECK();
    int bad = 0;
    read_back(*h, &bad, h->dflags.p + 14, 1);
    if (bad) fail(INVALID_ARG, "b contains NaN or Inf");
    std::vector<SolveOut> res;
    if (h->outer == NS_OUTER_FULL)
      pcg_full_core(*h, bu.p, xu.p, rtol, maxit, res);
    else
      pcg_core(*h, bu.p, xu.p, rtol, maxit, res);
    for (int q = 0; q < np; ++q)
      NS_HIP(hipMemcpyAsync(x[q], xu.p + h->h_noff[q], (h->h_noff[q + 1] - h->h_noff[q]) * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    ev.rec(1);
    const double t = ev.sec(0, 1);
    bool all = true;
    for (int q = 0; q < np; ++q) {
      all = all && res[q].converged;
      if (!info) continue;
      info[q].it_pcg = res[q].it;
      info[q].converged = res[q].converged;
      info[q].relres_schur = res[q].relres_schur;
      info[q].relres_true = res[q].relres_true;
      info[q].t_solve = t;
      if (info[q].res_hist && info[q].res_hist_cap > 0) {
        const size_t m = std::min<size_t>(res[q].hist.size(), size_t(info[q].res_hist_cap));
        std::memcpy(info[q].res_hist, res[q].hist.data(), m * sizeof(double));
      }
    }
    if (!all) fail(NOT_CONVERGED, "PCG did not reach rtol within maxit iterations for some problem");
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

ns_status nystrom_schur_schur_apply(ns_handle h, const double* X, double* Y, int32_t ncols, int32_t prec) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    StreamScope ss(h->stream);
    if (ncols < 1 || ncols > 1024 || !X || !Y) fail(INVALID_ARG, "bad arguments");
    if (prec == NS_FP32 || prec == NS_BF16) {
      if (!h->prec_inner) fail(INVALID_ARG, "FP32 operators exist only with prec_inner = NS_FP32 or NS_BF16");
      if (prec == NS_BF16 && !h->bf16) fail(INVALID_ARG, "BF16 operators exist only with prec_inner = NS_BF16");
      BF16Scope b16(*h, prec == NS_BF16);
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
    StreamScope ss(h->stream);
    if (ncols < 1 || ncols > 1024 || !X || !Y) fail(INVALID_ARG, "bad arguments");
    if (prec == NS_FP32 || prec == NS_BF16) {
      if (!h->prec_inner) fail(INVALID_ARG, "FP32 operators exist only with prec_inner = NS_FP32 or NS_BF16");
      if (prec == NS_BF16 && !h->bf16) fail(INVALID_ARG, "BF16 operators exist only with prec_inner = NS_BF16");
      BF16Scope b16(*h, prec == NS_BF16);
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
    StreamScope ss(h->stream);
    if (ncols < 1 || ncols > 1024 || !X || !Y) fail(INVALID_ARG, "bad arguments");
    if (prec == NS_FP32) {
      if (!h->prec_inner) fail(INVALID_ARG, "FP32 operators exist only with prec_inner = NS_FP32 or NS_BF16");
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
    StreamScope ss(h->stream);
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
  out[7] = h->nprob;
  return NS_OK;
}

ns_status nystrom_schur_get_lowrank(ns_handle h, double* Z, double* Sigma) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    StreamScope ss(h->stream);
    if (h->nprob != 1) fail(INVALID_ARG, "batched handle: low-rank terms are per problem");
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

ns_status nystrom_schur_get_basis(ns_handle h, double* U, double* rho) {
  if (!h) return finish(nullptr, Error{INVALID_ARG, "NULL handle"});
  try {
    StreamScope ss(h->stream);
    if (h->nprob != 1) fail(INVALID_ARG, "batched handle: bases are per problem");
    if (rho) *rho = h->proposal_rho;
    if (U && h->k_eff > 0) {
      if (h->proposal_accepted || !h->U.p) fail(INVALID_ARG, "no Nystrom basis (the proposal was accepted)");
      NS_HIP(hipMemcpy2DAsync(U, h->k_eff * sizeof(double), h->U.p, h->k * sizeof(double), h->k_eff * sizeof(double),
                              h->nG, hipMemcpyDeviceToDevice, h->stream));
      NS_HIP(hipStreamSynchronize(h->stream));
    }
    return NS_OK;
  } catch (const Error& e) {
    return finish(h, e);
  }
}

void nystrom_schur_destroy(ns_handle h) { destroy_handle(h); }

const char* nystrom_schur_last_error(ns_handle h) {
  if (h) return h->last_error.c_str();
  return g_last_error.c_str();
}

}  // extern "C"
