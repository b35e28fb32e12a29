// Tall-skinny block-vector kernels over row segments: Gram products X^T Y
// with a deterministic two-stage reduction, block updates Out = beta Out +
// X M (+ X2 M2), column norms, dot products and the fused vector updates of
// PCG with per-problem scalars and done flags.
#include <type_traits>

#include "ns_vec.h"

namespace ns {
namespace {

constexpr int CHUNK_MAX = 256;   // reduction chunks per segment (at most): one per compute unit
constexpr int CHUNK_ROWS = 128;  // target rows per chunk

// index p of the segment whose range [pre[p], pre[p + 1]) holds b
__device__ __forceinline__ int seg_of(const int* __restrict__ pre, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// rows [r0, r1) of reduction chunk b; returns the segment
__device__ __forceinline__ int chunk_rows(const Seg& sg, int b, int64_t& r0, int64_t& r1) {
  const int p = seg_of(sg.coff, sg.n, b);
  const int c = b - sg.coff[p], nch = sg.coff[p + 1] - sg.coff[p];
  const int64_t a = sg.off[p], e = sg.off[p + 1];
  const int64_t per = (e - a + nch - 1) / nch;
  r0 = a + int64_t(c) * per;
  r1 = r0 + per < e ? r0 + per : e;
  return p;
}

typedef double gv4d __attribute__((ext_vector_type(4)));

// Gram partials with more parallelism: workgroup (chunk, strip) computes the 16-row strip a0 = 16 strip of the
// chunk's A^T B (all column tiles of B, at most GS_MAXT per launch column group); its four waves split the chunk's
// rows in 4-row MFMA steps (wave w takes steps w, w + 4, ...), reading the operands straight from global memory
// (the chunk is reused from cache by the strips), and the four partial strips are summed in a fixed order.
constexpr int GS_MAXT = 5;
template <class TA, class TB, int TMAX>
__global__ __launch_bounds__(256) void k_gram_strip(Seg sg, const TA* __restrict__ A, int64_t lda, int ra,
                                                    const TB* __restrict__ B, int64_t ldb, int rb,
                                                    double* __restrict__ part, int sym) {
  __shared__ double red[3][GS_MAXT][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int a0 = 16 * blockIdx.y;
  const int bt0 = GS_MAXT * blockIdx.z;                 // first column tile of this group
  // column tiles in this group; with sym (A = B) only those on or left of the diagonal, mirrored on output
  const int tb = min(min(GS_MAXT, (rb + 15) / 16 - bt0), sym ? int(blockIdx.y) - bt0 + 1 : GS_MAXT);
  if (tb <= 0) return;
  int64_t r0, r1;
  const int pseg = chunk_rows(sg, blockIdx.x, r0, r1);
  if (sg.skip && sg.skip[pseg]) return;
  gv4d acc[GS_MAXT];
#pragma unroll
  for (int t = 0; t < GS_MAXT; ++t) acc[t] = gv4d{0.0, 0.0, 0.0, 0.0};
  const int ac = a0 + li;                        // column of A this lane feeds
  const bool aok = ac < ra;
  const TA* Ap = A + (aok ? ac : 0);
  int bc[GS_MAXT];
  bool bok[GS_MAXT];
#pragma unroll
  for (int t = 0; t < GS_MAXT; ++t) {
    bc[t] = 16 * (bt0 + t) + li;
    bok[t] = t < tb && bc[t] < rb;
    if (!bok[t]) bc[t] = 0;
  }
  // U k-steps per batch: all their loads are issued (unconditionally, from clamped in-bounds addresses) before
  // the products, so they are in flight together; out-of-range values are replaced by zero afterwards
  constexpr int U = 4;
  for (int64_t k = r0 + 4 * w; k < r1; k += 16 * U) {
    double xv[U], yv[U][GS_MAXT];
    bool rok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = k + 16 * u + lk;
      rok[u] = r < r1;
      const int64_t rr = rok[u] ? r : r0;
      xv[u] = double(Ap[rr * lda]);
#pragma unroll
      for (int t = 0; t < TMAX; ++t) yv[u][t] = double(B[rr * ldb + bc[t]]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double x = (rok[u] && aok) ? xv[u] : 0.0;
#pragma unroll
      for (int t = 0; t < TMAX; ++t)
        if (t < tb) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, (rok[u] && bok[t]) ? yv[u][t] : 0.0, acc[t], 0, 0, 0);
    }
  }
  // fixed-order sum of the four waves' strips: waves 1..3 park theirs, wave 0 adds them in order
  if (w > 0) {
#pragma unroll
    for (int t = 0; t < GS_MAXT; ++t)
      if (t < tb)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[w - 1][t][v][lane] = acc[t][v];
  }
  __syncthreads();
  if (w != 0) return;
  const int nout = ra * rb;
  double* out = part + int64_t(blockIdx.x) * nout;
#pragma unroll
  for (int t = 0; t < GS_MAXT; ++t)
    if (t < tb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double sum = ((acc[t][v] + red[0][t][v][lane]) + red[1][t][v][lane]) + red[2][t][v][lane];
        const int a = a0 + 4 * v + lk, b = 16 * (bt0 + t) + li;
        if (a < ra && b < rb) {
          out[a * rb + b] = sum;
          if (sym && bt0 + t != int(blockIdx.y)) out[b * rb + a] = sum;
        }
      }
}

// Gram partials of wide blocks (32..160 columns each side), one workgroup per reduction chunk: every output
// tile of the chunk's A^T B (with A = B only the lower ones and the diagonal, mirrored on output) is owned by one
// of the 8 waves, and the chunk's rows pass through LDS GC_K at a time, double-buffered with the next stage's
// loads in flight during the products, so each chunk of A and B is read from memory once (the strip kernel
// above reads B once per output strip).  Each tile sums the chunk's rows in row order.
// A^T b for one column b (FP64): part[chunk][a].  1024-thread workgroups, one per reduction chunk; lane l of a
// wave owns the columns l + 64 g (g < CPL) of A and wave w the rows w, w + 16, ... of the chunk, GV_U of them
// per batch with all their loads issued (from clamped in-bounds rows) before the first product; the sixteen
// waves' sums are added in a fixed order.
constexpr int GV_NT = 1024, GV_U = 4;
template <int CPL>
__global__ __launch_bounds__(GV_NT) void k_gram_col(Seg sg, const double* __restrict__ A, int64_t lda, int ra,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    double* __restrict__ part) {
  __shared__ double red[GV_NT / 64][64 * CPL];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t r0, r1;
  const int pseg = chunk_rows(sg, blockIdx.x, r0, r1);
  if (sg.skip && sg.skip[pseg]) return;
  int cc[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) cc[g] = min(lane + 64 * g, ra - 1);
  double acc[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) acc[g] = 0.0;
  for (int64_t r = r0 + w; r < r1; r += (GV_NT / 64) * GV_U) {
    double av[GV_U][CPL], bv[GV_U];
#pragma unroll
    for (int u = 0; u < GV_U; ++u) {
      const int64_t rr = r + (GV_NT / 64) * u < r1 ? r + (GV_NT / 64) * u : r;
      bv[u] = B[rr * ldb];
#pragma unroll
      for (int g = 0; g < CPL; ++g) av[u][g] = A[rr * lda + cc[g]];
    }
#pragma unroll
    for (int u = 0; u < GV_U; ++u)
      if (r + (GV_NT / 64) * u < r1)  // uniform over the wave
#pragma unroll
        for (int g = 0; g < CPL; ++g) acc[g] += av[u][g] * bv[u];
  }
#pragma unroll
  for (int g = 0; g < CPL; ++g) red[w][64 * g + lane] = acc[g];
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * CPL; e += GV_NT) {
    if (e >= ra) continue;
    double sum = red[0][e];
#pragma unroll
    for (int x = 1; x < GV_NT / 64; ++x) sum += red[x][e];
    part[int64_t(blockIdx.x) * ra + e] = sum;
  }
}

constexpr int GC_MAXC = 160;
constexpr int GC_K = 16;
constexpr int GC_LD = GC_MAXC + 4;  // LDS row stride (bank spread between the four rows of a k-step)
// NT threads, MT output tiles per wave: 512 threads with 13 tiles (256 registers a wave) for every tile of a
// product of up to 10 x 10 tiles, 1024 threads (4 waves per SIMD: while one waits for its fragments the others
// multiply) with 2 or 4 tiles for the lower triangles (55 tiles at 160 columns).  The products run
// unconditionally (a wave's spare slots multiply tile (0, 0) and are not stored): a per-tile branch would make
// every product wait for its own fragment reads.
template <class TA, class TB, int MT, int NT>
__global__ __launch_bounds__(NT) void k_gram_chunk(Seg sg, const TA* __restrict__ A, int64_t lda, int ra,
                                                     const TB* __restrict__ B, int64_t ldb, int rb,
                                                     double* __restrict__ part, int mode) {
  // mode 0: every tile of A^T B; 1: A = B, the lower tiles, mirrored; 2: the lower tiles of A^T B, mirrored
  // (a product known to be symmetric)
  const bool same = mode == 1, lower = mode != 0;
  constexpr int PL = (GC_K * GC_MAXC + NT - 1) / NT;  // staged values per thread and matrix
  __shared__ double sA[2][GC_K * GC_LD];
  __shared__ double sB[2][GC_K * GC_LD];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int li = lane & 15, lk = lane >> 4;
  int64_t r0, r1;
  const int pseg = chunk_rows(sg, blockIdx.x, r0, r1);
  if (sg.skip && sg.skip[pseg]) return;
  if (r0 >= r1) {  // a chunk without rows contributes zeros
    for (int o = threadIdx.x; o < ra * rb; o += NT) part[int64_t(blockIdx.x) * ra * rb + o] = 0.0;
    return;
  }
  const int ta = (ra + 15) / 16, tbn = (rb + 15) / 16;
  const int ntile = lower ? ta * (ta + 1) / 2 : ta * tbn;
  const int wa = 16 * ta, wb = 16 * tbn;  // staged columns (zero past ra, rb)
  int tA[MT], tB[MT];
  bool has[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int t = w + (NT / 64) * m;
    has[m] = t < ntile;
    int i = 0, j = 0;
    if (has[m]) {
      if (lower) {
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        j = t - i * (i + 1) / 2;
      } else {
        i = t / tbn;
        j = t - i * tbn;
      }
    }
    tA[m] = i;
    tB[m] = j;
  }
  gv4d acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = gv4d{0.0, 0.0, 0.0, 0.0};
  double xa[PL], xb[PL];
  auto load = [&](int64_t k0) {  // clamped, in-bounds addresses; out-of-range values are zeroed in store
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int e = threadIdx.x + NT * q;
      const int ea = min(e, GC_K * wa - 1), eb = min(e, GC_K * wb - 1);
      const int64_t rowa = min(k0 + ea / wa, r1 - 1), rowb = min(k0 + eb / wb, r1 - 1);
      xa[q] = double(A[rowa * lda + min(ea % wa, ra - 1)]);
      if (!same) xb[q] = double(B[rowb * ldb + min(eb % wb, rb - 1)]);
    }
  };
  auto store = [&](int64_t k0, int buf) {
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int e = threadIdx.x + NT * q;
      if (e < GC_K * wa) {
        const int r = e / wa, c = e % wa;
        sA[buf][r * GC_LD + c] = (k0 + r < r1 && c < ra) ? xa[q] : 0.0;
      }
      if (!same && e < GC_K * wb) {
        const int r = e / wb, c = e % wb;
        sB[buf][r * GC_LD + c] = (k0 + r < r1 && c < rb) ? xb[q] : 0.0;
      }
    }
  };
  load(r0);
  int buf = 0;
  for (int64_t k0 = r0; k0 < r1; k0 += GC_K, buf ^= 1) {
    store(k0, buf);
    __syncthreads();
    if (k0 + GC_K < r1) load(k0 + GC_K);
    const double* a_ = sA[buf];
    const double* b_ = same ? sA[buf] : sB[buf];
#pragma unroll
    for (int kk = 0; kk < GC_K; kk += 4) {
      const int ro = (kk + lk) * GC_LD + li;
#pragma unroll
      for (int m = 0; m < MT; ++m)
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_[ro + 16 * tA[m]], b_[ro + 16 * tB[m]], acc[m], 0, 0, 0);
    }
  }
  const int nout = ra * rb;
  double* out = part + int64_t(blockIdx.x) * nout;
#pragma unroll
  for (int m = 0; m < MT; ++m)
    if (has[m])
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * tA[m] + 4 * v + lk, b = 16 * tB[m] + li;
        if (a < ra && b < rb) {
          out[a * rb + b] = acc[m][v];
          if (lower && tA[m] != tB[m]) out[b * rb + a] = acc[m][v];
        }
      }
}

// The same products for FP64 blocks of exactly W = 16 TW columns stored with leading dimension W (the block-CG
// vectors): a GC_K-row stage of each operand is one contiguous run (loads without index arithmetic; rows past
// the chunk are zeroed when staged), and the fragment offsets within a stage are compile-time.
// NT = 1024 threads, MT tiles per wave, tile t = w + 16 m as in k_gram_chunk.
template <int TW, int MT>
__global__ __launch_bounds__(1024) void k_gram_tw(Seg sg, const double* __restrict__ A,
                                                 const double* __restrict__ B, double* __restrict__ part, int mode) {
  constexpr int NT = 1024, NW = NT / 64, W = 16 * TW, SE = GC_K * W, PL = (SE + NT - 1) / NT;
  constexpr int LD = W + 4;  // LDS row stride (W is a multiple of the bank count: the four rows of a fragment
                             // read would share banks)
  const bool same = mode == 1, lower = mode != 0;
  __shared__ double sA[2][GC_K * LD];
  __shared__ double sB[2][GC_K * LD];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int li = lane & 15, lk = lane >> 4;
  int64_t r0, r1;
  const int pseg = chunk_rows(sg, blockIdx.x, r0, r1);
  if (sg.skip && sg.skip[pseg]) return;
  if (r0 >= r1) {  // a chunk without rows contributes zeros
    for (int o = threadIdx.x; o < W * W; o += NT) part[int64_t(blockIdx.x) * W * W + o] = 0.0;
    return;
  }
  const int ntile = lower ? TW * (TW + 1) / 2 : TW * TW;
  int tA[MT], tB[MT];
  bool has[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int t = w + NW * m;
    has[m] = t < ntile;
    int i = 0, j = 0;
    if (has[m]) {
      if (lower) {
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        j = t - i * (i + 1) / 2;
      } else {
        i = t / TW;
        j = t - i * TW;
      }
    }
    tA[m] = 16 * i;
    tB[m] = 16 * j;
  }
  gv4d acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = gv4d{0.0, 0.0, 0.0, 0.0};
  double xa[PL], xb[PL];
  auto load = [&](int64_t k0) {  // elements past the chunk's last row read that row's last element (in bounds)
    const int lim = int(min(int64_t(GC_K), r1 - k0)) * W - 1;
    const double* a = A + k0 * W;
    const double* b = B + k0 * W;
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int e = min(int(threadIdx.x) + NT * q, lim);
      xa[q] = a[e];
      if (!same) xb[q] = b[e];
    }
  };
  auto store = [&](int64_t k0, int buf) {
    const int lim = int(min(int64_t(GC_K), r1 - k0)) * W;
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      const int e = threadIdx.x + NT * q;
      if (SE % NT == 0 || e < SE) {
        const int o = (e / W) * LD + e % W;
        sA[buf][o] = e < lim ? xa[q] : 0.0;
        if (!same) sB[buf][o] = e < lim ? xb[q] : 0.0;
      }
    }
  };
  load(r0);
  int buf = 0;
  for (int64_t k0 = r0; k0 < r1; k0 += GC_K, buf ^= 1) {
    store(k0, buf);
    __syncthreads();
    if (k0 + GC_K < r1) load(k0 + GC_K);
    const double* a_ = sA[buf] + lk * LD + li;
    const double* b_ = (same ? sA[buf] : sB[buf]) + lk * LD + li;
#pragma unroll
    for (int kk = 0; kk < GC_K; kk += 4) {
#pragma unroll
      for (int m = 0; m < MT; ++m)
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_[kk * LD + tA[m]], b_[kk * LD + tB[m]], acc[m], 0, 0, 0);
      if constexpr (MT > 4) __builtin_amdgcn_sched_barrier(0);  // one K step's fragments live at a time
    }
  }
  double* out = part + int64_t(blockIdx.x) * W * W;
#pragma unroll
  for (int m = 0; m < MT; ++m)
    if (has[m])
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = tA[m] + 4 * v + lk, b = tB[m] + li;
        out[a * W + b] = acc[m][v];
        if (lower && tA[m] != tB[m]) out[b * W + a] = acc[m][v];
      }
}

// G_p[o] = alpha * (sum of segment p's chunk partials of output o) + beta * G_p[o].  TX outputs per block;
// the TY = 1024 / TX threads of an output take the chunks c = ty, ty + TY, ... and a fixed tree combines them.
// With split > 1 every chunk c left split consecutive partials (chunk c's rows in split parts).
template <int TX>
__global__ __launch_bounds__(1024) void k_seg_final(Seg sg, int nout, const double* __restrict__ part,
                                                    double* __restrict__ G, int64_t gstride, double alpha,
                                                    double beta, const double* __restrict__ rscale = nullptr,
                                                    int64_t rsstride = 0, int rb = 1, int split = 1) {
  constexpr int TY = 1024 / TX;
  __shared__ double red[1024];
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int o = blockIdx.x * TX + tx;
  const int p = blockIdx.y;
  if (sg.skip && sg.skip[p]) return;
  const int c0 = sg.coff[p] * split, nch = (sg.coff[p + 1] - sg.coff[p]) * split;
  double s = 0.0;
  if (o < nout)
    for (int c = ty; c < nch; c += TY) s += part[int64_t(c0 + c) * nout + o];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = TY / 2; h > 0; h >>= 1) {
    if (ty < h) red[threadIdx.x] += red[threadIdx.x + h * TX];
    __syncthreads();
  }
  if (ty == 0 && o < nout) {
    double* g = G + int64_t(p) * gstride + o;
    const double a = rscale ? alpha * rscale[int64_t(p) * rsstride + o / rb] : alpha;  // output row o / rb
    *g = a * red[tx] + (beta != 0.0 ? beta * *g : 0.0);
  }
}

void seg_final(const Seg& sg, int nout, const double* part, double* G, int64_t gstride, double alpha, double beta,
               hipStream_t st, const double* rscale = nullptr, int64_t rsstride = 0, int rb = 1, int split = 1) {
  if (nout >= 16) {
    k_seg_final<64><<<dim3((nout + 63) / 64, sg.n), 1024, 0, st>>>(sg, nout, part, G, gstride, alpha, beta, rscale,
                                                                  rsstride, rb, split);
  } else {
    k_seg_final<1><<<dim3(nout, sg.n), 1024, 0, st>>>(sg, nout, part, G, gstride, alpha, beta, rscale, rsstride,
                                                     rb, split);
  }
  NS_LAUNCH_CHECK();
}

// Out[r, c] = beta * Out[r, c] + gamma * sum_m X[r, m] M_p[m, c] on 64-row tiles that never straddle two
// segments, on FP64 MFMA 16x16x4 (FP32 blocks are widened, so the products and sums are those of FP64).  A
// workgroup computes a 64 x 16 NTI output block (wave w: rows 16 w .. 16 w + 15, NTI column tiles); X and M are
// staged through LDS in batches of TS_K rows of M.
constexpr int TS_K = 32;
// Out[r][c] = X[r][c] for the rows [rbase, min(rbase + 64, rend)) and columns [c0, c1) (a skipped segment of a
// block update), 256 threads.
template <class T>
__device__ __forceinline__ void ts_copy_tile(int64_t rbase, int64_t rend, int c0, int c1, T* Out, int64_t ldo,
                                             const T* X, int64_t ldx) {
  const int nc = c1 - c0;
  if (nc <= 0 || (static_cast<const T*>(Out) == X && ldo == ldx)) return;  // in place: nothing to copy
  const int64_t nr = rend - rbase < 64 ? rend - rbase : 64;
  for (int e = threadIdx.x; e < nr * nc; e += 256) {
    const int64_t r = rbase + e / nc;
    const int c = c0 + e % nc;
    Out[r * ldo + c] = X[r * ldx + c];
  }
}

template <class T, int NTI>
__global__ __launch_bounds__(256) void k_ts_mfma(Seg sg, int ncols, T* Out, int64_t ldo, double beta,
                                                 double gamma, const T* X, int64_t ldx, int K,
                                                 const double* __restrict__ M, int64_t ldm, int64_t mstride) {
  constexpr int NC = 16 * NTI;
  __shared__ double sX[64 * (TS_K + 1)];
  __shared__ double sM[TS_K * (NC + 1)];
  const int p = seg_of(sg.toff, sg.n, blockIdx.x);
  const int64_t rbase = sg.off[p] + int64_t(blockIdx.x - sg.toff[p]) * 64;
  const int64_t rend = sg.off[p + 1];
  const double* Mp = M + int64_t(p) * mstride;
  const int c0 = blockIdx.y * NC;
  if (sg.skip && sg.skip[p]) {  // Out = X on this tile's rows and column group
    ts_copy_tile(rbase, rend, c0, min(c0 + NC, ncols), Out, ldo, X, ldx);
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  gv4d acc[NTI];
#pragma unroll
  for (int t = 0; t < NTI; ++t) acc[t] = gv4d{0.0, 0.0, 0.0, 0.0};
  // the old output values (beta != 0) are loaded first, from clamped in-bounds addresses, so their loads are in
  // flight during the products instead of one after another in the epilogue
  T ov[NTI][4];
  if (beta != 0.0) {
#pragma unroll
    for (int t = 0; t < NTI; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = min(rbase + 16 * w + 4 * v + lk, rend - 1);
        const int c = min(c0 + 16 * t + li, ncols - 1);
        ov[t][v] = Out[r * ldo + c];
      }
  }
  constexpr int PX = 64 * TS_K / 256, PM = (TS_K * NC + 255) / 256;
  for (int k0 = 0; k0 < K; k0 += TS_K) {
    // every load of the batch is issued (in-bounds addresses) before the LDS stores, zero outside
    T xv[PX];
    double mv[PM];
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / TS_K, k = k0 + e % TS_K;
      const int64_t row = rbase + r;
      const bool ok = row < rend && k < K;
      xv[q] = X[(ok ? row : rbase) * ldx + (ok ? k : 0)];
    }
#pragma unroll
    for (int q = 0; q < PM; ++q) {
      const int e = threadIdx.x + 256 * q, c = c0 + e % NC, k = k0 + e / NC;
      const bool ok = e < TS_K * NC && c < ncols && k < K;
      mv[q] = Mp[int64_t(ok ? k : 0) * ldm + (ok ? c : 0)];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / TS_K, kk = e % TS_K;
      const bool ok = rbase + r < rend && k0 + kk < K;
      sX[r * (TS_K + 1) + kk] = ok ? double(xv[q]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PM; ++q) {
      const int e = threadIdx.x + 256 * q, cc = e % NC, kk = e / NC;
      const bool ok = c0 + cc < ncols && k0 + kk < K;
      if (e < TS_K * NC) sM[kk * (NC + 1) + cc] = ok ? mv[q] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TS_K; kk += 4) {
      const double a = sX[(16 * w + li) * (TS_K + 1) + kk + lk];
#pragma unroll
      for (int t = 0; t < NTI; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sM[(kk + lk) * (NC + 1) + 16 * t + li], acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NTI; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = rbase + 16 * w + 4 * v + lk;
      const int c = c0 + 16 * t + li;
      if (r < rend && c < ncols) {
        double y = gamma * acc[t][v];
        if (beta != 0.0) y += beta * double(ov[t][v]);
        Out[r * ldo + c] = T(y);
      }
    }
}

// The same product for wide blocks (more than 80 columns): one workgroup computes all NTI column tiles of its
// 64 rows, so X is read once and no column tile is computed twice; K is staged in batches of 16 rows of M,
// double-buffered in LDS with the next batch's global loads in flight during the current batch's products (one
// barrier per batch).  The sums over K run in the same order as in k_ts_mfma (same bits).
constexpr int TW_K = 16;
template <class T, int NTI>
__global__ __launch_bounds__(256, 2) void k_ts_wide(Seg sg, int ncols, T* Out, int64_t ldo, double beta,
                                                 double gamma, const T* X, int64_t ldx, int K,
                                                 const double* __restrict__ M, int64_t ldm, int64_t mstride) {
  constexpr int NC = 16 * NTI;
  constexpr int XS = TW_K + 1, MS = NC + 1;
  __shared__ double sX[2][64 * XS];
  __shared__ double sM[2][TW_K * MS];
  const int p = seg_of(sg.toff, sg.n, blockIdx.x);
  const int64_t rbase = sg.off[p] + int64_t(blockIdx.x - sg.toff[p]) * 64;
  const int64_t rend = sg.off[p + 1];
  const double* Mp = M + int64_t(p) * mstride;
  if (sg.skip && sg.skip[p]) {  // Out = X on this tile's rows
    ts_copy_tile(rbase, rend, 0, ncols, Out, ldo, X, ldx);
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  gv4d acc[NTI];
#pragma unroll
  for (int t = 0; t < NTI; ++t) acc[t] = gv4d{0.0, 0.0, 0.0, 0.0};
  constexpr int PX = 64 * TW_K / 256, PM = (TW_K * NC + 255) / 256;
  T xv[PX];
  double mv[PM];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / TW_K, k = k0 + e % TW_K;
      const int64_t row = rbase + r;
      const bool ok = row < rend && k < K;
      xv[q] = X[(ok ? row : rbase) * ldx + (ok ? k : 0)];
    }
#pragma unroll
    for (int q = 0; q < PM; ++q) {
      const int e = threadIdx.x + 256 * q, c = e % NC, k = k0 + e / NC;
      const bool ok = e < TW_K * NC && c < ncols && k < K;
      mv[q] = Mp[int64_t(ok ? k : 0) * ldm + (ok ? c : 0)];
    }
  };
  auto store = [&](int k0, int buf) {
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / TW_K, kk = e % TW_K;
      const bool ok = rbase + r < rend && k0 + kk < K;
      sX[buf][r * XS + kk] = ok ? double(xv[q]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PM; ++q) {
      const int e = threadIdx.x + 256 * q, cc = e % NC, kk = e / NC;
      const bool ok = cc < ncols && k0 + kk < K;
      if (e < TW_K * NC) sM[buf][kk * MS + cc] = ok ? mv[q] : 0.0;
    }
  };
  load(0);
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += TW_K, buf ^= 1) {
    store(k0, buf);
    __syncthreads();
    if (k0 + TW_K < K) load(k0 + TW_K);
    const double* xs = sX[buf];
    const double* ms = sM[buf];
#pragma unroll
    for (int kk = 0; kk < TW_K; kk += 4) {
      const double a = xs[(16 * w + li) * XS + kk + lk];
#pragma unroll
      for (int t = 0; t < NTI; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, ms[(kk + lk) * MS + 16 * t + li], acc[t], 0, 0, 0);
    }
  }
  // epilogue four column tiles at a time: their old outputs (beta != 0) loaded together from clamped in-bounds
  // positions before the first store
#pragma unroll
  for (int t0 = 0; t0 < NTI; t0 += 4) {
    T o[4][4];
    if (beta != 0.0) {
#pragma unroll
      for (int t = t0; t < t0 + 4 && t < NTI; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = rbase + 16 * w + 4 * v + lk;
          const int c = 16 * t + li;
          o[t - t0][v] = Out[(r < rend ? r : rend - 1) * ldo + (c < ncols ? c : ncols - 1)];
        }
    }
#pragma unroll
    for (int t = t0; t < t0 + 4 && t < NTI; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = rbase + 16 * w + 4 * v + lk;
        const int c = 16 * t + li;
        if (r < rend && c < ncols) {
          double y = gamma * acc[t][v];
          if (beta != 0.0) y += beta * double(o[t - t0][v]);
          Out[r * ldo + c] = T(y);
        }
      }
  }
}

// Block updates of one problem's wide FP64 blocks (6..10 column tiles): 256-row workgroups of 8 waves, each wave
// two 16-row tiles across every column tile (80 accumulators); X and M pass through LDS TB_K values of K at a
// time, double-buffered with the next stage's loads in flight, so each M stage serves 256 rows (four times the
// rows of k_ts_wide) and each SIMD has two waves of products to cover the loads.  The sums over K run in the
// same order as in k_ts_mfma (same bits).
constexpr int TB_R = 256, TB_NT = 512, TB_K = 16;
template <int NTI>
__global__ __launch_bounds__(TB_NT) void k_ts_big(int64_t r0, int64_t rend, const int* skip, int ncols,
                                                  double* Out, int64_t ldo, double beta, double gamma,
                                                  const double* X, int64_t ldx, int K,
                                                  const double* __restrict__ M, int64_t ldm) {
  constexpr int NC = 16 * NTI;
  constexpr int XS = TB_K + 1, MS = NC + 1;
  __shared__ double sX[2][TB_R * XS];
  __shared__ double sM[2][TB_K * MS];
  const int64_t rbase = r0 + int64_t(blockIdx.x) * TB_R;
  if (skip && skip[0]) {  // Out = X on this workgroup's rows (a skipped segment; nothing to do in place)
    if (static_cast<const double*>(Out) == X && ldo == ldx) return;
    const int64_t nr = rend - rbase < TB_R ? rend - rbase : TB_R;
    for (int64_t e = threadIdx.x; e < nr * ncols; e += TB_NT) {
      const int64_t r = rbase + e / ncols;
      const int c = int(e % ncols);
      Out[r * ldo + c] = X[r * ldx + c];
    }
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  gv4d acc[2][NTI];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < NTI; ++t) acc[h][t] = gv4d{0.0, 0.0, 0.0, 0.0};
  constexpr int PX = TB_R * TB_K / TB_NT, PM = (TB_K * NC + TB_NT - 1) / TB_NT;
  double xv[PX], mv[PM];
  // 32-bit offsets from the workgroup's first row (its 256 rows span less than 2^31 elements)
  const double* Xw = X + rbase * ldx;
  const int rlast = int(min(int64_t(TB_R), rend - rbase)) - 1, ldx32 = int(ldx), ldm32 = int(ldm);
  auto load = [&](int k0) {  // clamped, in-bounds addresses; out-of-range values zeroed in store
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int e = threadIdx.x + TB_NT * q, r = min(e / TB_K, rlast), k = min(k0 + e % TB_K, K - 1);
      xv[q] = Xw[r * ldx32 + k];
    }
#pragma unroll
    for (int q = 0; q < PM; ++q) {
      const int e = min(threadIdx.x + TB_NT * q, TB_K * NC - 1), c = min(e % NC, ncols - 1);
      const int k = min(k0 + e / NC, K - 1);
      mv[q] = M[k * ldm32 + c];
    }
  };
  auto store = [&](int k0, int buf) {
#pragma unroll
    for (int q = 0; q < PX; ++q) {
      const int e = threadIdx.x + TB_NT * q, r = e / TB_K, kk = e % TB_K;
      sX[buf][r * XS + kk] = (rbase + r < rend && k0 + kk < K) ? xv[q] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PM; ++q) {
      const int e = threadIdx.x + TB_NT * q, c = e % NC, kk = e / NC;
      if (e < TB_K * NC) sM[buf][kk * MS + c] = (c < ncols && k0 + kk < K) ? mv[q] : 0.0;
    }
  };
  load(0);
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += TB_K, buf ^= 1) {
    store(k0, buf);
    __syncthreads();
    if (k0 + TB_K < K) load(k0 + TB_K);
    const double* xs = sX[buf];
    const double* ms = sM[buf];
#pragma unroll
    for (int kk = 0; kk < TB_K; kk += 4) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double a = xs[(32 * w + 16 * h + li) * XS + kk + lk];
#pragma unroll
        for (int t = 0; t < NTI; ++t)
          acc[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, ms[(kk + lk) * MS + 16 * t + li], acc[h][t], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);  // one k-step's operands at a time (80 accumulators stay in registers)
    }
  }
  // epilogue two column tiles at a time: their sixteen old outputs (beta != 0) are loaded together, from clamped
  // in-bounds positions, before the first store (one memory round trip per pair instead of one per value)
#pragma unroll
  for (int t0 = 0; t0 < NTI; t0 += 2) {
    double o[2][2][4];
    if (beta != 0.0) {
#pragma unroll
      for (int t = t0; t < t0 + 2 && t < NTI; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = rbase + 32 * w + 16 * h + 4 * v + lk;
            const int c = 16 * t + li;
            o[t - t0][h][v] = Out[(r < rend ? r : rend - 1) * ldo + (c < ncols ? c : ncols - 1)];
          }
    }
#pragma unroll
    for (int t = t0; t < t0 + 2 && t < NTI; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = rbase + 32 * w + 16 * h + 4 * v + lk;
          const int c = 16 * t + li;
          if (r < rend && c < ncols) {
            double y = gamma * acc[h][t][v];
            if (beta != 0.0) y += beta * o[t - t0][h][v];
            Out[r * ldo + c] = y;
          }
        }
  }
}

// One output column, FP64: Out[r] = beta Out[r] + gamma sum_m X[r, m] M_p[m] for K <= 16 KPL.  A workgroup
// takes a 64-row tile (never straddling two segments); sixteen lanes share a row, lane l holding the columns
// l + 16 i of it (a 128-byte run per i over the sixteen lanes), and all 4 KPL row loads of a lane are issued
// before the products; the sixteen partial sums meet in a butterfly.
template <int KPL>
__global__ __launch_bounds__(256) void k_ts_gemv(Seg sg, double* Out, int64_t ldo, double beta,
                                                 double gamma, const double* X, int64_t ldx, int K,
                                                 const double* __restrict__ M, int64_t ldm, int64_t mstride) {
  const int p = seg_of(sg.toff, sg.n, blockIdx.x);
  const int64_t rbase = sg.off[p] + int64_t(blockIdx.x - sg.toff[p]) * 64, rend = sg.off[p + 1];
  const int l16 = threadIdx.x & 15, grp = threadIdx.x >> 4;
  if (sg.skip && sg.skip[p]) {  // Out = X on this tile's rows (a skipped segment)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = rbase + 16 * u + grp;
      if (l16 == 0 && r < rend) Out[r * ldo] = X[r * ldx];
    }
    return;
  }
  const double* Mp = M + int64_t(p) * mstride;
  double mv[KPL];
#pragma unroll
  for (int i = 0; i < KPL; ++i) {
    const int k = l16 + 16 * i;
    const double m = Mp[int64_t(min(k, K - 1)) * ldm];
    mv[i] = k < K ? m : 0.0;  // the clamped duplicate columns below meet a zero
  }
  double xv[4][KPL];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = rbase + 16 * u + grp, rr = r < rend ? r : rbase;
#pragma unroll
    for (int i = 0; i < KPL; ++i) xv[u][i] = X[rr * ldx + min(l16 + 16 * i, K - 1)];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < KPL; ++i) s += xv[u][i] * mv[i];
    s += __shfl_xor(s, 8, 16);
    s += __shfl_xor(s, 4, 16);
    s += __shfl_xor(s, 2, 16);
    s += __shfl_xor(s, 1, 16);
    const int64_t r = rbase + 16 * u + grp;
    if (l16 == 0 && r < rend) {
      double y = gamma * s;
      if (beta != 0.0) y += beta * Out[r * ldo];
      Out[r * ldo] = y;
    }
  }
}

template <class T>
void ts_launch(const Seg& sg, int ncols, T* Out, int64_t ldo, double beta, double gamma, const T* X, int64_t ldx,
               int K, const double* M, int64_t ldm, int64_t mstride, hipStream_t st) {
  const int tiles = (ncols + 15) / 16;
  auto go = [&](auto nti) {
    constexpr int N = decltype(nti)::value;
    dim3 g(unsigned(sg.ntile), unsigned((tiles + N - 1) / N));
    k_ts_mfma<T, N><<<g, 256, 0, st>>>(sg, ncols, Out, ldo, beta, gamma, X, ldx, K, M, ldm, mstride);
  };
  auto wide = [&](auto nti) {
    constexpr int N = decltype(nti)::value;
    k_ts_wide<T, N><<<unsigned(sg.ntile), 256, 0, st>>>(sg, ncols, Out, ldo, beta, gamma, X, ldx, K, M, ldm, mstride);
  };
  if constexpr (sizeof(T) == 8) {
    if (ncols == 1 && K >= 16 && K <= 256) {  // one column (the deflation product Z c of the outer iteration)
      auto gemv = [&](auto kpl) {
        constexpr int KPL = decltype(kpl)::value;
        k_ts_gemv<KPL><<<unsigned(sg.ntile), 256, 0, st>>>(sg, Out, ldo, beta, gamma, X, ldx, K, M, ldm, mstride);
      };
      switch ((K + 31) / 32) {
        case 1: gemv(std::integral_constant<int, 2>()); break;
        case 2: gemv(std::integral_constant<int, 4>()); break;
        case 3: gemv(std::integral_constant<int, 6>()); break;
        case 4: gemv(std::integral_constant<int, 8>()); break;
        case 5: gemv(std::integral_constant<int, 10>()); break;
        case 6: gemv(std::integral_constant<int, 12>()); break;
        case 7: gemv(std::integral_constant<int, 14>()); break;
        default: gemv(std::integral_constant<int, 16>()); break;
      }
      NS_LAUNCH_CHECK();
      return;
    }
    if (sg.n == 1 && tiles > 5 && tiles <= 10 && sg.rows > sg.first) {  // one problem's wide FP64 block
      auto big = [&](auto nti) {
        constexpr int N = decltype(nti)::value;
        k_ts_big<N><<<unsigned((sg.rows - sg.first + TB_R - 1) / TB_R), TB_NT, 0, st>>>(
            sg.first, sg.rows, sg.skip, ncols, Out, ldo, beta, gamma, X, ldx, K, M, ldm);
      };
      switch (tiles) {
        case 6: big(std::integral_constant<int, 6>()); break;
        case 7: big(std::integral_constant<int, 7>()); break;
        case 8: big(std::integral_constant<int, 8>()); break;
        case 9: big(std::integral_constant<int, 9>()); break;
        default: big(std::integral_constant<int, 10>()); break;
      }
      NS_LAUNCH_CHECK();
      return;
    }
  }
  if (tiles > 5 && tiles <= 16) {
    switch (tiles) {
      case 6: wide(std::integral_constant<int, 6>()); break;
      case 7: wide(std::integral_constant<int, 7>()); break;
      case 8: wide(std::integral_constant<int, 8>()); break;
      case 9: wide(std::integral_constant<int, 9>()); break;
      case 10: wide(std::integral_constant<int, 10>()); break;
      case 11: wide(std::integral_constant<int, 11>()); break;
      case 12: wide(std::integral_constant<int, 12>()); break;
      case 13: wide(std::integral_constant<int, 13>()); break;
      case 14: wide(std::integral_constant<int, 14>()); break;
      case 15: wide(std::integral_constant<int, 15>()); break;
      default: wide(std::integral_constant<int, 16>()); break;
    }
    NS_LAUNCH_CHECK();
    return;
  }
  if (tiles > 16 && static_cast<const T*>(Out) == X)
    fail(INVALID_ARG, "block update in place wider than 256 columns");  // column groups would race
  if (tiles <= 1)
    go(std::integral_constant<int, 1>());
  else if (tiles <= 2)
    go(std::integral_constant<int, 2>());
  else if (tiles <= 3)
    go(std::integral_constant<int, 3>());
  else if (tiles <= 4)
    go(std::integral_constant<int, 4>());
  else if (tiles <= 5)
    go(std::integral_constant<int, 5>());
  else
    go(std::integral_constant<int, 8>());
  NS_LAUNCH_CHECK();
}

template <class T, class U>
__global__ void k_convert(int64_t n, int ncols, const T* __restrict__ X, int64_t ldx, U* __restrict__ Y, int64_t ldy) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t r = idx / ncols;
  const int c = int(idx % ncols);
  Y[r * ldy + c] = U(X[r * ldx + c]);
}

__device__ __forceinline__ double block_sum256(double s, double* red) {
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

// Sum over the 256 threads in a fixed order: butterfly within each wave, then the four wave sums.
__device__ __forceinline__ double block_sum256_w(double s, double* red4) {
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = s;
  __syncthreads();
  return (red4[0] + red4[1]) + (red4[2] + red4[3]);
}

// Sum of problem g's chunk partials part[coff[g] ..] (the same value in every block that asks).
__device__ __forceinline__ double seg_total(const Seg& sg, int g, const double* __restrict__ part, double* red4) {
  const int c0 = sg.coff[g], nch = sg.coff[g + 1] - c0;
  double s = 0.0;
  for (int c = threadIdx.x; c < nch; c += 256) s += part[c0 + c];
  return block_sum256_w(s, red4);
}

__global__ __launch_bounds__(256) void k_dot_partial(Seg sg, const double* __restrict__ x,
                                                     const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[256];
  int64_t r0, r1;
  chunk_rows(sg, blockIdx.x, r0, r1);
  double s = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) s += x[i] * y[i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// PCG: (p^T q)_g from the chunk partials pq_part of problem g (formed again by every block of g, in one fixed
// order), then w += alpha p, r -= alpha q on the chunk's rows unless its problem is done; partial ||r||^2.
__global__ __launch_bounds__(256) void k_pcg_wr(Seg sg, PcgState S, double* __restrict__ w, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                const double* __restrict__ pq_part, double* __restrict__ part) {
  __shared__ double red[256];
  __shared__ double red4[4];
  int64_t r0, r1;
  const int g = chunk_rows(sg, blockIdx.x, r0, r1);
  const double pq = seg_total(sg, g, pq_part, red4);
  double s = 0.0;
  if (!S.done[g] && *S.j < S.maxit) {
    double* ps = S.ps + int64_t(g) * PS;
    if (threadIdx.x == 0 && blockIdx.x == sg.coff[g]) ps[PS_PQ] = pq;
    const double alpha = ps[PS_RHO] / pq;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
      w[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      s += ri * ri;
    }
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ||r||^2 per problem from the chunk partials (one block per problem, fixed summation order), then the
// stopping test of iteration j.
__global__ __launch_bounds__(256) void k_pcg_check(Seg sg, PcgState S, const double* __restrict__ part) {
  __shared__ double red[256];
  const int g = blockIdx.x;
  const int j = *S.j;
  if (S.done[g] || j >= S.maxit) return;
  const int c0 = sg.coff[g], nch = sg.coff[g + 1] - c0;
  double s = 0.0;
  for (int c = threadIdx.x; c < nch; c += 256) s += part[c0 + c];
  const double rn2 = block_sum256(s, red);
  if (threadIdx.x != 0) return;
  double* ps = S.ps + int64_t(g) * PS;
  ps[PS_RN2] = rn2;
  const double rel = sqrt(rn2) / ps[PS_NF];
  S.hist[int64_t(g) * S.hstride + j + 1] = rel;
  S.it[g] = j + 1;
  if (!(rel > S.rtol)) {
    S.done[g] = rel <= S.rtol ? 1 : 2;
    atomicAdd(S.ndone, 1);
  }
}

__global__ void k_pcg_init(int nseg, PcgState S) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) *S.j = 0;
  if (g >= nseg) return;
  const double* ps = S.ps + int64_t(g) * PS;
  const double nf = ps[PS_NF];
  S.it[g] = 0;
  S.done[g] = 0;
  if (nf == 0.0) {
    S.hist[int64_t(g) * S.hstride] = 0.0;
    S.done[g] = 1;
    atomicAdd(S.ndone, 1);
    return;
  }
  const double rel = sqrt(ps[PS_RN2]) / nf;
  S.hist[int64_t(g) * S.hstride] = rel;
  if (!(rel > S.rtol)) {
    S.done[g] = rel <= S.rtol ? 1 : 2;
    atomicAdd(S.ndone, 1);
  }
}

// rho_{j+1} = (r^T z)_g from the chunk partials (formed again by every block of g), then
// p = z + (rho_{j+1} / rho_j) p on the chunk's rows; the problem's first block stores rho_{j+1}.
__global__ __launch_bounds__(256) void k_pcg_p(Seg sg, PcgState S, const double* __restrict__ z, double* __restrict__ p,
                                               const double* __restrict__ rz_part) {
  __shared__ double red4[4];
  int64_t r0, r1;
  const int g = chunk_rows(sg, blockIdx.x, r0, r1);
  const double rho_new = seg_total(sg, g, rz_part, red4);
  double* ps = S.ps + int64_t(g) * PS;
  const double beta = rho_new / ps[PS_RHO];
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) p[i] = z[i] + beta * p[i];
  if (threadIdx.x == 0 && blockIdx.x == sg.coff[g]) ps[PS_RHO_NEW] = rho_new;
}

// one workgroup: rho_j <- rho_{j+1} for every problem, then j <- j + 1
__global__ __launch_bounds__(256) void k_pcg_advance(int nseg, PcgState S) {
  for (int g = threadIdx.x; g < nseg; g += 256) {
    double* ps = S.ps + int64_t(g) * PS;
    ps[PS_RHO] = ps[PS_RHO_NEW];
  }
  if (threadIdx.x == 0) *S.j += 1;
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = a * x[i] + (b != 0.0 ? b * y[i] : 0.0);
}

// Column sums of squares of each chunk's rows: 1024-thread workgroups, one per chunk.  Lane l of a wave owns
// the columns l, l + 64, ... of a group of CQ_CG column blocks (one pass over the rows per group); wave w takes
// the rows w, w + 16, ..., CQ_U of them per batch with every load of the batch issued (from clamped in-bounds
// rows) before the first product, and the sixteen waves' sums are combined in a fixed order.
constexpr int CQ_NT = 1024, CQ_W = CQ_NT / 64, CQ_U = 4, CQ_CG = 3;
template <class T>
__global__ __launch_bounds__(CQ_NT) void k_colsq_partial(Seg sg, int ncols, const T* __restrict__ X, int64_t ldx,
                                                         double* __restrict__ part) {
  __shared__ double red[CQ_W - 1][CQ_CG][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t r0, r1;
  chunk_rows(sg, blockIdx.x, r0, r1);
  for (int g0 = 0; g0 < ncols; g0 += 64 * CQ_CG) {
    int col[CQ_CG];
#pragma unroll
    for (int g = 0; g < CQ_CG; ++g) col[g] = min(g0 + 64 * g + lane, ncols - 1);
    double s[CQ_CG];
#pragma unroll
    for (int g = 0; g < CQ_CG; ++g) s[g] = 0.0;
    for (int64_t r = r0 + w; r < r1; r += CQ_W * CQ_U) {
      double v[CQ_U][CQ_CG];
#pragma unroll
      for (int u = 0; u < CQ_U; ++u) {
        const int64_t rr = r + CQ_W * u < r1 ? r + CQ_W * u : r;
#pragma unroll
        for (int g = 0; g < CQ_CG; ++g) v[u][g] = double(X[rr * ldx + col[g]]);
      }
#pragma unroll
      for (int u = 0; u < CQ_U; ++u)
        if (r + CQ_W * u < r1)  // uniform over the wave
#pragma unroll
          for (int g = 0; g < CQ_CG; ++g) s[g] += v[u][g] * v[u][g];
    }
    if (w > 0)
#pragma unroll
      for (int g = 0; g < CQ_CG; ++g) red[w - 1][g][lane] = s[g];
    __syncthreads();
    if (w == 0)
#pragma unroll
      for (int g = 0; g < CQ_CG; ++g) {
        const int c = g0 + 64 * g + lane;
        double t = s[g];
#pragma unroll
        for (int x = 0; x < CQ_W - 1; ++x) t += red[x][g][lane];
        if (c < ncols) part[int64_t(blockIdx.x) * ncols + c] = t;
      }
    __syncthreads();
  }
}

__global__ void k_build_seg(int n, const int64_t* __restrict__ off, const int* __restrict__ toff,
                            int* __restrict__ rseg) {
  const int p = blockIdx.y;
  const int64_t i = off[p] + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < off[p + 1]) rseg[i] = p;
  (void)n;
  (void)toff;
}

}  // namespace

int seg_chunks(int64_t rows) {
  if (rows <= 0) return 0;
  const int64_t c = (rows + CHUNK_ROWS - 1) / CHUNK_ROWS;
  return int(c < CHUNK_MAX ? c : CHUNK_MAX);
}

void SegBuf::build(const std::vector<int64_t>& offsets, hipStream_t st) {
  const int n = int(offsets.size()) - 1;
  h_off = offsets;
  std::vector<int> co(n + 1, 0), to(n + 1, 0);
  int64_t maxrows = 0;
  for (int p = 0; p < n; ++p) {
    const int64_t rows = offsets[p + 1] - offsets[p];
    co[p + 1] = co[p] + seg_chunks(rows);
    to[p + 1] = to[p] + int((rows + 63) / 64);
    maxrows = std::max(maxrows, rows);
  }
  off.alloc(n + 1);
  coff.alloc(n + 1);
  toff.alloc(n + 1);
  const int64_t rows = offsets[n];
  rseg.alloc(rows > 0 ? rows : 1);
  upload(off.p, offsets.data(), (n + 1) * sizeof(int64_t), st);
  upload(coff.p, co.data(), (n + 1) * sizeof(int), st);
  upload(toff.p, to.data(), (n + 1) * sizeof(int), st);
  if (rows > 0 && n > 0) {
    dim3 g(unsigned((maxrows + 255) / 256), unsigned(n));
    k_build_seg<<<g, 256, 0, st>>>(n, off.p, toff.p, rseg.p);
    NS_LAUNCH_CHECK();
  }
  view.n = n;
  view.rows = rows;
  view.first = offsets[0];
  view.off = off.p;
  view.coff = coff.p;
  view.toff = toff.p;
  view.rseg = rseg.p;
  view.nchunk = co[n];
  view.ntile = to[n];
}

template <class TA, class TB>
void gram(const Seg& sg, const TA* A, int64_t lda, int ra, const TB* B, int64_t ldb, int rb, double* G,
          int64_t gstride, double alpha, double beta, double* work, hipStream_t st, const double* rscale,
          int64_t rsstride, bool symmetric) {
  const int nout = ra * rb;
  if (nout == 0 || sg.n == 0) return;
  const int ta = (ra + 15) / 16, tbt = (rb + 15) / 16;
  if (ta > 65535) fail(INVALID_ARG, "Gram product too wide");
  dim3 g(unsigned(sg.nchunk), unsigned(ta), unsigned((tbt + GS_MAXT - 1) / GS_MAXT));
  const int sym = (static_cast<const void*>(A) == static_cast<const void*>(B) && lda == ldb && ra == rb) ? 1 : 0;
  // algorithmic work: A and B read once (once in all when they are the same block), the products of the
  // output entries (the lower triangle and the diagonal when symmetric)
  const double rows = double(sg.rows);
  KScope ks(ra > 16 && rb > 16 ? KF_GRAM : KF_GRAM_NARROW, st,
            rows * (double(ra) * sizeof(TA) + (sym ? 0.0 : double(rb) * sizeof(TB))),
            sym || (symmetric && ra == rb) ? rows * ra * (ra + 1.0) : 2.0 * rows * ra * rb);
  // one FP64 column against a block of 16..256 columns (the deflation products Z^T r of the outer iteration)
  if constexpr (sizeof(TA) == 8 && sizeof(TB) == 8) {
    if (rb == 1 && !sym && ra >= 16 && ra <= 256) {
      auto col = [&](auto cpl) {
        constexpr int CPL = decltype(cpl)::value;
        k_gram_col<CPL><<<unsigned(sg.nchunk), GV_NT, 0, st>>>(sg, reinterpret_cast<const double*>(A), lda, ra,
                                                                reinterpret_cast<const double*>(B), ldb, work);
      };
      switch ((ra + 63) / 64) {
        case 1: col(std::integral_constant<int, 1>()); break;
        case 2: col(std::integral_constant<int, 2>()); break;
        case 3: col(std::integral_constant<int, 3>()); break;
        default: col(std::integral_constant<int, 4>()); break;
      }
      NS_LAUNCH_CHECK();
      seg_final(sg, nout, work, G, gstride, alpha, beta, st, rscale, rsstride, rb);
      return;
    }
  }
  // wide FP64 blocks: one workgroup per chunk (FP32 blocks stay on the strip kernel, faster for them)
  if (sizeof(TA) == 8 && sizeof(TB) == 8 && ra >= 32 && rb >= 32 && ra <= GC_MAXC && rb <= GC_MAXC) {
    const int mode = sym ? 1 : (symmetric && ra == rb ? 2 : 0);
    if constexpr (sizeof(TA) == 8 && sizeof(TB) == 8) {
      // every tile of a product of contiguous 80- or 160-column blocks (the lower-triangle products are faster
      // on the general kernel's 16-wave form)
      if (mode == 0 && ra == rb && lda == ra && ldb == rb && (ra == 80 || ra == 160)) {
        const double* Ad = reinterpret_cast<const double*>(A);
        const double* Bd = reinterpret_cast<const double*>(B);
        if (ra == 80)
          k_gram_tw<5, 2><<<unsigned(sg.nchunk), 1024, 0, st>>>(sg, Ad, Bd, work, mode);
        else
          k_gram_tw<10, 7><<<unsigned(sg.nchunk), 1024, 0, st>>>(sg, Ad, Bd, work, mode);
        NS_LAUNCH_CHECK();
        seg_final(sg, nout, work, G, gstride, alpha, beta, st, rscale, rsstride, rb);
        return;
      }
    }
    const int ntile = mode ? ta * (ta + 1) / 2 : ta * tbt;
    const dim3 grid(unsigned(sg.nchunk));
    if (ntile <= 16 * 2)
      k_gram_chunk<TA, TB, 2, 1024><<<grid, 1024, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, mode);
    else if (ntile <= 16 * 4)
      k_gram_chunk<TA, TB, 4, 1024><<<grid, 1024, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, mode);
    else
      k_gram_chunk<TA, TB, 13, 512><<<grid, 512, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, mode);
    NS_LAUNCH_CHECK();
    seg_final(sg, nout, work, G, gstride, alpha, beta, st, rscale, rsstride, rb);
    return;
  }
  switch (std::min(tbt, GS_MAXT)) {  // column tiles per launch column group
    case 1: k_gram_strip<TA, TB, 1><<<g, 256, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, sym); break;
    case 2: k_gram_strip<TA, TB, 2><<<g, 256, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, sym); break;
    case 3: k_gram_strip<TA, TB, 3><<<g, 256, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, sym); break;
    case 4: k_gram_strip<TA, TB, 4><<<g, 256, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, sym); break;
    default: k_gram_strip<TA, TB, GS_MAXT><<<g, 256, 0, st>>>(sg, A, lda, ra, B, ldb, rb, work, sym); break;
  }
  NS_LAUNCH_CHECK();
  seg_final(sg, nout, work, G, gstride, alpha, beta, st, rscale, rsstride, rb);
}

size_t gram_work_elems(const Seg& sg, int maxw) { return size_t(std::max(sg.nchunk, 1)) * maxw * maxw; }

template <class T>
void ts_update(const Seg& sg, int ncols, T* Out, int64_t ldo, double beta, double gamma, const T* X, int64_t ldx,
               int rm, const double* M, int64_t ldm, int64_t mstride, const T* X2, int64_t ldx2, int rm2,
               const double* M2, int64_t ldm2, int64_t m2stride, hipStream_t st) {
  if (sg.rows == 0 || ncols == 0) return;
  // algorithmic work: X (and X2) read once, Out read (beta != 0) and written once, 2 rm ncols flops per row
  const double rows = double(sg.rows);
  KScope ks(ncols > 16 ? KF_BLOCK_UPDATE : KF_BLOCK_UPDATE_NARROW, st,
            rows * sizeof(T) * (double(rm) + rm2 + ncols * (beta != 0.0 ? 2.0 : 1.0)),
            2.0 * rows * ncols * (double(rm) + rm2));
  ts_launch<T>(sg, ncols, Out, ldo, beta, gamma, X, ldx, rm, M, ldm, mstride, st);
  if (rm2 > 0) ts_launch<T>(sg, ncols, Out, ldo, 1.0, gamma, X2, ldx2, rm2, M2, ldm2, m2stride, st);
}

template <class T, class U>
void convert_block(int64_t n, int ncols, const T* X, int64_t ldx, U* Y, int64_t ldy, hipStream_t st) {
  if (n == 0 || ncols == 0) return;
  const int64_t tot = n * ncols;
  k_convert<T, U><<<unsigned((tot + 255) / 256), 256, 0, st>>>(n, ncols, X, ldx, Y, ldy);
  NS_LAUNCH_CHECK();
}

template <class T>
void col_sumsq(const Seg& sg, int ncols, const T* X, int64_t ldx, double* out, double* work, hipStream_t st) {
  if (ncols == 0 || sg.n == 0) return;
  k_colsq_partial<T><<<unsigned(sg.nchunk), CQ_NT, 0, st>>>(sg, ncols, X, ldx, work);
  NS_LAUNCH_CHECK();
  seg_final(sg, ncols, work, out, ncols, 1.0, 0.0, st);
}

void dot(const Seg& sg, const double* x, const double* y, double* out, int64_t ostride, double* work,
         hipStream_t st) {
  if (sg.n == 0) return;
  k_dot_partial<<<sg.nchunk, 256, 0, st>>>(sg, x, y, work);
  NS_LAUNCH_CHECK();
  seg_final(sg, 1, work, out, ostride, 1.0, 0.0, st);
}

void dot_partials(const Seg& sg, const double* x, const double* y, double* part, hipStream_t st) {
  if (sg.n == 0) return;
  k_dot_partial<<<sg.nchunk, 256, 0, st>>>(sg, x, y, part);
  NS_LAUNCH_CHECK();
}

void pcg_update_wr(const Seg& sg, const PcgState& s, double* w, double* r, const double* p, const double* q,
                   const double* pq_part, double* work, hipStream_t st) {
  k_pcg_wr<<<sg.nchunk, 256, 0, st>>>(sg, s, w, r, p, q, pq_part, work);
  NS_LAUNCH_CHECK();
  k_pcg_check<<<sg.n, 256, 0, st>>>(sg, s, work);
  NS_LAUNCH_CHECK();
}

void pcg_update_p(const Seg& sg, const PcgState& s, const double* z, double* p, const double* rz_part,
                  hipStream_t st) {
  k_pcg_p<<<sg.nchunk, 256, 0, st>>>(sg, s, z, p, rz_part);
  NS_LAUNCH_CHECK();
}

void pcg_advance(int nseg, const PcgState& s, hipStream_t st) {
  k_pcg_advance<<<1, 256, 0, st>>>(nseg, s);
  NS_LAUNCH_CHECK();
}

void pcg_init_check(int nseg, const PcgState& s, hipStream_t st) {
  k_pcg_init<<<(nseg + 255) / 256, 256, 0, st>>>(nseg, s);
  NS_LAUNCH_CHECK();
}

void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
  if (n == 0) return;
  k_axpby<<<unsigned(std::min<int64_t>((n + 255) / 256, 2048)), 256, 0, st>>>(n, a, x, b, y);
  NS_LAUNCH_CHECK();
}

template void gram<double, double>(const Seg&, const double*, int64_t, int, const double*, int64_t, int, double*,
                                   int64_t, double, double, double*, hipStream_t, const double*, int64_t, bool);
template void gram<float, float>(const Seg&, const float*, int64_t, int, const float*, int64_t, int, double*,
                                 int64_t, double, double, double*, hipStream_t, const double*, int64_t, bool);
template void ts_update<double>(const Seg&, int, double*, int64_t, double, double, const double*, int64_t, int,
                                const double*, int64_t, int64_t, const double*, int64_t, int, const double*, int64_t,
                                int64_t, hipStream_t);
template void ts_update<float>(const Seg&, int, float*, int64_t, double, double, const float*, int64_t, int,
                               const double*, int64_t, int64_t, const float*, int64_t, int, const double*, int64_t,
                               int64_t, hipStream_t);
template void convert_block<double, float>(int64_t, int, const double*, int64_t, float*, int64_t, hipStream_t);
template void convert_block<float, double>(int64_t, int, const float*, int64_t, double*, int64_t, hipStream_t);
template void convert_block<double, double>(int64_t, int, const double*, int64_t, double*, int64_t, hipStream_t);
template void col_sumsq<double>(const Seg&, int, const double*, int64_t, double*, double*, hipStream_t);
template void col_sumsq<float>(const Seg&, int, const float*, int64_t, double*, double*, hipStream_t);

}  // namespace ns
