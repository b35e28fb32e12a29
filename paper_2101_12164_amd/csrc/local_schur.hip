// Explicit local Schur complements.  For every subdomain j let Gamma_j be the
// interface nodes coupled to block j and B_j = A_{I_j, Gamma_j}.  Then
//   A_GammaI A_I^{-1} A_IGamma = sum_j E_j^T S_j E_j,   S_j = W_j^T W_j,
//   W_j = L_j^{-1} B_j,
// with E_j selecting the rows Gamma_j (the Schur complement of eq.
// schur_complement assembled block by block, never as one global matrix).
// Each application of S_Gamma is then a gather, one batched GEMM S_j X_j on
// MFMA, and a deterministic gather-reduce into A_Gamma X - sum_j E_j^T (...).
#include <algorithm>

#include "ns_handle.h"
#include "ns_vec.h"

namespace ns {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
struct MFL;
template <>
struct MFL<double> {
  using acc_t = v4d;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int q, int v) { return 4 * v + q; }
};
template <>
struct MFL<float> {
  using acc_t = v4f;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int q, int v) { return 4 * q + v; }
};

// Mark the interface columns touched by each block: flag[j * ldf + g - gbase_j] = 1, where block j's
// interface columns lie in [gbase_j, gbase_j + ldf) (its problem's interface rows).
// frow[j ldf + g] = first block-local row of block j coupled to interface node gbase_j + g (NO_ROW: none)
constexpr int NO_ROW = 0x7F7F7F7F;
__global__ void k_mark(int64_t nrows, const int32_t* __restrict__ rblk, const int64_t* __restrict__ roff,
                       const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                       const int64_t* __restrict__ gbase, int64_t ldf, int* __restrict__ frow,
                       int* __restrict__ ccnt, int* __restrict__ over) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int j = rblk[r];
  if (j < 0) return;
  const int lr = int(r - roff[j]);
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int64_t q = int64_t(j) * ldf + (col[e] - gbase[j]);
    atomicMin(&frow[q], lr);
    // entries per column of A_{I_j Gamma_j}: only a count beyond the sparse cap is recorded
    if (atomicAdd(&ccnt[q], 1) + 1 > SPARSE_RHS_CAP) atomicMax(over, 1);
  }
}

// One workgroup per block: its interface list ordered by the first coupled row (ties by node), cidx
// rewritten to the new positions.  Column c of W_j = L_j^{-1} A_{I_j Gamma_j} is zero above that row, so in
// this order every 64-column tile of W_j starts close to its columns' own first rows and the forward sweep
// and W_j^T W_j skip the zero rows of whole tiles.  Lists longer than SORT_MAX keep the node order.
constexpr int SORT_MAX = 4096;
__global__ __launch_bounds__(1024) void k_sort_lists(const int* __restrict__ cnt, const int64_t* __restrict__ gbase,
                                                     int64_t ldf, const int* __restrict__ frow,
                                                     const int64_t* __restrict__ goff, int32_t* __restrict__ cidx,
                                                     int32_t* __restrict__ glist) {
  __shared__ unsigned long long key[SORT_MAX];
  const int j = blockIdx.x;
  const int m = cnt[j];
  if (m > SORT_MAX || m < 2) return;
  int P = 2;
  while (P < m) P <<= 1;
  const int64_t gb = gbase[j];
  int32_t* gl = glist + goff[j];
  for (int i = threadIdx.x; i < P; i += 1024) {
    if (i < m) {
      const uint32_t g = uint32_t(gl[i] - gb);
      key[i] = (uint64_t(uint32_t(frow[int64_t(j) * ldf + g])) << 32) | g;
    } else {
      key[i] = ~0ull;
    }
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)  // bitonic sort, ascending
    for (int h = k >> 1; h > 0; h >>= 1) {
      for (int i = threadIdx.x; i < P; i += 1024) {
        const int o = i ^ h;
        if (o > i) {
          const unsigned long long a = key[i], b = key[o];
          if ((a > b) == ((i & k) == 0)) {
            key[i] = b;
            key[o] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < m; i += 1024) {
    const uint32_t g = uint32_t(key[i] & 0xFFFFFFFFu);
    gl[i] = int32_t(gb + g);
    cidx[int64_t(j) * ldf + g] = i;
  }
}

__global__ void k_row_block(const int* __restrict__ nt, const int64_t* __restrict__ roff, int32_t* __restrict__ rblk) {
  const int j = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nt[j] * TILE) rblk[roff[j] + r] = j;
}

// One workgroup per block: count (mode 0) or compact (mode 1) the flags in
// ascending interface order: cidx[j ldf + g] = local index, glist[off_j + c] = gbase_j + g.
__global__ __launch_bounds__(1024) void k_compact(const int64_t* __restrict__ gcnt, const int64_t* __restrict__ gbase,
                                                  int64_t ldf, const int* __restrict__ flag, int* __restrict__ cnt,
                                                  const int64_t* __restrict__ goff, int32_t* __restrict__ cidx,
                                                  int32_t* __restrict__ glist, int mode) {
  __shared__ int s[1024];
  __shared__ int base;
  const int j = blockIdx.x;
  const int64_t nG = gcnt[j];
  const int* f = flag + int64_t(j) * ldf;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t g0 = 0; g0 < nG; g0 += 1024) {
    const int64_t g = g0 + threadIdx.x;
    const int v = g < nG ? (f[g] != NO_ROW ? 1 : 0) : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    const int incl = s[threadIdx.x];
    if (mode == 1 && g < nG) {
      const int c = base + incl - v;
      cidx[int64_t(j) * ldf + g] = v ? c : -1;
      if (v) glist[goff[j] + c] = int32_t(gbase[j] + g);
    }
    __syncthreads();
    if (threadIdx.x == 1023) base += s[1023];
    __syncthreads();
  }
  if (mode == 0 && threadIdx.x == 0) cnt[j] = base;
}

// B (rows row0 .. row0 + nrows of the padded interior rows, x ldb) = A_IGamma restricted to each block's
// Gamma_j columns; first[j * ldb + c] = first block-local row with a nonzero in column c.
// The sparse form of B_j = A_{I_j Gamma_j} (columns in the sorted order): per column its entries as
// (local row, value) in a slot taken by an atomic counter (each entry has its own row, so the slot order
// does not change any result), and the first nonzero row.
__global__ void k_fill_sparse(int64_t nrows, int64_t row0, const int32_t* __restrict__ rblk,
                              const int64_t* __restrict__ roff, const int64_t* __restrict__ ptr,
                              const int32_t* __restrict__ col, const double* __restrict__ val,
                              const int64_t* __restrict__ gbase, int64_t ldf, const int32_t* __restrict__ cidx,
                              int64_t ldw, int* __restrict__ cnt, int* __restrict__ crow, double* __restrict__ cval,
                              int* __restrict__ first) {
  const int64_t rr = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (rr >= nrows) return;
  const int64_t r = row0 + rr;
  const int j = rblk[r];
  if (j < 0) return;
  const int lr = int(r - roff[j]);
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int64_t q = int64_t(j) * ldw + cidx[int64_t(j) * ldf + (col[e] - gbase[j])];
    const int slot = atomicAdd(&cnt[q], 1);
    if (slot < SPARSE_RHS_CAP) {  // always: the counts were checked when the layout was planned
      crow[q * SPARSE_RHS_CAP + slot] = lr;
      cval[q * SPARSE_RHS_CAP + slot] = val[e];
    }
    atomicMin(&first[q], lr);
  }
}

__global__ void k_fill_B(int64_t nrows, int64_t row0, const int32_t* __restrict__ rblk,
                         const int64_t* __restrict__ roff, const int64_t* __restrict__ ptr,
                         const int32_t* __restrict__ col, const double* __restrict__ val,
                         const int64_t* __restrict__ gbase, int64_t ldf, const int32_t* __restrict__ cidx,
                         double* __restrict__ B, int64_t ldb, int* __restrict__ first) {
  const int64_t rr = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (rr >= nrows) return;
  const int64_t r = row0 + rr;
  const int j = rblk[r];
  if (j < 0) return;
  const int lr = int(r - roff[j]);
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int c = cidx[int64_t(j) * ldf + (col[e] - gbase[j])];
    B[rr * ldb + c] = val[e];
    atomicMin(&first[int64_t(j) * ldb + c], lr);
  }
}

// per (block, 64-column tile): first tile row holding a nonzero of any column
__global__ void k_first_tiles(int nb, int ldb, int ntiles, const int* __restrict__ first, int* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * ntiles) return;
  const int j = idx / ntiles, t = idx % ntiles;
  int m = INT32_MAX;
  for (int c = t * 64; c < min(ldb, t * 64 + 64); ++c) m = min(m, first[int64_t(j) * ldb + c]);
  out[idx] = m == INT32_MAX ? INT32_MAX / 128 : m / TILE;
}

// Batched C_j = A_j^T B_j on MFMA.  A_j: K_j x M_j, B_j: K_j x N (row-major,
// leading dimensions lda_j / ldb_j), C_j: M_j x N (ld ldc_j).  Output tile
// 64 x NC per workgroup; K in chunks of 32 rows staged through LDS with a
// one-deep register prefetch.  With sym != 0 (A = B, square C) only tiles on
// or below the diagonal are computed and each is also written transposed.
struct GemmBatch {
  const int* kstart;    // optional [j * kstride + tile]: first 64-row tile of nonzeros of A/B column tile
  int kstride;
  const int* M;         // rows of C per block
  const int* K;         // reduction length per block
  const int64_t* aoff;  // element offset of A_j
  const int64_t* lda;   // leading dimension of A_j
  const int64_t* boff;  // offset of B_j = boff[j] * bscale
  int64_t bscale;
  int64_t ldb;          // leading dimension of every B_j
  const int64_t* coff;  // offset of C_j = coff[j] * cscale
  int64_t cscale;
  const int64_t* ldc;   // per block, or NULL: ldc_s
  int64_t ldc_s;
  const int* perm = nullptr;  // optional [8][plen]: blocks whose tiles run on each XCD (-1: none)
  int plen = 0;
};

// Blocks dealt to the 8 XCDs so that their work is balanced (largest first, each to the least loaded XCD):
// [8][plen] block lists padded with -1.
std::vector<int> xcd_lists(const std::vector<double>& work, int& plen) {
  const int n = int(work.size());
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<std::vector<int>> lists(8);
  double load[8] = {};
  for (int j : order) {
    int x = 0;
    for (int y = 1; y < 8; ++y)
      if (load[y] < load[x]) x = y;
    lists[x].push_back(j);
    load[x] += work[j];
  }
  plen = 0;
  for (auto& l : lists) plen = std::max(plen, int(l.size()));
  std::vector<int> flat(size_t(8) * std::max(plen, 1), -1);
  for (int x = 0; x < 8; ++x)
    for (size_t k = 0; k < lists[x].size(); ++k) flat[size_t(x) * plen + k] = lists[x][k];
  return flat;
}

// One-dimensional launch of nb blocks x (gx x gy) output tiles.  Workgroup ids are dispatched round-robin
// over the 8 XCDs; with 8 or more blocks, the ids of all tiles of a block are taken on one XCD (slot s of XCD
// x: list entry s / tiles of x, tile s % tiles, row-major over (tm, tn)), so the tiles that share operand
// columns share that XCD's L2.  The lists come from perm (work-balanced) or are x, x + 8, ...  With fewer
// blocks the tiles of a block are spread over every XCD.
inline unsigned gemm_grid(int gx, int gy, int nb, int plen = 0) {
  const unsigned tiles = unsigned(gx) * unsigned(gy);
  if (nb < 8) return unsigned(nb) * tiles;
  return unsigned(8 * (plen > 0 ? plen : (nb + 7) / 8)) * tiles;
}

template <class T, int NC>
__global__ __launch_bounds__(256) void k_gemm_tn(GemmBatch g, const T* __restrict__ A, const T* __restrict__ B,
                                                 T* __restrict__ C, int N, int sym, int gx, int gy, int nb) {
  using acc_t = typename MFL<T>::acc_t;
  constexpr int KC = 32;
  constexpr int AP = 64 + 1, BP = NC + 1;
  // wave layout: NC == 64: wave w owns rows [32*(w>>1), +32) x cols [32*(w&1), +32) (2 x 2 MFMA tiles)
  //              NC == 16: wave w owns rows [16 w, +16) x cols [0, 16)
  //              NC == 80: wave w owns rows [16 w, +16) x cols [0, 80) (1 x 5 tiles sharing the A operand)
  constexpr int MR = NC == 64 ? 2 : 1;          // MFMA row tiles per wave
  constexpr int MC = NC == 64 ? 2 : NC / 16;    // MFMA column tiles per wave
  __shared__ T sA[KC * AP];
  __shared__ T sB[KC * BP];
  const int tiles = gx * gy;
  int j, t;
  if (nb < 8) {
    j = int(blockIdx.x) / tiles;
    t = int(blockIdx.x) % tiles;
  } else {
    const int slot = int(blockIdx.x >> 3), x = int(blockIdx.x & 7), lb = slot / tiles;
    t = slot % tiles;
    j = g.perm ? (lb < g.plen ? g.perm[x * g.plen + lb] : -1) : x + 8 * lb;
  }
  if (j < 0 || j >= nb) return;
  const int tm = t / gx, tn = t % gx;
  const int M = g.M[j], K = g.K[j];
  const int m0 = tm * 64, n0 = tn * NC;
  if (m0 >= M || n0 >= (sym ? M : N)) return;
  if (sym && tn * NC > tm * 64 + 63) return;  // strictly above the diagonal
  const T* Aj = A + g.aoff[j];
  const T* Bj = B + g.boff[j] * g.bscale;
  const int64_t lda = g.lda[j], ldb = g.ldb;
  const int Nj = sym ? M : N;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rl = lane & 15, kq = lane >> 4;
  const int wr = NC == 64 ? 32 * (w >> 1) : 16 * w;
  const int wc = NC == 64 ? 32 * (w & 1) : 0;
  // columns of A and B are zero above their first nonzero tile row: start K there
  int kbeg = 0;
  if (g.kstart) {
    const int ka = g.kstart[j * g.kstride + tm];
    const int kb = g.kstart[j * g.kstride + (n0 >> 6)];
    kbeg = min(max(ka, kb) * 64, K);
  }
  acc_t acc[MR][MC];
#pragma unroll
  for (int a = 0; a < MR; ++a)
#pragma unroll
    for (int b = 0; b < MC; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  constexpr int PA = KC * 64 / 256, PB = (KC * NC + 255) / 256;
  T ra[PA], rb[PB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int e = threadIdx.x + 256 * q, kk = e / 64, m = e % 64;
      ra[q] = (k0 + kk < K && m0 + m < M) ? Aj[int64_t(k0 + kk) * lda + m0 + m] : T(0);
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = threadIdx.x + 256 * q, kk = e / NC, n = e % NC;
      rb[q] = (kk < KC && k0 + kk < K && n0 + n < Nj) ? Bj[int64_t(k0 + kk) * ldb + n0 + n] : T(0);
    }
  };
  if (kbeg < K) gload(kbeg);
  for (int k0 = kbeg; k0 < K; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int e = threadIdx.x + 256 * q;
      sA[(e / 64) * AP + e % 64] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < KC * NC) sB[(e / NC) * BP + e % NC] = rb[q];
    }
    if (k0 + KC < K) gload(k0 + KC);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T a[MR], b[MC];
#pragma unroll
      for (int q = 0; q < MR; ++q) a[q] = sA[(kk + kq) * AP + wr + 16 * q + rl];
#pragma unroll
      for (int q = 0; q < MC; ++q) b[q] = sB[(kk + kq) * BP + wc + 16 * q + rl];
#pragma unroll
      for (int x = 0; x < MR; ++x)
#pragma unroll
        for (int y = 0; y < MC; ++y) acc[x][y] = MFL<T>::mma(a[x], b[y], acc[x][y]);
    }
  }
  T* Cj = C + g.coff[j] * g.cscale;
  const int64_t ldc = g.ldc ? g.ldc[j] : g.ldc_s;
#pragma unroll
  for (int x = 0; x < MR; ++x)
#pragma unroll
    for (int y = 0; y < MC; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wr + 16 * x + MFL<T>::row(kq, v);
        const int c = n0 + wc + 16 * y + rl;
        if (r < M && c < Nj) {
          Cj[int64_t(r) * ldc + c] = acc[x][y][v];
          if (sym && tm != tn) Cj[int64_t(c) * ldc + r] = acc[x][y][v];
        }
      }
}

// Products C_b = A_b^T B_b with few output tiles (the explicit inverse of a
// single dense junction block applied to up to 80 columns): one workgroup per
// 16-row strip of C, its eight waves taking every eighth k-step of the
// reduction with the operands read straight from the cache, the eight partial
// strips summed in LDS in a fixed order.  NQ 16-column MFMA tiles per strip; with ncg > 1 column groups of
// 16 NQ columns each take a workgroup of their own.
constexpr int KSPLIT_WAVES = 8;
template <class T, int NQ>
__global__ __launch_bounds__(64 * KSPLIT_WAVES) void k_gemm_tn_ksplit(GemmBatch g, const T* __restrict__ A,
                                                                      const T* __restrict__ B, T* __restrict__ C,
                                                                      int N, int strips, int nb, int ncg = 1) {
  using acc_t = typename MFL<T>::acc_t;
  __shared__ T red[KSPLIT_WAVES][NQ * 4][64];
  const int n0 = 16 * NQ * (int(blockIdx.x) % ncg), wg = int(blockIdx.x) / ncg;
  const int j = wg / strips, tm = wg % strips;
  if (j >= nb) return;
  const int M = g.M[j], K = g.K[j];
  const int m0 = 16 * tm;
  if (m0 >= M) return;
  const T* Aj = A + g.aoff[j];
  const int64_t lda = g.lda[j];
  const T* Bj = B + g.boff[j] * g.bscale;
  const int64_t ldb = g.ldb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rl = lane & 15, kq = lane >> 4;
  acc_t acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = acc_t{0, 0, 0, 0};
  // the loads of U k-steps are issued together (unconditional, from clamped indices; out-of-range values are
  // replaced by zero) before their products, so they are in flight at the same time
  constexpr int U = 4;
  const int mc = min(m0 + rl, M - 1);
  const bool mok = m0 + rl < M;
  for (int kk = 4 * w; kk < K; kk += 4 * KSPLIT_WAVES * U) {
    T av[U], bv[U][NQ];
    bool kin[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kk + 4 * KSPLIT_WAVES * u + kq;
      kin[u] = k < K;
      const int64_t kc = min(k, K - 1);
      av[u] = Aj[kc * lda + mc];
#pragma unroll
      for (int q = 0; q < NQ; ++q) bv[u][q] = Bj[kc * ldb + min(n0 + 16 * q + rl, N - 1)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T a = (kin[u] && mok) ? av[u] : T(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        acc[q] = MFL<T>::mma(a, (kin[u] && n0 + 16 * q + rl < N) ? bv[u][q] : T(0), acc[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[w][4 * q + v][lane] = acc[q][v];
  __syncthreads();
  T* Cj = C + g.coff[j] * g.cscale;
  const int64_t ldc = g.ldc ? g.ldc[j] : g.ldc_s;
  for (int e = threadIdx.x; e < NQ * 4 * 64; e += 64 * KSPLIT_WAVES) {
    const int qv = e >> 6, ln = e & 63;
    T sum = red[0][qv][ln];
#pragma unroll
    for (int x = 1; x < KSPLIT_WAVES; ++x) sum += red[x][qv][ln];
    const int r = m0 + MFL<T>::row(ln >> 4, qv & 3), c = n0 + 16 * (qv >> 2) + (ln & 15);
    if (r < M && c < N) Cj[int64_t(r) * ldc + c] = sum;
  }
}

// Symmetric product C_j = W_j^T W_j (FP64, the lower 64 x 64 tiles, each also
// stored transposed) for the local Schur formation.  K runs in chunks of KC
// rows from the later first nonzero tile row of the two column tiles; each
// chunk of both operands is staged in LDS in MFMA fragment order (one 16-byte
// read gives a wave both row blocks it needs for a k-step) with the next
// chunk's global loads in flight in registers.  Wave w computes the 32 x 32
// quarter (w >> 1, w & 1) of the tile as 2 x 2 MFMA blocks.
__device__ __forceinline__ int syrk_frag(int r, int k) {  // operand element (row r of the tile, k) in fragment order
  return (((k >> 2) * 64 + (k & 3) * 16 + (r & 15)) << 2) + (r >> 4);
}
template <int KC>
__global__ __launch_bounds__(256) void k_syrk64(GemmBatch g, const double* __restrict__ W, double* __restrict__ C,
                                                int gx, int nb, float* __restrict__ C32, double* __restrict__ P,
                                                const int64_t* __restrict__ ptoff) {
  __shared__ __align__(16) double sA[KC * 64];
  __shared__ __align__(16) double sB[KC * 64];
  const int tiles = gx * gx;
  int j, t;
  if (nb < 8) {
    j = int(blockIdx.x) / tiles;
    t = int(blockIdx.x) % tiles;
  } else {
    const int slot = int(blockIdx.x >> 3), x = int(blockIdx.x & 7), lb = slot / tiles;
    t = slot % tiles;
    j = g.perm ? (lb < g.plen ? g.perm[x * g.plen + lb] : -1) : x + 8 * lb;
  }
  if (j < 0 || j >= nb) return;
  const int tm = t / gx, tn = t % gx;
  if (tn > tm) return;
  const int M = g.M[j], K = g.K[j];
  const int m0 = tm * 64, n0 = tn * 64;
  if (m0 >= M) return;
  const double* Wj = W + g.aoff[j];
  const int64_t ld = g.lda[j];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kq = lane >> 4, rl = lane & 15;
  const int ha = w >> 1, hb = w & 1;  // row-block pair of A (rows 32 ha ..) and of B (columns 32 hb ..)
  int kbeg = 0;
  if (g.kstart) {
    const int ka = g.kstart[j * g.kstride + tm], kb = g.kstart[j * g.kstride + tn];
    kbeg = min(max(ka, kb) * 64, K);
  }
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  // thread's share of a chunk: element e = threadIdx.x + 256 q is row k = e / 64, column e % 64 (each wave
  // reads whole 512-byte rows)
  constexpr int PQ = KC * 64 / 256;
  double ra[PQ], rb[PQ];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int e = threadIdx.x + 256 * q, k = k0 + (e >> 6), c = e & 63;
      const bool kin = k < K;
      const double* row = Wj + int64_t(k) * ld;
      ra[q] = (kin && m0 + c < M) ? row[m0 + c] : 0.0;
      rb[q] = (kin && n0 + c < M) ? row[n0 + c] : 0.0;
    }
  };
  // K is walked from the end down to kbeg: every tile of a block then starts on the same last rows of W_j and
  // the tiles running together on an XCD read the same rows at about the same time (shared in its L2),
  // while tiles with a later first row simply stop earlier
  const int klast = kbeg < K ? kbeg + (K - 1 - kbeg) / KC * KC : kbeg;
  if (kbeg < K) gload(klast);
  for (int k0 = klast; k0 >= kbeg && kbeg < K; k0 -= KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int pos = syrk_frag(e & 63, e >> 6);
      sA[pos] = ra[q];
      sB[pos] = rb[q];
    }
    if (k0 - KC >= kbeg) gload(k0 - KC);
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const double2 a = reinterpret_cast<const double2*>(sA + ((k4 * 64 + lane) << 2))[ha];
      const double2 b = reinterpret_cast<const double2*>(sB + ((k4 * 64 + lane) << 2))[hb];
      acc[0][0] = MFL<double>::mma(a.x, b.x, acc[0][0]);
      acc[0][1] = MFL<double>::mma(a.x, b.y, acc[0][1]);
      acc[1][0] = MFL<double>::mma(a.y, b.x, acc[1][0]);
      acc[1][1] = MFL<double>::mma(a.y, b.y, acc[1][1]);
    }
  }
  // outputs: C (both triangles), optionally its FP32 copy and the packed lower tile (row-major, zero beyond M)
  double* Cj = C + g.coff[j] * g.cscale;
  float* Cj32 = C32 ? C32 + g.coff[j] * g.cscale : nullptr;
  double* Pt = P ? P + (ptoff[j] + tm * (tm + 1) / 2 + tn) * int64_t(64 * 64) : nullptr;
  const int64_t ldc = g.ldc ? g.ldc[j] : g.ldc_s;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = 32 * ha + 16 * x + MFL<double>::row(kq, v), cc = 32 * hb + 16 * y + rl;
        const int r = m0 + rr, c = n0 + cc;
        const bool in = r < M && c < M;
        if (in) {
          Cj[int64_t(r) * ldc + c] = acc[x][y][v];
          if (tm != tn) Cj[int64_t(c) * ldc + r] = acc[x][y][v];
          if (Cj32) {
            Cj32[int64_t(r) * ldc + c] = float(acc[x][y][v]);
            if (tm != tn) Cj32[int64_t(c) * ldc + r] = float(acc[x][y][v]);
          }
        }
        if (Pt) Pt[rr * 64 + cc] = in ? acc[x][y][v] : 0.0;
      }
}

// Contributor lists: for each interface row g the stacked positions p with
// glist[p] == g, in ascending p (deterministic summation order).
__global__ void k_contrib_count(int64_t npos, const int32_t* __restrict__ glist, int64_t* __restrict__ ptr1) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= npos) return;
  const int g = glist[p];
  if (g >= 0) atomicAdd(reinterpret_cast<unsigned long long*>(&ptr1[g + 1]), 1ull);
}

__global__ void k_contrib_fill(int64_t npos, const int32_t* __restrict__ glist, const int64_t* __restrict__ ptr,
                               int* __restrict__ fillc, int32_t* __restrict__ col) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= npos) return;
  const int g = glist[p];
  if (g < 0) return;
  const int slot = atomicAdd(&fillc[g], 1);
  col[ptr[g] + slot] = int32_t(p);
}

__global__ void k_contrib_sort(int64_t nG, const int64_t* __restrict__ ptr, int32_t* __restrict__ col,
                               double* __restrict__ v64, float* __restrict__ v32) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= nG) return;
  const int64_t a = ptr[g], b = ptr[g + 1];
  for (int64_t i = a + 1; i < b; ++i) {  // insertion sort (a handful of entries per row)
    const int32_t x = col[i];
    int64_t k = i - 1;
    while (k >= a && col[k] > x) {
      col[k + 1] = col[k];
      --k;
    }
    col[k + 1] = x;
  }
  for (int64_t i = a; i < b; ++i) {
    v64[i] = 1.0;
    v32[i] = 1.0f;
  }
}


template <class T, int TPR>
__global__ __launch_bounds__(256) void k_schur_epi_local(int64_t nrows, const int64_t* __restrict__ pG,
                                                         const int32_t* __restrict__ cG, const T* __restrict__ vG,
                                                         const T* __restrict__ X, int64_t ldx,
                                                         const int64_t* __restrict__ pC, const int32_t* __restrict__ cC,
                                                         const T* __restrict__ Yg, int64_t ldy_g, T* __restrict__ Y,
                                                         int64_t ldy, int ncols, int w_only) {
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  for (int c = lane; c < ncols; c += TPR) {
    T a = T(0), w = T(0);
    if (!w_only) csr_row_visit(pG[row], pG[row + 1], cG, vG, X, ldx, c, [&](T v, T x) { a += v * x; });
    csr_row_visit(pC[row], pC[row + 1], cC, static_cast<const T*>(nullptr), Yg, ldy_g, c, [&](T, T x) { w += x; });
    Y[row * ldy + c] = w_only ? w : a - w;
  }
}

// The same epilogue for 17..256 columns: one row per wave, lane l owns the columns l + 64 g (g < CPL), and each
// batch of four entries of both lists issues its index loads, then all 4 x CPL data loads of each list, before
// the first sum (a handful of dependent memory round trips per row instead of a few per column group).  The
// sums run in list order per column, as in k_schur_epi_local (same bits).
template <class T, int CPL, int TPR = 64, bool EXACT = false, int BC = 4>
__global__ __launch_bounds__(256) void k_schur_epi_wide(int64_t nrows, const int64_t* __restrict__ pG,
                                                        const int32_t* __restrict__ cG, const T* __restrict__ vG,
                                                        const T* __restrict__ X, int64_t ldx,
                                                        const int64_t* __restrict__ pC, const int32_t* __restrict__ cC,
                                                        const T* __restrict__ Yg, int64_t ldy_g, T* __restrict__ Y,
                                                        int64_t ldy, int ncols, int w_only) {
  // TPR threads per row (64 / TPR rows per wave: their chains of dependent loads overlap)
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  // EXACT: ncols = CPL TPR, so no column is clamped and the loads of a row share one address (immediate offsets)
  int cc[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) cc[g] = EXACT ? lane + TPR * g : min(lane + TPR * g, ncols - 1);
  T a[CPL], w[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) a[g] = w[g] = T(0);
  const int64_t ga = w_only ? 0 : pG[row], gb = w_only ? 0 : pG[row + 1], ca = pC[row], cb = pC[row + 1];
  // batches of 4 A_Gamma entries and BC contributors (an interface row of a two-dimensional box partition has
  // three entries and two contributors, or five and four at a cross point)
  for (int64_t e = ga, f = ca; e < gb || f < cb; e += 4, f += BC) {
    const bool ha = e < gb, hc = f < cb;  // uniform over the row's threads
    int ja[4], jc[BC];
    T va[4], xa[4][CPL], xc[BC][CPL];
    if (ha) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t ek = e + k < gb ? e + k : e;
        ja[k] = cG[ek];
        va[k] = vG[ek];
      }
    }
    if (hc) {
#pragma unroll
      for (int k = 0; k < BC; ++k) jc[k] = cC[f + k < cb ? f + k : f];
    }
    if (ha) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int g = 0; g < CPL; ++g) xa[k][g] = X[int64_t(ja[k]) * ldx + cc[g]];
    }
    if (hc) {
#pragma unroll
      for (int k = 0; k < BC; ++k)
#pragma unroll
        for (int g = 0; g < CPL; ++g) xc[k][g] = Yg[int64_t(jc[k]) * ldy_g + cc[g]];
    }
    if (ha) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (e + k < gb)
#pragma unroll
          for (int g = 0; g < CPL; ++g) a[g] += va[k] * xa[k][g];
    }
    if (hc) {
#pragma unroll
      for (int k = 0; k < BC; ++k)
        if (f + k < cb)
#pragma unroll
          for (int g = 0; g < CPL; ++g) w[g] += xc[k][g];
    }
  }
#pragma unroll
  for (int g = 0; g < CPL; ++g) {
    const int c = lane + TPR * g;
    if (c < ncols) Y[row * ldy + c] = w_only ? w[g] : a[g] - w[g];
  }
}

template <class T, int TPR>
__global__ __launch_bounds__(256) void k_gather_ls(int64_t nrows, const int32_t* __restrict__ src,
                                                   const T* __restrict__ R, int64_t ldr, T* __restrict__ Out,
                                                   int64_t ldo, int ncols) {
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  const int s = src[row];
  for (int c = lane; c < ncols; c += TPR) Out[row * ldo + c] = s >= 0 ? R[int64_t(s) * ldr + c] : T(0);
}

// The same for 17..256 columns: one row per wave, the CPL loads of a lane issued together.
template <class T, int CPL, int TPR = 64>
__global__ __launch_bounds__(256) void k_gather_ls_wide(int64_t nrows, const int32_t* __restrict__ src,
                                                        const T* __restrict__ R, int64_t ldr, T* __restrict__ Out,
                                                        int64_t ldo, int ncols) {
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;  // TPR threads per row
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  const int s = src[row];
  T v[CPL];
  if (s >= 0) {
#pragma unroll
    for (int g = 0; g < CPL; ++g) v[g] = R[int64_t(s) * ldr + min(lane + TPR * g, ncols - 1)];
  } else {
#pragma unroll
    for (int g = 0; g < CPL; ++g) v[g] = T(0);
  }
#pragma unroll
  for (int g = 0; g < CPL; ++g) {
    const int c = lane + TPR * g;
    if (c < ncols) Out[row * ldo + c] = v[g];
  }
}

// C_j = S_j B_j with S_j symmetric and stored as BF16 (so S_j^T = S_j: rows of S_j are read with their K
// entries contiguous), B_j FP32, C_j FP32: 16x16x32 BF16 MFMA with FP32 accumulation.  A workgroup computes a
// 64 x 64 tile of C_j (four waves in 2 x 2, each 32 x 32 = 2 x 2 MFMA tiles); K is staged by 64 through LDS,
// both operands with K contiguous (B converted to BF16, round to nearest even, and transposed on the way in),
// so each lane reads its eight K values of an operand in one 16-byte LDS load.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
constexpr int BKB = 64, BSP = BKB + 8;  // K per batch, LDS row stride (uint16)
__global__ __launch_bounds__(256) void k_gemm_bf16_sym(GemmBatch g, const uint16_t* __restrict__ A,
                                                       const float* __restrict__ B, float* __restrict__ C, int N,
                                                       int gx, int gy, int nb) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[64 * BSP];
  __shared__ __attribute__((aligned(16))) uint16_t sB[64 * BSP];
  const int tiles = gx * gy;
  int j, t;
  if (nb < 8) {
    j = int(blockIdx.x) / tiles;
    t = int(blockIdx.x) % tiles;
  } else {
    const int slot = int(blockIdx.x >> 3), x = int(blockIdx.x & 7), lb = slot / tiles;
    t = slot % tiles;
    j = g.perm ? (lb < g.plen ? g.perm[x * g.plen + lb] : -1) : x + 8 * lb;
  }
  if (j < 0 || j >= nb) return;
  const int tm = t / gx, tn = t % gx;
  const int M = g.M[j], K = g.K[j];
  const int m0 = tm * 64, n0 = tn * 64;
  if (m0 >= M || n0 >= N) return;
  const uint16_t* Aj = A + g.aoff[j];
  const float* Bj = B + g.boff[j] * g.bscale;
  const int64_t lda = g.lda[j], ldb = g.ldb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  f32x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  // per batch: thread e loads 16 K entries of row e / 4 of S_j (two 8-wide pieces) and 16 entries of B_j
  // (K row e / 4, four 4-wide pieces of N); out-of-range entries are zero
  const int ar = threadIdx.x >> 2, ak = 16 * (threadIdx.x & 3);
  uint16_t va[16];
  float vb[16];
  auto gload = [&](int k0) {
    const int m = m0 + ar;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int k = k0 + ak + e;
      va[e] = (m < M && k < K) ? Aj[int64_t(m) * lda + k] : uint16_t(0);
    }
    const int kb = k0 + ar;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int n = n0 + ak + e;
      vb[e] = (kb < K && n < N) ? Bj[int64_t(kb) * ldb + n] : 0.f;
    }
  };
  gload(0);
  for (int k0 = 0; k0 < K; k0 += BKB) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) sA[ar * BSP + ak + e] = va[e];
#pragma unroll
    for (int e = 0; e < 16; ++e) sB[(ak + e) * BSP + ar] = f32_to_bf16(vb[e]);
    __syncthreads();
    if (k0 + BKB < K) gload(k0 + BKB);
#pragma unroll
    for (int kk = 0; kk < BKB; kk += 32) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) a[x] = *reinterpret_cast<const bf16x8*>(&sA[(wr + 16 * x + li) * BSP + kk + 8 * lg]);
#pragma unroll
      for (int y = 0; y < 2; ++y) b[y] = *reinterpret_cast<const bf16x8*>(&sB[(wc + 16 * y + li) * BSP + kk + 8 * lg]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
  float* Cj = C + g.coff[j] * g.cscale;
  const int64_t ldc = g.ldc ? g.ldc[j] : g.ldc_s;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wr + 16 * x + 4 * lg + v, c = n0 + wc + 16 * y + li;
        if (r < M && c < N) Cj[int64_t(r) * ldc + c] = acc[x][y][v];
      }
}

void launch_gemm_bf16(const GemmBatch& g, const uint16_t* A, const float* B, float* C, int N, int maxM, int nblk,
                      hipStream_t st) {
  if (maxM == 0 || nblk == 0 || N == 0) return;
  const int tilesM = (maxM + 63) / 64, tilesN = (N + 63) / 64;
  k_gemm_bf16_sym<<<gemm_grid(tilesN, tilesM, nblk, g.plen), 256, 0, st>>>(g, A, B, C, N, tilesN, tilesM, nblk);
  NS_LAUNCH_CHECK();
}

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = f32_to_bf16(x[i]);
}

// Output tiles of 80 columns instead of 64 where they pad the columns less (160 columns: two tiles of 80 instead
// of three of 64, the last half empty).  Either width sums each output in the same order (same bits).
inline bool cols80(int N) { return N > 80 && 80 * ((N + 79) / 80) < 64 * ((N + 63) / 64); }

template <class T>
void launch_gemm(const LocalSchur& ls, const T* A, const T* B, T* C, int N, hipStream_t st, bool sym,
                 const GemmBatch& g, int maxM, int nblk = -1) {
  if (maxM == 0) return;
  if (nblk < 0) nblk = ls.nblk;
  if (nblk == 0) return;
  const int tilesM = (maxM + 63) / 64;
  if (N <= 16 && !sym) {
    k_gemm_tn<T, 16><<<gemm_grid(1, tilesM, nblk, g.plen), 256, 0, st>>>(g, A, B, C, N, 0, 1, tilesM, nblk);
  } else if (N > 64 && N <= 80 && !sym && tuned("ls_gemm_cols", sizeof(T) == 8 ? "f64" : "f32", N, 80) == 80) {
    k_gemm_tn<T, 80><<<gemm_grid(1, tilesM, nblk, g.plen), 256, 0, st>>>(g, A, B, C, N, 0, 1, tilesM, nblk);
  } else if (!sym && !g.kstart && cols80(N)) {  // first-nonzero tile starts are kept per 64 columns
    const int tilesN = (N + 79) / 80;
    k_gemm_tn<T, 80><<<gemm_grid(tilesN, tilesM, nblk, g.plen), 256, 0, st>>>(g, A, B, C, N, 0, tilesN, tilesM,
                                                                               nblk);
  } else {
    const int tilesN = sym ? tilesM : (N + 63) / 64;
    k_gemm_tn<T, 64><<<gemm_grid(tilesN, tilesM, nblk, g.plen), 256, 0, st>>>(g, A, B, C, N, sym ? 1 : 0, tilesN,
                                                                               tilesM, nblk);
  }
  NS_LAUNCH_CHECK();
}

}  // namespace

template <class T>
void tile_apply_inverse(const TileLevel& lv, const T* B, T* C, int ncols, hipStream_t st, const int32_t* bidx,
                        bool bf16) {
  if (lv.nblk == 0 || ncols == 0) return;
  if constexpr (sizeof(T) == 4) {
    if (bf16 && lv.Ainv16.p) {  // BF16 operands of the symmetric inverses, FP32 accumulation
      GemmBatch g{nullptr, 0, lv.npad_d, lv.npad_d, lv.inv_off, lv.inv_lda, lv.roff, ncols, ncols, lv.roff, ncols,
                  nullptr, ncols};
      double sq = 0;
      for (int b = 0; b < lv.nblk; ++b) sq += double(lv.h_nb[b]) * lv.h_nb[b];
      KScope ks(KF_INV16, st, sq * 2.0 + 2.0 * lv.alg_rows * ncols * sizeof(float), 2.0 * sq * ncols);
      launch_gemm_bf16(g, lv.Ainv16.p, B, C, ncols, lv.max_nt * TILE, lv.nblk, st);
      return;
    }
  }
  const T* A;
  if constexpr (sizeof(T) == 8)
    A = lv.Ainv64.p;
  else
    A = lv.Ainv32.p;
  GemmBatch g{nullptr, 0, lv.npad_d, lv.npad_d, lv.inv_off, lv.inv_lda, lv.roff, ncols, ncols, lv.roff, ncols, nullptr,
              ncols};
  if constexpr (sizeof(T) == 8) {
    if (ncols == 1 && lv.inv_sym.built()) {  // packed symmetric tiles: every stored entry read once
      KScope ks(KF_INV64_NARROW, st, lv.inv_sym.alg_bytes + 2.0 * lv.alg_rows * sizeof(T), lv.inv_sym.alg_flops);
      sym_gemv(lv.inv_sym, B, C, st, bidx);
      return;
    }
  }
  double sq = 0;
  for (int b = 0; b < lv.nblk; ++b) sq += double(lv.h_nb[b]) * lv.h_nb[b];
  KScope ks(sizeof(T) == 8 ? (ncols <= 16 ? KF_INV64_NARROW : KF_INV64) : KF_INV32, st,
            (sq + 2.0 * lv.alg_rows * ncols) * sizeof(T), 2.0 * sq * ncols);
  const int tilesM = lv.max_nt;
  if (ncols <= 160 && lv.nblk * tilesM < 128) {  // few output tiles: split the reduction over eight waves
    const int strips = 4 * tilesM, ncg = (ncols + 79) / 80, grid = strips * lv.nblk * ncg;
    switch (ncg > 1 ? 5 : (ncols + 15) / 16) {
      case 1: k_gemm_tn_ksplit<T, 1><<<grid, 64 * KSPLIT_WAVES, 0, st>>>(g, A, B, C, ncols, strips, lv.nblk); break;
      case 2: k_gemm_tn_ksplit<T, 2><<<grid, 64 * KSPLIT_WAVES, 0, st>>>(g, A, B, C, ncols, strips, lv.nblk); break;
      case 3: k_gemm_tn_ksplit<T, 3><<<grid, 64 * KSPLIT_WAVES, 0, st>>>(g, A, B, C, ncols, strips, lv.nblk); break;
      case 4: k_gemm_tn_ksplit<T, 4><<<grid, 64 * KSPLIT_WAVES, 0, st>>>(g, A, B, C, ncols, strips, lv.nblk); break;
      default:
        k_gemm_tn_ksplit<T, 5><<<grid, 64 * KSPLIT_WAVES, 0, st>>>(g, A, B, C, ncols, strips, lv.nblk, ncg);
        break;
    }
  } else if (ncols <= 16) {
    k_gemm_tn<T, 16><<<gemm_grid(1, tilesM, lv.nblk), 256, 0, st>>>(g, A, B, C, ncols, 0, 1, tilesM, lv.nblk);
  } else if (ncols > 64 && ncols <= 80) {
    k_gemm_tn<T, 80><<<gemm_grid(1, tilesM, lv.nblk), 256, 0, st>>>(g, A, B, C, ncols, 0, 1, tilesM, lv.nblk);
  } else {
    const int tilesN = (ncols + 63) / 64;
    k_gemm_tn<T, 64><<<gemm_grid(tilesN, tilesM, lv.nblk), 256, 0, st>>>(g, A, B, C, ncols, 0, tilesN, tilesM,
                                                                          lv.nblk);
  }
  NS_LAUNCH_CHECK();
}

void tri_gram(const TileLevel& lv, const double* Y, double* C, int64_t ld, const int* kstart, int kstride,
              double alg_flops, hipStream_t st) {
  if (lv.nblk == 0) return;
  // C_b = Y_b^T Y_b: block b at element offset inv_off[b] of both, every leading dimension ld
  GemmBatch g{kstart, kstride, lv.npad_d, lv.npad_d, lv.inv_off, lv.inv_lda, lv.inv_off, 1, ld, lv.inv_off, 1,
              lv.inv_lda, 0};
  double sq = 0;
  for (int b = 0; b < lv.nblk; ++b) sq += double(lv.h_nt[b]) * TILE * lv.h_nt[b] * TILE;
  KScope ks(KF_INV64, st, 2.0 * sq * sizeof(double), alg_flops);
  k_gemm_tn<double, 64><<<gemm_grid(lv.max_nt, lv.max_nt, lv.nblk), 256, 0, st>>>(g, Y, Y, C, 0, 1, lv.max_nt,
                                                                                   lv.max_nt, lv.nblk);
  NS_LAUNCH_CHECK();
}

template void tile_apply_inverse<double>(const TileLevel&, const double*, double*, int, hipStream_t, const int32_t*,
                                         bool);
template void tile_apply_inverse<float>(const TileLevel&, const float*, float*, int, hipStream_t, const int32_t*,
                                        bool);

void tile_make_bf16_inverse(TileLevel& lv, hipStream_t st) {
  if (!lv.Ainv32.p) return;
  lv.Ainv16.alloc(lv.Ainv32.n);
  k_to_bf16<<<2048, 256, 0, st>>>(lv.Ainv32.p, lv.Ainv16.p, int64_t(lv.Ainv32.n));
  NS_LAUNCH_CHECK();
}

void local_schur_make_bf16(Handle& h) {
  LocalSchur& ls = h.LS;
  if (!ls.built || !ls.S32.p) return;
  ls.S16.alloc(ls.S32.n);
  k_to_bf16<<<2048, 256, 0, h.stream>>>(ls.S32.p, ls.S16.p, int64_t(ls.S32.n));
  NS_LAUNCH_CHECK();
}

void local_schur_plan(Handle& h) {
  hipStream_t st = h.stream;
  LocalSchur& ls = h.LS;
  const TileLevel& lv = h.L1;
  const int nb = lv.nblk;
  const int64_t nIp = lv.nrows_pad;
  ls.nblk = nb;
  // row -> block map of the padded interior rows
  LocalSchurPlan& pl = ls.plan;
  DBuf<int32_t>& rblk = pl.rblk;
  rblk.alloc(nIp);
  NS_HIP(hipMemsetAsync(rblk.p, 0xFF, nIp * sizeof(int32_t), st));
  k_row_block<<<dim3((lv.max_nt * TILE + 255) / 256, nb), 256, 0, st>>>(lv.nt, lv.roff, rblk);
  NS_LAUNCH_CHECK();
  // interface range of every block: its problem's interface rows
  std::vector<int64_t> gbase(nb), gcnt(nb);
  int64_t& ldf = pl.ldf;
  ldf = 1;
  for (int q = 0; q < h.nprob; ++q) {
    const int64_t g0 = h.h_goff[q], g1 = h.h_goff[q + 1];
    ldf = std::max(ldf, g1 - g0);
    for (int j = h.h_sub[q]; j < h.h_sub[q + 1]; ++j) {
      gbase[j] = g0;
      gcnt[j] = g1 - g0;
    }
  }
  DBuf<int64_t>& gbase_d = pl.gbase_d;
  DBuf<int64_t> gcnt_d;
  gbase_d.alloc(nb);
  gcnt_d.alloc(nb);
  upload(gbase_d.p, gbase.data(), nb * sizeof(int64_t), st);
  upload(gcnt_d.p, gcnt.data(), nb * sizeof(int64_t), st);
  DBuf<int> flag, cnt;
  DBuf<int32_t>& cidx = pl.cidx;
  flag.alloc(int64_t(nb) * ldf);
  cnt.alloc(nb);
  cidx.alloc(int64_t(nb) * ldf);
  NS_HIP(hipMemsetAsync(flag.p, 0x7F, int64_t(nb) * ldf * sizeof(int), st));  // NO_ROW
  DBuf<int> ccnt;
  ccnt.alloc(int64_t(nb) * ldf + 1);  // per (block, interface row) entry counts, then the overflow flag
  NS_HIP(hipMemsetAsync(ccnt.p, 0, (int64_t(nb) * ldf + 1) * sizeof(int), st));
  int* over = ccnt.p + int64_t(nb) * ldf;
  k_mark<<<unsigned((nIp + 255) / 256), 256, 0, st>>>(nIp, rblk, lv.roff, h.AIG.ptr, h.AIG.col, gbase_d, ldf, flag,
                                                      ccnt, over);
  NS_LAUNCH_CHECK();
  k_compact<<<nb, 1024, 0, st>>>(gcnt_d, gbase_d, ldf, flag, cnt, nullptr, nullptr, nullptr, 0);
  NS_LAUNCH_CHECK();
  ls.h_m.resize(nb);
  int* h_over = static_cast<int*>(pinned_scratch(sizeof(int)));
  NS_HIP(hipMemcpyAsync(ls.h_m.data(), cnt.p, nb * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(h_over, over, sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  pl.sparse_rhs = *h_over == 0;
  // stacked layouts: Gamma_j lists padded to 64 rows; S_j with ld = padded m_j
  std::vector<int64_t> goff(nb), soff(nb), sld(nb), wld(nb);
  std::vector<int>& Kv = pl.Kv;
  Kv.assign(nb, 0);
  int64_t gp = 0, sp = 0;
  ls.max_m = 0;
  for (int j = 0; j < nb; ++j) {
    const int m = ls.h_m[j], mp = (m + 63) / 64 * 64;
    goff[j] = gp;
    soff[j] = sp;
    sld[j] = mp > 0 ? mp : 1;
    gp += mp;
    sp += int64_t(mp) * mp;
    ls.max_m = std::max(ls.max_m, m);
    Kv[j] = lv.h_nt[j] * TILE;
  }
  ls.npos = gp;
  ls.s_elems = sp;
  {
    // applies S_j^T X: blocks dealt to the XCDs by their work m_j^2
    std::vector<double> wk(nb);
    for (int j = 0; j < nb; ++j) wk[j] = double(ls.h_m[j]) * ls.h_m[j];
    const std::vector<int> lists = xcd_lists(wk, ls.xplen);
    ls.xperm.alloc(lists.size());
    upload(ls.xperm.p, lists.data(), lists.size() * sizeof(int), st);
  }
  const int64_t ldw = std::max(ls.max_m, 1);
  pl.ldw = ldw;
  for (int j = 0; j < nb; ++j) wld[j] = ldw;
  ls.goff.alloc(nb);
  upload(ls.goff.p, goff.data(), nb * sizeof(int64_t), st);
  ls.glist.alloc(gp > 0 ? gp : 1);
  NS_HIP(hipMemsetAsync(ls.glist.p, 0xFF, ls.glist.n * sizeof(int32_t), st));
  k_compact<<<nb, 1024, 0, st>>>(gcnt_d, gbase_d, ldf, flag, cnt, ls.goff, cidx, ls.glist, 1);
  NS_LAUNCH_CHECK();
  k_sort_lists<<<nb, 1024, 0, st>>>(cnt, gbase_d, ldf, flag, ls.goff, cidx, ls.glist);
  NS_LAUNCH_CHECK();
  // per-block metadata for the batched GEMMs
  auto up = [&](DBuf<int64_t>& d, const std::vector<int64_t>& v) {
    d.alloc(nb);
    upload(d.p, v.data(), nb * sizeof(int64_t), st);
  };
  ls.M.alloc(nb);
  ls.K.alloc(nb);
  ls.Kg.alloc(nb);
  upload(ls.M.p, ls.h_m.data(), nb * sizeof(int), st);
  upload(ls.K.p, Kv.data(), nb * sizeof(int), st);
  upload(ls.Kg.p, ls.h_m.data(), nb * sizeof(int), st);
  up(ls.soff, soff);
  up(ls.sld, sld);
  up(ls.wld, wld);
  ls.S64.alloc(sp > 0 ? sp : 1);
  NS_HIP(hipMemsetAsync(ls.S64.p, 0, ls.S64.n * sizeof(double), st));
}

void local_schur_form(Handle& h) {
  hipStream_t st = h.stream;
  LocalSchur& ls = h.LS;
  const TileLevel& lv = h.L1;
  const int nb = lv.nblk;
  const int64_t nG = h.nG;
  LocalSchurPlan& pl = ls.plan;
  const DBuf<int32_t>& rblk = pl.rblk;
  const DBuf<int64_t>& gbase_d = pl.gbase_d;
  const DBuf<int32_t>& cidx = pl.cidx;
  const int64_t ldf = pl.ldf, ldw = pl.ldw;
  const std::vector<int>& Kv = pl.Kv;
  const int64_t gp = ls.npos;
  // W_j = L_j^{-1} B_j (forward sweep only), then S_j = W_j^T W_j, for groups of consecutive blocks whose
  // W fits a fixed budget (the groups only bound memory: every block is computed the same way)
  const int64_t budget = std::max<int64_t>(int64_t(1) << 30, int64_t(lv.max_nt) * TILE * ldw);
  const int ctiles = int((ldw + 63) / 64);
  DBuf<int> first, ftile;
  first.alloc(int64_t(nb) * ldw);
  NS_HIP(hipMemsetAsync(first.p, 0x7F, int64_t(nb) * ldw * sizeof(int), st));  // ~INT_MAX
  ftile.alloc(int64_t(nb) * ctiles);
  int64_t wmax = 0;
  std::vector<std::pair<int, int>> groups;
  for (int b0 = 0; b0 < nb;) {
    int b1 = b0 + 1;
    while (b1 < nb && (lv.h_roff[b1] + int64_t(lv.h_nt[b1]) * TILE - lv.h_roff[b0]) * ldw <= budget) ++b1;
    groups.push_back({b0, b1});
    wmax = std::max(wmax, (lv.h_roff[b1 - 1] + int64_t(lv.h_nt[b1 - 1]) * TILE - lv.h_roff[b0]) * ldw);
    b0 = b1;
  }
  DBuf<double> W;
  W.alloc(wmax > 0 ? wmax : 1);
  // the product also writes the FP32 copy of S_j and the packed lower tiles of the single-column applies
  if (h.prec_inner) ls.S32.alloc(ls.S64.n);
  sym_layout(ls.sym, ls.h_m, ls.goff.p, st);
  // sparse right-hand sides: the sweep builds each tile row of B_j from the column entries, so W is neither
  // cleared nor filled (rows above a chunk's first tile are never read)
  const bool sparse = pl.sparse_rhs && tile_sparse_rhs_ok(lv);
  DBuf<int> scnt, srow;
  DBuf<double> sval;
  if (sparse) {
    scnt.alloc(int64_t(nb) * ldw);
    srow.alloc(int64_t(nb) * ldw * SPARSE_RHS_CAP);
    sval.alloc(int64_t(nb) * ldw * SPARSE_RHS_CAP);
    NS_HIP(hipMemsetAsync(scnt.p, 0, int64_t(nb) * ldw * sizeof(int), st));
  }
  DBuf<int64_t> woffg;
  woffg.alloc(nb);
  DBuf<int> gperm;
  std::vector<int64_t> hwo(nb);
  for (const auto& gr : groups) {
    const int b0 = gr.first, b1 = gr.second, nbs = b1 - b0;
    const int64_t row0 = lv.h_roff[b0];
    const int64_t rows = lv.h_roff[b1 - 1] + int64_t(lv.h_nt[b1 - 1]) * TILE - row0;
    if (sparse) {
      k_fill_sparse<<<unsigned((rows + 255) / 256), 256, 0, st>>>(rows, row0, rblk, lv.roff, h.AIG.ptr, h.AIG.col,
                                                                  h.AIG.val64, gbase_d, ldf, cidx, ldw, scnt, srow,
                                                                  sval, first);
    } else {
      NS_HIP(hipMemsetAsync(W.p, 0, rows * ldw * sizeof(double), st));
      k_fill_B<<<unsigned((rows + 255) / 256), 256, 0, st>>>(rows, row0, rblk, lv.roff, h.AIG.ptr, h.AIG.col,
                                                             h.AIG.val64, gbase_d, ldf, cidx, W, ldw, first);
    }
    NS_LAUNCH_CHECK();
    k_first_tiles<<<(nbs * ctiles + 255) / 256, 256, 0, st>>>(nbs, int(ldw), ctiles, first.p + int64_t(b0) * ldw,
                                                               ftile.p + int64_t(b0) * ctiles);
    NS_LAUNCH_CHECK();
    // the formation's algorithmic flops are added once all groups are queued (they need the first rows)
    SparseRhs sr;
    if (sparse) {
      const int64_t q0 = int64_t(b0) * ldw;
      sr = SparseRhs{scnt.p + q0, srow.p + q0 * SPARSE_RHS_CAP, sval.p + q0 * SPARSE_RHS_CAP, ldw};
    }
    tile_solve_fwd<double>(lv, W.p, ldw, int(ldw), 64, st, ls.M.p, ftile.p, 0.0, b0, b1, row0, KF_LS_FORM,
                           sparse ? &sr : nullptr);  // W_j = L_j^{-1} B_j
    for (int j = b0; j < b1; ++j) hwo[j] = (lv.h_roff[j] - row0) * ldw;
    upload(woffg.p + b0, hwo.data() + b0, nbs * sizeof(int64_t), st);
    // B_j = W_j: offset woff[j] inside the group, common leading dimension ldw
    GemmBatch g{ftile.p + int64_t(b0) * ctiles, ctiles, ls.M.p + b0, ls.K.p + b0, woffg.p + b0, ls.wld.p + b0,
                woffg.p + b0, 1, ldw, ls.soff.p + b0, 1, ls.sld.p + b0, 0};
    // blocks of the group dealt to the XCDs by their work (m_j^2 K_j)
    std::vector<double> wk(nbs);
    for (int j = b0; j < b1; ++j) wk[j - b0] = double(ls.h_m[j]) * ls.h_m[j] * Kv[j];
    int plen = 0;
    const std::vector<int> lists = xcd_lists(wk, plen);
    gperm.alloc(lists.size());
    upload(gperm.p, lists.data(), lists.size() * sizeof(int), st);
    g.perm = gperm.p;
    g.plen = plen;
    KScope ks(KF_LS_FORM, st, double(rows) * ldw * 8.0, 0.0);
    if (ls.max_m > 0) {
      const int tilesM = (ls.max_m + 63) / 64;
      k_syrk64<32><<<gemm_grid(tilesM, tilesM, nbs, g.plen), 256, 0, st>>>(
          g, W.p, ls.S64.p, tilesM, nbs, h.prec_inner ? ls.S32.p : nullptr, ls.sym.built() ? ls.sym.tiles.p : nullptr,
          ls.sym.built() ? ls.sym.toff.p + b0 : nullptr);
      NS_LAUNCH_CHECK();
    }
  }
  // contributor CSR (interface row -> stacked positions), values 1
  Csr& C = ls.contrib;
  C.nrows = nG;
  C.ptr.alloc(nG + 1);
  NS_HIP(hipMemsetAsync(C.ptr.p, 0, (nG + 1) * sizeof(int64_t), st));
  k_contrib_count<<<unsigned((gp + 255) / 256), 256, 0, st>>>(gp, ls.glist, C.ptr);
  NS_LAUNCH_CHECK();
  scan_inclusive(C.ptr.p + 1, nG, st);
  NS_HIP(hipMemcpyAsync(&C.nnz, C.ptr.p + nG, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  // Algorithmic flops of the formation, from the first nonzero row f_c of every column of B_j (exact per
  // column): the forward sweep of a column costs, over the rem = n_b - f_c rows from f_c on, two flops per
  // factor entry within the half-bandwidth bw_j plus the diagonal, t(t-1) + 2 (rem - t) bw_j + rem with
  // t = min(rem, bw_j); the product W_j^T W_j forms the lower triangle, entry (a, b) over the rows from
  // max(f_a, f_b) on, i.e. with f sorted ascending sum_k 2 k (n_b - f_(k)).
  std::vector<int> hfc(size_t(nb) * ldw);
  NS_HIP(hipMemcpyAsync(hfc.data(), first.p, hfc.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  stream_idle(st);
  {
    double fl = 0.0;
    std::vector<int> fs;
    for (int j = 0; j < nb; ++j) {
      const int nbj = lv.h_nb[j], bw = lv.h_bw[j], m = ls.h_m[j];
      fs.assign(hfc.begin() + size_t(j) * ldw, hfc.begin() + size_t(j) * ldw + m);
      for (int& f : fs) f = std::min(f, nbj);
      std::sort(fs.begin(), fs.end());
      for (int k = 0; k < m; ++k) {
        const double rem = double(nbj - fs[k]);
        const double tb = std::min(rem, double(bw));
        fl += tb * (tb - 1.0) + 2.0 * (rem - tb) * bw + rem;  // sweep of this column
        fl += 2.0 * (k + 1) * rem;                           // its row of W_j^T W_j
      }
    }
    kscope_add_work(KF_LS_FORM, 0.0, fl);
  }
  C.col.alloc(C.nnz > 0 ? C.nnz : 1);
  C.val64.alloc(C.nnz > 0 ? C.nnz : 1);
  C.val32.alloc(C.nnz > 0 ? C.nnz : 1);
  DBuf<int> fillc;
  fillc.alloc(nG);
  NS_HIP(hipMemsetAsync(fillc.p, 0, nG * sizeof(int), st));
  k_contrib_fill<<<unsigned((gp + 255) / 256), 256, 0, st>>>(gp, ls.glist, C.ptr, fillc, C.col);
  NS_LAUNCH_CHECK();
  k_contrib_sort<<<unsigned((nG + 255) / 256), 256, 0, st>>>(nG, C.ptr, C.col, C.val64, C.val32);
  NS_LAUNCH_CHECK();
  // algorithmic work of one apply (per column): S_j read once, 2 m_j^2 flops
  ls.alg_bytes = 0;
  ls.alg_flops = 0;
  for (int j = 0; j < nb; ++j) {
    ls.alg_bytes += double(ls.h_m[j]) * ls.h_m[j];
    ls.alg_flops += 2.0 * ls.h_m[j] * ls.h_m[j];
  }
  ls.built = true;
  pl.rblk.release();
  pl.cidx.release();
  pl.gbase_d.release();
}

template <class T>
void op_schur_local(Handle& h, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, bool w_only) {
  hipStream_t st = h.stream;
  LocalSchur& ls = h.LS;
  ensure_local_workspace(h, ncols);
  T *Xg, *Yg;
  const T* S;
  if constexpr (sizeof(T) == 8) {
    Xg = ls.wsX64.p;
    Yg = ls.wsY64.p;
    S = ls.S64.p;
  } else {
    Xg = ls.wsX32.p;
    Yg = ls.wsY32.p;
    S = ls.S32.p;
  }
  const int64_t np = ls.npos;
#define NS_TPR_DISPATCH_LS(ncols, BODY) \
  do {                                  \
    if ((ncols) == 1) {                 \
      constexpr int TPR = 1;            \
      BODY;                             \
    } else if ((ncols) <= 16) {         \
      constexpr int TPR = 16;           \
      BODY;                             \
    } else {                            \
      constexpr int TPR = 64;           \
      BODY;                             \
    }                                   \
  } while (0)
  if (sizeof(T) == 8 && ncols == 1 && ldx == 1 && ls.sym.built()) {
    // one column: the packed symmetric tiles (every stored entry of S_j read once), x gathered through glist
    KScope ks(KF_LS_APPLY64_NARROW, st, ls.sym.alg_bytes + 2.0 * np * sizeof(T), ls.sym.alg_flops);
    sym_gemv(ls.sym, reinterpret_cast<const double*>(X), reinterpret_cast<double*>(Yg), st, ls.glist.p);
  } else {
    if (ncols > 16 && ncols <= 256) {
      auto wide = [&](auto cpl, auto tpr) {
        constexpr int CPL = decltype(cpl)::value, TPR = decltype(tpr)::value;
        k_gather_ls_wide<T, CPL, TPR><<<unsigned((np * TPR + 255) / 256), 256, 0, st>>>(np, ls.glist, X, ldx, Xg,
                                                                                        ncols, ncols);
      };
      using T64 = std::integral_constant<int, 64>;
      using T16 = std::integral_constant<int, 16>;
      if (ncols <= 80)  // four rows per wave
        wide(std::integral_constant<int, 5>(), T16());
      else if (ncols <= 160)
        wide(std::integral_constant<int, 10>(), T16());
      else if (ncols <= 192)
        wide(std::integral_constant<int, 3>(), T64());
      else
        wide(std::integral_constant<int, 4>(), T64());
    } else {
      NS_TPR_DISPATCH_LS(ncols, (k_gather_ls<T, TPR><<<unsigned((np * TPR + 255) / 256), 256, 0, st>>>(
                                     np, ls.glist, X, ldx, Xg, ncols, ncols)));
    }
    NS_LAUNCH_CHECK();
    // X_j / Y_j: stacked rows goff[j], leading dimension ncols
    GemmBatch g{nullptr, 0, ls.M, ls.Kg, ls.soff, ls.sld, ls.goff, ncols, ncols, ls.goff, ncols, nullptr, ncols,
                ls.xperm.p, ls.xplen};
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (h.op_bf16 && h.bf16_schur && ls.S16.p) {  // BF16 operands of the symmetric S_j, FP32 accumulation
        KScope ks(KF_LS_APPLY16, st, ls.alg_bytes * 2.0 + 2.0 * np * ncols * sizeof(float), ls.alg_flops * ncols);
        launch_gemm_bf16(g, ls.S16.p, Xg, Yg, ncols, ls.max_m, ls.nblk, st);
        done = true;
      }
    }
    if (!done) {
      KScope ks(sizeof(T) == 8 ? (ncols <= 16 ? KF_LS_APPLY64_NARROW : KF_LS_APPLY64) : KF_LS_APPLY32, st,
                ls.alg_bytes * sizeof(T) + 2.0 * np * ncols * sizeof(T), ls.alg_flops * ncols);
      launch_gemm<T>(ls, S, Xg, Yg, ncols, st, false, g, ls.max_m);
    }
  }
  const T* vG;
  if constexpr (sizeof(T) == 8)
    vG = h.AGG.val64.p;
  else
    vG = h.AGG.val32.p;
  if (ncols > 16 && ncols <= 256) {
    auto wide = [&](auto cpl, auto tpr) {
      constexpr int CPL = decltype(cpl)::value, TPR = decltype(tpr)::value;
      if (ncols == CPL * TPR)
        k_schur_epi_wide<T, CPL, TPR, true, 2><<<unsigned((h.nG * TPR + 255) / 256), 256, 0, st>>>(
            h.nG, h.AGG.ptr, h.AGG.col, vG, X, ldx, ls.contrib.ptr, ls.contrib.col, Yg, ncols, Y, ldy, ncols,
            w_only ? 1 : 0);
      else
        k_schur_epi_wide<T, CPL, TPR><<<unsigned((h.nG * TPR + 255) / 256), 256, 0, st>>>(
            h.nG, h.AGG.ptr, h.AGG.col, vG, X, ldx, ls.contrib.ptr, ls.contrib.col, Yg, ncols, Y, ldy, ncols,
            w_only ? 1 : 0);
    };
    using T64 = std::integral_constant<int, 64>;
    using T32 = std::integral_constant<int, 32>;
    using T16 = std::integral_constant<int, 16>;
    // two rows per wave up to 160 columns (four would hold 80 operand values a lane: one wave per SIMD); 80
    // columns four rows per wave
    if (ncols == 80)
      wide(std::integral_constant<int, 5>(), T16());
    else if (ncols <= 96)
      wide(std::integral_constant<int, 3>(), T32());
    else if (ncols <= 160)
      wide(std::integral_constant<int, 5>(), T32());
    else if (ncols <= 192)
      wide(std::integral_constant<int, 3>(), T64());
    else
      wide(std::integral_constant<int, 4>(), T64());
  } else {
    NS_TPR_DISPATCH_LS(ncols, (k_schur_epi_local<T, TPR><<<unsigned((h.nG * TPR + 255) / 256), 256, 0, st>>>(
                                   h.nG, h.AGG.ptr, h.AGG.col, vG, X, ldx, ls.contrib.ptr, ls.contrib.col, Yg,
                                   ncols, Y, ldy, ncols, w_only ? 1 : 0)));
  }
  NS_LAUNCH_CHECK();
#undef NS_TPR_DISPATCH_LS
}

void ensure_local_workspace(Handle& h, int64_t ncols) {
  LocalSchur& ls = h.LS;
  if (ncols <= ls.ws_cols) return;
  const int64_t n = ls.npos > 0 ? ls.npos * ncols : 1;
  if (h.prec_inner) {
    ls.wsX32.alloc(n);
    ls.wsY32.alloc(n);
  }
  ls.wsX64.alloc(n);
  ls.wsY64.alloc(n);
  ls.ws_cols = ncols;
}

template void op_schur_local<double>(Handle&, const double*, int64_t, double*, int64_t, int, bool);
template void op_schur_local<float>(Handle&, const float*, int64_t, float*, int64_t, int, bool);

}  // namespace ns
