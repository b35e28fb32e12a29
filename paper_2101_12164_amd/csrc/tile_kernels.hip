// Dense tile kernels for gfx950: batched right-looking Cholesky of the subdomain
// blocks (per tile column, one launch applies the previous column to the
// trailing band tiles and factorises the diagonal tile; a second forms the
// panel below it, all on FP64 MFMA) and the batched forward/backward
// triangular solves with many right-hand sides used by every Schur-operator
// application.
//
// The paper factorises the diagonal blocks of A_I independently of each other
// with a direct method (section on Schur complement preconditioners); here
// every block of every size is factorised in the same sequence of launches.
#include <algorithm>
#include <type_traits>

#include "ns_internal.h"

namespace ns {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
struct MF;
// MFMA 16x16x4 operand layout on gfx950 (lane l of a 64-wide wave):
//   A fragment: A[l % 16][l / 16]   (16 rows x 4 k)
//   B fragment: B[l / 16][l % 16]   (4 k x 16 cols)
//   D, FP32: element v of lane l is D[4 * (l / 16) + v][l % 16]
//   D, FP64: element v of lane l is D[4 * v + l / 16][l % 16]
// (measured on the device; row(q, v) below gives the D row for q = l / 16).
template <>
struct MF<double> {
  using acc_t = v4d;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int q, int v) { return 4 * v + q; }
};
template <>
struct MF<float> {
  using acc_t = v4f;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int q, int v) { return 4 * q + v; }
};

constexpr int LDT = TILE + 1;  // LDS row stride of a staged tile (bank spread)


// Tile <-> LDS copies by a 256-thread workgroup: every thread issues its 16
// global loads before the LDS stores, so the loads are in flight together.
constexpr int WG = 256;
template <class T>
__device__ __forceinline__ void load_tile_lds(T* s, const T* __restrict__ g) {
  T r[TILE2 / WG];
#pragma unroll
  for (int q = 0; q < TILE2 / WG; ++q) r[q] = g[threadIdx.x + WG * q];
#pragma unroll
  for (int q = 0; q < TILE2 / WG; ++q) {
    const int e = threadIdx.x + WG * q;
    s[(e >> 6) * LDT + (e & 63)] = r[q];
  }
}
template <class T>
__device__ __forceinline__ void store_tile_lds(T* __restrict__ g, const T* s) {
#pragma unroll
  for (int q = 0; q < TILE2 / WG; ++q) {
    const int e = threadIdx.x + WG * q;
    g[e] = s[(e >> 6) * LDT + (e & 63)];
  }
}

constexpr int PB = 16;  // panel width of the tile factorisation

__device__ __forceinline__ double lane_value(double v, int lane) {  // v of `lane` (lane uniform)
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Value of v in lane N of the calling lane's row of 16 lanes (DPP row broadcast, one VALU move).
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + N, 0xF, 0xF, false);
}
// f(integral_constant<int, I>) for I = B .. E - 1 in order (indices usable as template arguments)
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Inverse of the PB x PB lower triangular block L_kk (rows and columns k0 .. k0 + PB - 1 of s, stride
// LDT) by one wave: every row of 16 lanes holds the block (lane m of a row holds row m), so the factor's
// columns reach the lanes by row broadcasts.  Row m of X from X L = I, columns right to left:
// x_mc = (delta_mc - sum_{i>c} x_mi l_ic) / l_cc, with 1 / l_cc taken from inv_d.  Written by lanes 0-15
// to the same block of x (zeros above the diagonal).
__device__ __forceinline__ void diag_block_inverse(const double* s, double* x, const double* inv_d, int k0,
                                                   int lane) {
  const int m = lane & 15;
  double a[PB], xi[PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) a[q] = s[(k0 + q) * LDT + k0 + m];
  static_for<0, PB>([&](auto cc) {
    constexpr int c = PB - 1 - decltype(cc)::value;
    double acc0 = (m == c) ? 1.0 : 0.0, acc1 = 0.0;
    static_for<c + 1, PB>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const double lic = row_bcast<i>(a[c]);
      if constexpr (i & 1)
        acc1 = fma(-xi[i], lic, acc1);
      else
        acc0 = fma(-xi[i], lic, acc0);
    });
    xi[c] = (acc0 + acc1) * inv_d[k0 + c];
    asm volatile("" : "+v"(xi[c]));  // keeps the row in registers as it is formed (not sunk into the store)
  });
  if (lane < PB) {
#pragma unroll
    for (int q = 0; q < PB; ++q) x[(k0 + q) * LDT + k0 + lane] = xi[q];
  }
}

// Cholesky factor and its inverse of the TILE x TILE SPD tile in s (LDS, column-major, stride LDT; lower
// triangle used), computed by the whole 256-thread workgroup in four panels of PB = 16 columns:
//  * wave 0 factors the panel below the current diagonal in registers (lane r holds row k0 + r; each
//    column's multipliers reach the other lanes by readlane, and the next pivot is formed in its own
//    lane, so no barrier or LDS round trip sits on the chain of pivots);
//  * the four waves then apply the panel to the trailing lower blocks, A_ij -= L_ik L_jk^T, with FP64
//    MFMA.
// Each wave then inverts one 16 x 16 diagonal block, and the inverse is assembled block row by block row,
// X_ij = -X_ii sum_{m=j}^{i-1} L_im X_mj, again on MFMA.
// On return s holds L and x holds L^{-1} (zeros above the diagonal in both).  A pivot <= 0 records
// (block, column) in err once and is replaced by 1 so the sweep finishes.
__device__ __forceinline__ void potrf_trtri_tile(double* s, double* x, double* inv_d, int blk, int jt, int* err) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  // blocks above the diagonal: zero in both outputs
  for (int e = t; e < TILE2; e += 256) {
    const int r = e & 63, c = e >> 6;
    if ((r >> 4) < (c >> 4)) {
      s[c * LDT + r] = 0.0;
      x[c * LDT + r] = 0.0;
    }
  }
  int badc = -1;  // first non-positive pivot (wave 0)
  for (int kb = 0; kb < TILE / PB; ++kb) {
    const int k0 = kb * PB;
    if (w == 0) {
      const int row = k0 + lane;
      const bool act = row < TILE;
      double a[PB], invd[PB];
#pragma unroll
      for (int q = 0; q < PB; ++q) a[q] = act ? s[(k0 + q) * LDT + row] : 0.0;
      // right-looking over the panel: column c is scaled by its pivot, then updates the columns to its right
      double d = lane_value(a[0], 0);
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        if (!(d > 0.0)) {
          if (badc < 0) badc = k0 + c;
          d = 1.0;
        }
        // 1 / sqrt(d): hardware estimate and two Newton steps y <- y (3 - d y^2) / 2; the last step's
        // factor is applied to a_rc * y directly
        const double nh = -0.5 * d;
        double y = __builtin_amdgcn_rsq(d);
        y = y * fma(nh * y, y, 1.5);
        const double e = fma(nh * y, y, 1.5);
        const double inv = y * e;
        invd[c] = inv;  // 1 / l_cc
        const double l = (a[c] * y) * e;
        a[c] = (lane == c) ? d * inv : l;
        // the next pivot from its own lane: a_{c+1,c+1} - l_{c+1,c}^2
        if (c + 1 < PB) d = lane_value(fma(-l, l, a[c + 1]), c + 1);
#pragma unroll
        for (int q = c + 1; q < PB; ++q) a[q] = fma(-l, lane_value(l, q), a[q]);  // a_rq -= l_rc l_qc
      }
      if (act) {
#pragma unroll
        for (int q = 0; q < PB; ++q) s[(k0 + q) * LDT + row] = (lane >= q) ? a[q] : 0.0;
      }
      if (lane < PB) {
        double v = invd[0];
#pragma unroll
        for (int c = 1; c < PB; ++c) v = (lane == c) ? invd[c] : v;
        inv_d[k0 + lane] = v;
      }
    }
    __syncthreads();
    if (kb + 1 < TILE / PB) {
      // trailing lower blocks (i, j), kb < j <= i, spread over the waves
      int nb = 0;
      for (int j = kb + 1; j < TILE / PB; ++j)
        for (int i = j; i < TILE / PB; ++i, ++nb) {
          if ((nb & 3) != w) continue;
          v4d acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] = s[(PB * j + lr) * LDT + PB * i + 4 * v + lq];
#pragma unroll
          for (int st = 0; st < PB / 4; ++st) {
            const int kc = (k0 + 4 * st + lq) * LDT;
            acc = MF<double>::mma(-s[kc + PB * i + lr], s[kc + PB * j + lr], acc);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) s[(PB * j + lr) * LDT + PB * i + 4 * v + lq] = acc[v];
        }
      __syncthreads();
    }
  }
  diag_block_inverse(s, x, inv_d, PB * w, lane);  // wave w: the diagonal block w
  __syncthreads();
  // off-diagonal blocks of the inverse, block row i by wave j < i
  for (int i = 1; i < TILE / PB; ++i) {
    const int j = w;
    if (j < i) {
      v4d tacc = {0, 0, 0, 0};
      for (int m = j; m < i; ++m)
#pragma unroll
        for (int st = 0; st < PB / 4; ++st)  // T += L_im X_mj
          tacc = MF<double>::mma(s[(PB * m + 4 * st + lq) * LDT + PB * i + lr],
                                 x[(PB * j + lr) * LDT + PB * m + 4 * st + lq], tacc);
      v4d xacc = {0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < PB / 4; ++st)  // X_ij = -X_ii T (T's accumulator layout is the B operand layout)
        xacc = MF<double>::mma(-x[(PB * i + 4 * st + lq) * LDT + PB * i + lr], tacc[st], xacc);
#pragma unroll
      for (int v = 0; v < 4; ++v) x[(PB * j + lr) * LDT + PB * i + 4 * v + lq] = xacc[v];
    }
    __syncthreads();
  }
  if (t == 0 && badc >= 0) {
    if (atomicCAS(err, 0, 1) == 0) {
      err[1] = blk;
      err[2] = jt * TILE + badc;
    }
  }
}

// Right-looking step j: every trailing tile (i, k), j <= k <= i, within the band of column j - 1 gets
// A_ik -= L_{i,j-1} L_{k,j-1}^T (one tile product per workgroup, all of them in parallel); the workgroup of
// the diagonal tile (j, j) then factorises it and inverts L_jj.  Pair p of a block numbers the tiles
// (j + di, j + dk), p = di (di + 1) / 2 + dk, so pair 0 (the diagonal, the step's critical path) gets the
// lowest workgroup ids of every block and is dispatched first.  Ids map all tiles of one block to one XCD.
__global__ __launch_bounds__(256) void k_chol_step(int j, int nblk, const int* __restrict__ nt_arr,
                                                   const int* __restrict__ nbt_arr, const int64_t* __restrict__ foff,
                                                   const int64_t* __restrict__ ioff, double* __restrict__ L,
                                                   double* __restrict__ Linv, int* err) {
  __shared__ double sA[TILE * LDT];
  __shared__ double sB[TILE * LDT];
  __shared__ double inv_d[TILE];
  const int nbp8 = (nblk + 7) >> 3;
  const int g = blockIdx.x;
  const int slot = g >> 3;
  const int b = (g & 7) + 8 * (slot % nbp8);
  const int pair = slot / nbp8;
  if (b >= nblk) return;
  int di = 0;
  while ((di + 1) * (di + 2) / 2 <= pair) ++di;
  const int dk = pair - di * (di + 1) / 2;
  const int nt = nt_arr[b], nbt = nbt_arr[b];
  const int i = j + di, k = j + dk, l = j - 1;
  if (i >= nt) return;
  const bool upd = l >= 0 && i - l <= nbt;  // L_il (and L_kl, k <= i) inside the band
  if (!upd && di != 0) return;
  double* Lb = L + foff[b];
  double* Tik = Lb + band_tile_index(nt, nbt, i, k) * TILE2;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (upd) {
    constexpr int PT = TILE2 / 256;
    double ra[PT], rb[PT];
    const double* ga = Lb + band_tile_index(nt, nbt, i, l) * TILE2;
    const double* gb = Lb + band_tile_index(nt, nbt, k, l) * TILE2;
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      ra[q] = ga[threadIdx.x + 256 * q];
      rb[q] = gb[threadIdx.x + 256 * q];
    }
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int e = threadIdx.x + 256 * q;
      sA[(e >> 6) * LDT + (e & 63)] = ra[q];
      sB[(e >> 6) * LDT + (e & 63)] = rb[q];
    }
    __syncthreads();
    const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
    v4d acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
#pragma unroll 4
    for (int kk = 0; kk < TILE; kk += 4) {
      const int kr = (kk + (lane >> 4)) * LDT + (lane & 15);
      const double a0 = sA[kr + r0], a1 = sA[kr + r0 + 16];
      const double b0 = sB[kr + c0], b1 = sB[kr + c0 + 16];
      acc00 = MF<double>::mma(a0, b0, acc00);
      acc01 = MF<double>::mma(a0, b1, acc01);
      acc10 = MF<double>::mma(a1, b0, acc10);
      acc11 = MF<double>::mma(a1, b1, acc11);
    }
    __syncthreads();
    load_tile_lds(sA, Tik);
    __syncthreads();
    const int cb = c0 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rb = r0 + MF<double>::row(lane >> 4, v);
      sA[(cb)*LDT + rb] -= acc00[v];
      sA[(cb + 16) * LDT + rb] -= acc01[v];
      sA[(cb)*LDT + rb + 16] -= acc10[v];
      sA[(cb + 16) * LDT + rb + 16] -= acc11[v];
    }
    __syncthreads();
    if (di != 0) {
      store_tile_lds(Tik, sA);
      return;
    }
  } else {
    load_tile_lds(sA, Tik);
    __syncthreads();
  }
  potrf_trtri_tile(sA, sB, inv_d, b, j, err);
  __syncthreads();
  store_tile_lds(Tik, sA);
  store_tile_lds(Linv + ioff[b] + int64_t(j) * TILE2, sB);
}

// Panel: L_ij = C_ij L_jj^{-T} = C_ij * (L_jj^{-1})^T for i > j.
__global__ __launch_bounds__(256) void k_chol_panel(int j, const int* __restrict__ nt_arr,
                                                    const int* __restrict__ nbt_arr,
                                                    const int64_t* __restrict__ foff,
                                                    const int64_t* __restrict__ ioff, double* __restrict__ L,
                                                    const double* __restrict__ Linv) {
  __shared__ double sA[TILE * LDT];
  __shared__ double sB[TILE * LDT];
  const int b = blockIdx.y;
  const int nt = nt_arr[b], nbt = nbt_arr[b];
  const int i = j + 1 + blockIdx.x;
  if (i >= nt || i - j > nbt) return;
  double* Tij = L + foff[b] + band_tile_index(nt, nbt, i, j) * TILE2;
  load_tile_lds(sA, Tij);
  load_tile_lds(sB, Linv + ioff[b] + int64_t(j) * TILE2);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  v4d acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
#pragma unroll 4
  for (int kk = 0; kk < TILE; kk += 4) {
    const int kr = (kk + (lane >> 4)) * LDT + (lane & 15);
    const double a0 = sA[kr + r0], a1 = sA[kr + r0 + 16];
    const double b0 = sB[kr + c0], b1 = sB[kr + c0 + 16];
    acc00 = MF<double>::mma(a0, b0, acc00);
    acc01 = MF<double>::mma(a0, b1, acc01);
    acc10 = MF<double>::mma(a1, b0, acc10);
    acc11 = MF<double>::mma(a1, b1, acc11);
  }
  __syncthreads();
  {
    const int cb = c0 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rb = r0 + MF<double>::row(lane >> 4, v);
      sA[(cb)*LDT + rb] = acc00[v];
      sA[(cb + 16) * LDT + rb] = acc01[v];
      sA[(cb)*LDT + rb + 16] = acc10[v];
      sA[(cb + 16) * LDT + rb + 16] = acc11[v];
    }
  }
  __syncthreads();
  store_tile_lds(Tij, sA);
}

// --------------------------------------------------------------------------
// Batched triangular solves with many right-hand sides.
//
// One workgroup owns CW columns of one block's padded right-hand side and
// walks its tile rows; wave w computes rows [16w, 16w+16) of each 64-row tile
// with CW/16 MFMA column blocks.  Workgroup ids are mapped so that all column
// chunks of a block run on the same XCD (ids are dispatched round-robin over
// the 8 XCDs) and share that XCD's L2 while they stream the block's factor.

__device__ __forceinline__ void map_block_chunk(int nblk, int& b, int& chunk) {
  const int nbp8 = (nblk + 7) >> 3;  // blocks per XCD
  const int g = blockIdx.x;
  const int xcd = g & 7, slot = g >> 3;
  b = xcd + 8 * (slot % nbp8);
  chunk = slot / nbp8;
}

template <class T, int CW>
__device__ __forceinline__ void load_rows(T* sY, const T* __restrict__ g, int64_t ldb, int c0, int ncols) {
  constexpr int PY = TILE * CW / WG;
  T v[PY];
#pragma unroll
  for (int q = 0; q < PY; ++q) {
    const int e = threadIdx.x + WG * q, r = e / CW, c = e % CW;
    v[q] = (c0 + c < ncols) ? g[int64_t(r) * ldb + c0 + c] : T(0);
  }
#pragma unroll
  for (int q = 0; q < PY; ++q) {
    const int e = threadIdx.x + WG * q, r = e / CW, c = e % CW;
    sY[r * (CW + 1) + c] = v[q];
  }
}

// Register pipeline: each thread holds its share of the next two (tile, rhs
// rows) pairs while the MFMAs run on the pair staged in LDS, so two global
// loads per thread stream are always in flight.
template <class T, int CW>
struct TrsmStage {
  static constexpr int PT = TILE2 / 256;      // tile elements per thread
  static constexpr int PY = TILE * CW / 256;  // rhs elements per thread
  T t[PT];
  T y[PY];
  __device__ __forceinline__ void load(const T* __restrict__ gt, const T* __restrict__ gy, int64_t ldb, int c0,
                                       int ncols) {
#pragma unroll
    for (int q = 0; q < PT; ++q) t[q] = gt[threadIdx.x + 256 * q];
#pragma unroll
    for (int q = 0; q < PY; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / CW, c = e % CW;
      y[q] = (c0 + c < ncols) ? gy[int64_t(r) * ldb + c0 + c] : T(0);
    }
  }
  __device__ __forceinline__ void store(T* sL, T* sY) const {
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int e = threadIdx.x + 256 * q;
      sL[(e >> 6) * LDT + (e & 63)] = t[q];
    }
#pragma unroll
    for (int q = 0; q < PY; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / CW, c = e % CW;
      sY[r * (CW + 1) + c] = y[q];
    }
  }
};

template <class T, int CW, bool FWD>
__global__ __launch_bounds__(256) void k_trsm(int nblk, const int* __restrict__ nt_arr,
                                              const int* __restrict__ nbt_arr, const int64_t* __restrict__ foff, const int64_t* __restrict__ ioff,
                                              const int64_t* __restrict__ roff, const T* __restrict__ L,
                                              const T* __restrict__ Linv, T* __restrict__ B, int64_t ldb,
                                              int ncols, const int* __restrict__ ncols_blk = nullptr,
                                              const int* __restrict__ first_tile = nullptr, int nchunk_all = 0,
                                              int64_t row0 = 0) {
  using acc_t = typename MF<T>::acc_t;
  constexpr int NB = CW / 16;
  constexpr int YP = CW + 1;
  __shared__ T sL[TILE * LDT];
  __shared__ T sY[TILE * YP];
  int b, chunk;
  map_block_chunk(nblk, b, chunk);
  if (b >= nblk) return;
  const int c0 = chunk * CW;
  if (c0 >= ncols) return;
  if (ncols_blk && c0 >= ncols_blk[b]) return;  // this block's columns beyond its count are zero
  const int nt = nt_arr[b], nbt = nbt_arr[b];
  T* Bb = B + (roff[b] - row0) * ldb;  // B holds the padded rows from row0 on
  const T* Lb = L + foff[b];
  const T* Ib = Linv + ioff[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int rl = lane & 15, kq = lane >> 4;
  TrsmStage<T, CW> s0, s1;
  // forward sweeps whose right-hand side is zero above tile row `first` start there; with first_tile the
  // backward sweep only uses it to skip chunks that are entirely zero (first >= nt)
  const int first = first_tile ? min(first_tile[b * nchunk_all + chunk], nt) : 0;
  if (!FWD && first >= nt) return;  // a chunk that is zero on entry stays zero
  for (int step = FWD ? first : 0; step < nt; ++step) {
    const int i = FWD ? step : nt - 1 - step;
    acc_t acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = acc_t{0, 0, 0, 0};
    // FWD: L_il for l in [max(first, i - nbt), i); BWD: L_li for l in (i, min(nt - 1, i + nbt)]
    const int l0 = FWD ? max(first, i - nbt) : i + 1, nl = FWD ? i - l0 : min(nt - 1, i + nbt) - i;
    auto tile = [&](int t) {
      return Lb + (FWD ? band_tile_index(nt, nbt, i, l0 + t) : band_tile_index(nt, nbt, l0 + t, i)) * TILE2;
    };
    auto rows = [&](int t) { return Bb + int64_t(l0 + t) * TILE * ldb; };
    auto mma_stage = [&]() {
#pragma unroll 4
      for (int kk = 0; kk < TILE; kk += 4) {
        // FWD: A = L_il (row 16w+rl, col kk+kq); BWD: A = L_li^T
        const T a = FWD ? sL[(kk + kq) * LDT + 16 * w + rl] : sL[(16 * w + rl) * LDT + kk + kq];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = MF<T>::mma(a, sY[(kk + kq) * YP + 16 * q + rl], acc[q]);
      }
    };
    __syncthreads();  // rows written at the previous step are visible to every thread
    if (nl > 0) s0.load(tile(0), rows(0), ldb, c0, ncols);
    if (nl > 1) s1.load(tile(1), rows(1), ldb, c0, ncols);
    for (int t = 0; t < nl; t += 2) {
      __syncthreads();
      s0.store(sL, sY);
      if (t + 2 < nl) s0.load(tile(t + 2), rows(t + 2), ldb, c0, ncols);
      __syncthreads();
      mma_stage();
      if (t + 1 < nl) {
        __syncthreads();
        s1.store(sL, sY);
        if (t + 3 < nl) s1.load(tile(t + 3), rows(t + 3), ldb, c0, ncols);
        __syncthreads();
        mma_stage();
      }
    }
    __syncthreads();
    load_tile_lds(sL, Ib + int64_t(i) * TILE2);
    load_rows<T, CW>(sY, Bb + int64_t(i) * TILE * ldb, ldb, c0, ncols);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) sY[(16 * w + MF<T>::row(kq, v)) * YP + 16 * q + rl] -= acc[q][v];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = acc_t{0, 0, 0, 0};
#pragma unroll 4
    for (int kk = 0; kk < TILE; kk += 4) {
      const T a = FWD ? sL[(kk + kq) * LDT + 16 * w + rl] : sL[(16 * w + rl) * LDT + kk + kq];
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[q] = MF<T>::mma(a, sY[(kk + kq) * YP + 16 * q + rl], acc[q]);
    }
    T* Bi = Bb + int64_t(i) * TILE * ldb;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int col = c0 + 16 * q + rl;
      if (col < ncols) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Bi[int64_t(16 * w + MF<T>::row(kq, v)) * ldb + col] = acc[q][v];
      }
    }
  }
}

// Forward sweep X = L^{-1} B (FP64) with the band's solved tiles held in
// registers.  A workgroup takes 64 columns of one block; wave w owns columns
// 16w .. 16w + 15 and all 64 rows of every tile row.  On gfx950 the FP64 MFMA
// result layout of a 16 x 64 block column (element v of row block m on lane l
// is row 16m + 4v + l/16, column l%16) is exactly the B operand layout of the
// k-steps 16m + 4v, so each solved tile X_i stays in the wave's registers and
// feeds the products L_{i',i} X_i of the next NBT tile rows directly: only the
// factor tiles pass through LDS, staged once per workgroup in MFMA fragment
// order, double-buffered with one barrier per tile.  Step i:
//   R = B_i - sum_{l in band, l >= first} L_il X_l   (negated tiles, so the
//       products accumulate onto B_i), then X_i = L_ii^{-1} R, whose
//       fragments above the diagonal (all zero) are skipped.
// Requires nbt <= NBT for every block of the launch.  (Skipping the factor's
// zero fragments beyond the band with run-time tests measured slower: the
// branches break the schedule of the unrolled products.)
constexpr int FRAG = TILE2;  // one staged tile in fragment order
// fragment position of tile element (r, c): k-step c/4, lane (c%4)*16 + r%16, row block r/16
__device__ __forceinline__ int frag_pos(int r, int c) { return (((c >> 2) * 64 + (c & 3) * 16 + (r & 15)) << 2) + (r >> 4); }

struct SweepTile {
  double2 v[TILE2 / 512];  // 8 x 2 elements per thread
  __device__ __forceinline__ void load(const double* __restrict__ g) {
#pragma unroll
    for (int q = 0; q < TILE2 / 512; ++q) v[q] = reinterpret_cast<const double2*>(g)[threadIdx.x + 256 * q];
  }
  __device__ __forceinline__ void store(double* s, bool neg) const {
    const double sg = neg ? -1.0 : 1.0;
#pragma unroll
    for (int q = 0; q < TILE2 / 512; ++q) {
      const int e = 2 * (threadIdx.x + 256 * q), c = e >> 6, r = e & 63;
      s[frag_pos(r, c)] = sg * v[q].x;
      s[frag_pos(r + 1, c)] = sg * v[q].y;
    }
  }
};

template <int NBT, bool SPB>
__device__ __forceinline__ void trsm_fwd_reg(int nblk, const int* __restrict__ nt_arr,
                                                      const int* __restrict__ nbt_arr,
                                                      const int64_t* __restrict__ foff,
                                                      const int64_t* __restrict__ ioff,
                                                      const int64_t* __restrict__ roff, const double* __restrict__ L,
                                                      const double* __restrict__ Linv, double* __restrict__ B,
                                                      int64_t ldb, int ncols, const int* __restrict__ ncols_blk,
                                                      const int* __restrict__ first_tile, int nchunk_all,
                                                      int64_t row0, SparseRhs sp) {
  __shared__ __align__(16) double sF[2][FRAG];
  int b, chunk;
  map_block_chunk(nblk, b, chunk);
  if (b >= nblk) return;
  const int c0 = chunk * TILE;
  if (c0 >= ncols) return;
  if (ncols_blk && c0 >= ncols_blk[b]) return;
  const int nt = nt_arr[b], nbt = nbt_arr[b];
  const int first = first_tile ? min(first_tile[b * nchunk_all + chunk], nt) : 0;
  if (first >= nt) return;
  double* Bb = B + (roff[b] - row0) * ldb;
  const double* Lb = L + foff[b];
  const double* Ib = Linv + ioff[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kq = lane >> 4, col = c0 + 16 * w + (lane & 15);
  const bool cok = col < ncols;
  auto nl_of = [&](int i) { return i - max(first, i - nbt); };
  // first staged tile of step i: its farthest band tile, or the diagonal inverse when it has none
  auto first_tile_of = [&](int i, bool& neg) -> const double* {
    const int nl = nl_of(i);
    neg = nl > 0;
    return nl > 0 ? Lb + band_tile_index(nt, nbt, i, i - nl) * TILE2 : Ib + int64_t(i) * TILE2;
  };
  // SPB: this lane's column of the right-hand side as (local row, value) pairs (row -2^30: none)
  constexpr int CAP = SPB ? SPARSE_RHS_CAP : 1;
  int er[CAP];
  double ev[CAP];
#pragma unroll
  for (int e = 0; e < CAP; ++e) {
    er[e] = -(1 << 30);
    ev[e] = 0.0;
  }
  if (SPB && cok) {
    const int64_t q = int64_t(b) * sp.ld + col;
    const int ne = min(sp.cnt[q], CAP);
#pragma unroll
    for (int e = 0; e < CAP; ++e)
      if (e < ne) {
        er[e] = sp.row[q * CAP + e];
        ev[e] = sp.val[q * CAP + e];
      }
  }
  // the 16 values of this lane's column in tile row i, in MFMA result order (row block m, element v)
  auto load_b = [&](int i, double* x) {
    if constexpr (SPB) {
#pragma unroll
      for (int t = 0; t < 16; ++t) x[t] = 0.0;
      bool any = false;
#pragma unroll
      for (int e = 0; e < CAP; ++e) any |= unsigned(er[e] - TILE * i) < unsigned(TILE);
      if (__any(any)) {
#pragma unroll
        for (int e = 0; e < CAP; ++e) {
          const int r = er[e] - TILE * i;  // row 16m + 4v + kq of the tile: slot 4m + v = r / 4
          const bool hit = unsigned(r) < unsigned(TILE) && (r & 3) == kq;
          const int sl = r >> 2;
#pragma unroll
          for (int t = 0; t < 16; ++t) x[t] = (hit && sl == t) ? ev[e] : x[t];
        }
      }
    } else {
      const double* g = Bb + int64_t(i) * TILE * ldb + col;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) x[4 * m + v] = cok ? g[int64_t(16 * m + 4 * v + kq) * ldb] : 0.0;
    }
  };
  double xr[NBT][16];
#pragma unroll
  for (int s = 0; s < NBT; ++s)
#pragma unroll
    for (int e = 0; e < 16; ++e) xr[s][e] = 0.0;
  SweepTile pre;
  {
    bool neg;
    pre.load(first_tile_of(first, neg));
    pre.store(sF[0], neg);
  }
  double bcur[16];
  load_b(first, bcur);
  __syncthreads();
  int buf = 0;
  for (int i = first; i < nt; ++i) {
    const int nl = nl_of(i);
    v4d acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = v4d{bcur[4 * m], bcur[4 * m + 1], bcur[4 * m + 2], bcur[4 * m + 3]};
    // band tiles, farthest first: slot s holds X_{i-1-s}
#pragma unroll
    for (int s = NBT - 1; s >= 0; --s) {
      if (s < nl) {
        const double* nx = s > 0 ? Lb + band_tile_index(nt, nbt, i, i - s) * TILE2 : Ib + int64_t(i) * TILE2;
        pre.load(nx);
        const double* f = sF[buf];
#pragma unroll
        for (int k4 = 0; k4 < 16; ++k4) {
          const double2 a01 = reinterpret_cast<const double2*>(f + ((k4 * 64 + lane) << 2))[0];
          const double2 a23 = reinterpret_cast<const double2*>(f + ((k4 * 64 + lane) << 2))[1];
          const double bx = xr[s][k4];
          acc[0] = MF<double>::mma(a01.x, bx, acc[0]);
          acc[1] = MF<double>::mma(a01.y, bx, acc[1]);
          acc[2] = MF<double>::mma(a23.x, bx, acc[2]);
          acc[3] = MF<double>::mma(a23.y, bx, acc[3]);
        }
        pre.store(sF[buf ^ 1], s > 0);
        __syncthreads();
        buf ^= 1;
      }
    }
    // diagonal inverse: X_i = L_ii^{-1} R, R (in acc) used as the B operand
    const bool more = i + 1 < nt;
    bool nneg = false;
    if (more) {
      pre.load(first_tile_of(i + 1, nneg));
      load_b(i + 1, bcur);
    }
    v4d xn[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) xn[m] = v4d{0, 0, 0, 0};
    {
      const double* f = sF[buf];
#pragma unroll
      for (int k4 = 0; k4 < 16; ++k4) {
        const double2 a01 = reinterpret_cast<const double2*>(f + ((k4 * 64 + lane) << 2))[0];
        const double2 a23 = reinterpret_cast<const double2*>(f + ((k4 * 64 + lane) << 2))[1];
        const double bx = acc[k4 >> 2][k4 & 3];
        // L_ii^{-1} is lower triangular: fragment (m, k4) is zero for k4 >= 4m + 4
        if (k4 < 4) xn[0] = MF<double>::mma(a01.x, bx, xn[0]);
        if (k4 < 8) xn[1] = MF<double>::mma(a01.y, bx, xn[1]);
        if (k4 < 12) xn[2] = MF<double>::mma(a23.x, bx, xn[2]);
        xn[3] = MF<double>::mma(a23.y, bx, xn[3]);
      }
    }
    if (cok) {
      double* g = Bb + int64_t(i) * TILE * ldb + col;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) g[int64_t(16 * m + 4 * v + kq) * ldb] = xn[m][v];
    }
#pragma unroll
    for (int s = NBT - 1; s > 0; --s)
#pragma unroll
      for (int e = 0; e < 16; ++e) xr[s][e] = xr[s - 1][e];
#pragma unroll
    for (int e = 0; e < 16; ++e) xr[0][e] = xn[e >> 2][e & 3];
    if (more) pre.store(sF[buf ^ 1], nneg);
    __syncthreads();
    buf ^= 1;
  }
}

template <int NBT, bool SPB>
__global__ __launch_bounds__(256) void k_trsm_fwd_reg(int nblk, const int* __restrict__ nt_arr,
                                                      const int* __restrict__ nbt_arr,
                                                      const int64_t* __restrict__ foff,
                                                      const int64_t* __restrict__ ioff,
                                                      const int64_t* __restrict__ roff, const double* __restrict__ L,
                                                      const double* __restrict__ Linv, double* __restrict__ B,
                                                      int64_t ldb, int ncols, const int* __restrict__ ncols_blk,
                                                      const int* __restrict__ first_tile, int nchunk_all,
                                                      int64_t row0, SparseRhs sp) {
  trsm_fwd_reg<NBT, SPB>(nblk, nt_arr, nbt_arr, foff, ioff, roff, L, Linv, B, ldb, ncols, ncols_blk, first_tile,
                         nchunk_all, row0, sp);
}
// two-tile ring, compiled for two waves per SIMD (the narrow bands of two-dimensional subdomains)
template <bool SPB>
__global__ __launch_bounds__(256, 2) void k_trsm_fwd_reg2(int nblk, const int* __restrict__ nt_arr,
                                                          const int* __restrict__ nbt_arr,
                                                          const int64_t* __restrict__ foff,
                                                          const int64_t* __restrict__ ioff,
                                                          const int64_t* __restrict__ roff,
                                                          const double* __restrict__ L,
                                                          const double* __restrict__ Linv, double* __restrict__ B,
                                                          int64_t ldb, int ncols, const int* __restrict__ ncols_blk,
                                                          const int* __restrict__ first_tile, int nchunk_all,
                                                          int64_t row0, SparseRhs sp) {
  trsm_fwd_reg<2, SPB>(nblk, nt_arr, nbt_arr, foff, ioff, roff, L, Linv, B, ldb, ncols, ncols_blk, first_tile,
                       nchunk_all, row0, sp);
}

__global__ void k_tile_export(int nt, int nbt, int nb, const double* __restrict__ Lb, double* __restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(nb) * nb) return;
  const int c = int(idx / nb), r = int(idx % nb);
  double v = 0.0;
  if (r >= c && (r >> 6) - (c >> 6) <= nbt) v = Lb[band_elem(nt, nbt, r, c)];
  out[idx] = v;
}

__global__ void k_to_fp32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = float(a[i]);
}

template <class T, int CW>
void launch_trsm(const TileLevel& lv, T* B, int64_t ldb, int ncols, const T* L, const T* Linv, hipStream_t st) {
  const int nchunk = (ncols + CW - 1) / CW;
  const int nbp8 = (lv.nblk + 7) / 8;
  const int grid = nbp8 * 8 * nchunk;
  constexpr bool f64 = sizeof(T) == 8;
  const int fam = lv.role == 0 ? (f64 ? KF_TRSM_I64 : KF_TRSM_I32) : (f64 ? KF_TRSM_G64 : KF_TRSM_G32);
  // algorithmic work of one triangular sweep: the factor once, the rhs read + written
  const double bytes = (lv.alg_tri + 2.0 * lv.alg_rows * ncols) * sizeof(T);
  const double flops = lv.alg_sq * ncols;
  {
    KScope ks(fam, st, bytes, flops);
    k_trsm<T, CW, true><<<grid, 256, 0, st>>>(lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, L, Linv, B, ldb, ncols);
    NS_LAUNCH_CHECK();
  }
  {
    KScope ks(fam, st, bytes, flops);
    k_trsm<T, CW, false><<<grid, 256, 0, st>>>(lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, L, Linv, B, ldb, ncols);
    NS_LAUNCH_CHECK();
  }
}

// the register-ring sweep holds REG_NBT solved tiles per wave (a ring of 2 when every band of the launch is
// that narrow: fewer registers, two waves per SIMD)
constexpr int REG_NBT = 4;
int max_nbt_of(const TileLevel& lv, int b0, int b1) {
  int m = 0;
  for (int b = b0; b < b1; ++b) m = std::max(m, lv.h_nbt[b]);
  return m;
}
bool reg_sweep_ok(const TileLevel& lv, int b0, int b1) { return max_nbt_of(lv, b0, b1) <= REG_NBT; }
template <bool SPB>
void launch_fwd_reg(int ring, int grid, hipStream_t st, int nblk, const int* nt, const int* nbt, const int64_t* foff,
                    const int64_t* ioff, const int64_t* roff, const double* L, const double* Li, double* B,
                    int64_t ldb, int ncols, const int* nc, const int* ft, int nchunk_all, int64_t row0, SparseRhs sp) {
  if (ring <= 2)
    k_trsm_fwd_reg2<SPB><<<grid, 256, 0, st>>>(nblk, nt, nbt, foff, ioff, roff, L, Li, B, ldb, ncols, nc, ft,
                                               nchunk_all, row0, sp);
  else
    k_trsm_fwd_reg<REG_NBT, SPB><<<grid, 256, 0, st>>>(nblk, nt, nbt, foff, ioff, roff, L, Li, B, ldb, ncols, nc,
                                                       ft, nchunk_all, row0, sp);
}

}  // namespace

bool tile_sparse_rhs_ok(const TileLevel& lv) { return reg_sweep_ok(lv, 0, lv.nblk); }

void tile_cholesky(TileLevel& lv, int* d_err, hipStream_t st) {
  if (lv.nblk == 0) return;
  const int nbp8 = (lv.nblk + 7) / 8;
  for (int j = 0; j < lv.max_nt; ++j) {
    // tile rows j .. j + max_nbt of every block (rows outside a block's band exit at once)
    const int rows = std::min(lv.max_nt - j, lv.max_nbt + 1);
    {
      // the work is attributed per tile column as in the left-looking order (the same total)
      KScope ks(KF_CHOL_UPDATE, st, lv.chol_bytes[j], lv.chol_upd_flops[j]);
      // trailing tiles of column j - 1: rows and columns j .. j - 1 + max_nbt
      const int d = j == 0 ? 1 : std::max(1, std::min(lv.max_nbt, lv.max_nt - j));
      const int pairs = d * (d + 1) / 2;
      k_chol_step<<<pairs * nbp8 * 8, 256, 0, st>>>(j, lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.L64, lv.Linv64,
                                                    d_err);
      NS_LAUNCH_CHECK();
    }
    if (rows > 1) {
      KScope ks(KF_CHOL_PANEL, st, 0.0, lv.chol_pan_flops[j]);
      dim3 g2(rows - 1, lv.nblk);
      k_chol_panel<<<g2, 256, 0, st>>>(j, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.L64, lv.Linv64);
      NS_LAUNCH_CHECK();
    }
  }
}

void tile_make_fp32(TileLevel& lv, hipStream_t st) {
  if (lv.nblk == 0) return;
  lv.L32.alloc(lv.f_elems);
  lv.Linv32.alloc(lv.i_elems);
  k_to_fp32<<<2048, 256, 0, st>>>(lv.L64, lv.L32, lv.f_elems);
  NS_LAUNCH_CHECK();
  k_to_fp32<<<1024, 256, 0, st>>>(lv.Linv64, lv.Linv32, lv.i_elems);
  NS_LAUNCH_CHECK();
}

template <class T>
void tile_solve(const TileLevel& lv, T* B, int64_t ldb, int ncols, int cw, hipStream_t st) {
  if (lv.nblk == 0 || ncols == 0) return;
  if constexpr (sizeof(T) == 8) {
    if (ncols == 1 && trsv1_supported(lv)) {
      tile_solve1(lv, B, ldb, st);
      return;
    }
  }
  const T* L;
  const T* Li;
  if constexpr (sizeof(T) == 8) {
    L = lv.L64.p;
    Li = lv.Linv64.p;
  } else {
    L = lv.L32.p;
    Li = lv.Linv32.p;
  }
  if (cw <= 0) cw = tuned("trsm_cols", sizeof(T) == 8 ? "f64" : "f32", ncols, ncols <= 16 ? 16 : 32);
  if (cw != 16 && cw != 32 && cw != 64) cw = 32;
  if (cw == 16)
    launch_trsm<T, 16>(lv, B, ldb, ncols, L, Li, st);
  else if (cw == 32)
    launch_trsm<T, 32>(lv, B, ldb, ncols, L, Li, st);
  else
    launch_trsm<T, 64>(lv, B, ldb, ncols, L, Li, st);
}

template <class T>
void tile_solve_fwd(const TileLevel& lv, T* B, int64_t ldb, int ncols, int cw, hipStream_t st,
                    const int* ncols_blk, const int* first_tile, double alg_flops, int b0, int b1, int64_t row0,
                    int family, const SparseRhs* sparse) {
  if (b1 < 0) b1 = lv.nblk;
  const int nblk = b1 - b0;
  if (nblk <= 0 || ncols == 0) return;
  const T* L;
  const T* Li;
  if constexpr (sizeof(T) == 8) {
    L = lv.L64.p;
    Li = lv.Linv64.p;
  } else {
    L = lv.L32.p;
    Li = lv.Linv32.p;
  }
  if (cw != 16 && cw != 32) cw = 64;
  const int nbp8 = (nblk + 7) / 8;
  double tri = lv.alg_tri, rows = lv.alg_rows;
  if (b0 != 0 || b1 != lv.nblk) {  // a range of the blocks: its band entries n (w + 1) - w (w + 1) / 2 and rows
    tri = rows = 0;
    for (int b = b0; b < b1; ++b) {
      const double n = lv.h_nb[b], w = lv.h_bw[b];
      tri += n * (w + 1) - w * (w + 1) / 2;
      rows += n;
    }
  }
  const double bytes = (tri + 2.0 * rows * ncols) * sizeof(T);
  const double flops = alg_flops >= 0 ? alg_flops : (2.0 * tri - rows) * ncols;
  const int fam = family >= 0 ? family
                              : (lv.role == 0 ? (sizeof(T) == 8 ? KF_TRSM_I64 : KF_TRSM_I32)
                                              : (sizeof(T) == 8 ? KF_TRSM_G64 : KF_TRSM_G32));
  KScope ks(fam, st, bytes, flops);
  const int nchunk_all = (ncols + cw - 1) / cw;
  const int* nc = ncols_blk ? ncols_blk + b0 : nullptr;
  const int* ft = first_tile ? first_tile + int64_t(b0) * nchunk_all : nullptr;
  const int grid = nbp8 * 8 * nchunk_all;
  if constexpr (sizeof(T) == 8) {
    if (cw == 64 && reg_sweep_ok(lv, b0, b1)) {
      const int ring = max_nbt_of(lv, b0, b1);
      if (sparse)
        launch_fwd_reg<true>(ring, grid, st, nblk, lv.nt + b0, lv.nbt + b0, lv.foff + b0, lv.ioff + b0, lv.roff + b0,
                             L, Li, B, ldb, ncols, nc, ft, nchunk_all, row0, *sparse);
      else
        launch_fwd_reg<false>(ring, grid, st, nblk, lv.nt + b0, lv.nbt + b0, lv.foff + b0, lv.ioff + b0,
                              lv.roff + b0, L, Li, B, ldb, ncols, nc, ft, nchunk_all, row0, SparseRhs{});
      NS_LAUNCH_CHECK();
      return;
    }
  }
  if (sparse) fail(INVALID_ARG, "sparse right-hand side needs the 64-column FP64 register sweep");
  if (cw == 16)
    k_trsm<T, 16, true><<<grid, 256, 0, st>>>(nblk, lv.nt + b0, lv.nbt + b0, lv.foff + b0, lv.ioff + b0,
                                              lv.roff + b0, L, Li, B, ldb, ncols, nc, ft, nchunk_all, row0);
  else if (cw == 32)
    k_trsm<T, 32, true><<<grid, 256, 0, st>>>(nblk, lv.nt + b0, lv.nbt + b0, lv.foff + b0, lv.ioff + b0,
                                              lv.roff + b0, L, Li, B, ldb, ncols, nc, ft, nchunk_all, row0);
  else
    k_trsm<T, 64, true><<<grid, 256, 0, st>>>(nblk, lv.nt + b0, lv.nbt + b0, lv.foff + b0, lv.ioff + b0,
                                              lv.roff + b0, L, Li, B, ldb, ncols, nc, ft, nchunk_all, row0);
  NS_LAUNCH_CHECK();
}

template <class T>
void tile_solve_bwd(const TileLevel& lv, T* B, int64_t ldb, int ncols, int cw, hipStream_t st) {
  if (lv.nblk == 0 || ncols == 0) return;
  const T* L;
  const T* Li;
  if constexpr (sizeof(T) == 8) {
    L = lv.L64.p;
    Li = lv.Linv64.p;
  } else {
    L = lv.L32.p;
    Li = lv.Linv32.p;
  }
  if (cw != 16 && cw != 32) cw = 64;
  const int nchunk = (ncols + cw - 1) / cw;
  const int grid = (lv.nblk + 7) / 8 * 8 * nchunk;
  const bool f64 = sizeof(T) == 8;
  const int fam = lv.role == 0 ? (f64 ? KF_TRSM_I64 : KF_TRSM_I32) : (f64 ? KF_TRSM_G64 : KF_TRSM_G32);
  KScope ks(fam, st, (lv.alg_tri + 2.0 * lv.alg_rows * ncols) * sizeof(T), lv.alg_sq * ncols);
  if (cw == 16)
    k_trsm<T, 16, false><<<grid, 256, 0, st>>>(lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, L, Li, B, ldb,
                                               ncols);
  else if (cw == 32)
    k_trsm<T, 32, false><<<grid, 256, 0, st>>>(lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, L, Li, B, ldb,
                                               ncols);
  else
    k_trsm<T, 64, false><<<grid, 256, 0, st>>>(lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, L, Li, B, ldb,
                                               ncols);
  NS_LAUNCH_CHECK();
}

void tile_solve_chunks(const TileLevel& lv, double* B, int64_t ldb, int ncols, const int* first_tile,
                       hipStream_t st) {
  if (lv.nblk == 0 || ncols == 0) return;
  const int nchunk = (ncols + TILE - 1) / TILE;
  const int grid = (lv.nblk + 7) / 8 * 8 * nchunk;
  const int fam = lv.role == 0 ? KF_TRSM_I64 : KF_TRSM_G64;
  const double bytes = (lv.alg_tri + 2.0 * lv.alg_rows * ncols) * sizeof(double);
  {
    KScope ks(fam, st, bytes, lv.alg_sq * ncols);
    if (reg_sweep_ok(lv, 0, lv.nblk))
      launch_fwd_reg<false>(max_nbt_of(lv, 0, lv.nblk), grid, st, lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff,
                            lv.L64, lv.Linv64, B, ldb, ncols, nullptr, first_tile, nchunk, 0, SparseRhs{});
    else
      k_trsm<double, TILE, true><<<grid, 256, 0, st>>>(lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, lv.L64,
                                                       lv.Linv64, B, ldb, ncols, nullptr, first_tile, nchunk);
    NS_LAUNCH_CHECK();
  }
  {
    KScope ks(fam, st, bytes, lv.alg_sq * ncols);
    k_trsm<double, TILE, false><<<grid, 256, 0, st>>>(lv.nblk, lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, lv.L64,
                                                      lv.Linv64, B, ldb, ncols, nullptr, first_tile, nchunk);
    NS_LAUNCH_CHECK();
  }
}

template void tile_solve_fwd<double>(const TileLevel&, double*, int64_t, int, int, hipStream_t, const int*, const int*,
                                     double, int, int, int64_t, int, const SparseRhs*);
template void tile_solve<double>(const TileLevel&, double*, int64_t, int, int, hipStream_t);
template void tile_solve_bwd<double>(const TileLevel&, double*, int64_t, int, int, hipStream_t);
template void tile_solve_bwd<float>(const TileLevel&, float*, int64_t, int, int, hipStream_t);
template void tile_solve<float>(const TileLevel&, float*, int64_t, int, int, hipStream_t);

void tile_export(const TileLevel& lv, int block, double* out, hipStream_t st) {
  const int nb = lv.h_nb[block];
  const int64_t n2 = int64_t(nb) * nb;
  const int grid = int((n2 + 255) / 256);
  k_tile_export<<<grid, 256, 0, st>>>(lv.h_nt[block], lv.h_nbt[block], nb, lv.L64.p + lv.h_foff[block], out);
  NS_LAUNCH_CHECK();
}

void TileLevel::layout(const std::vector<int>& sizes) {
  nblk = int(sizes.size());
  h_nb = sizes;
  h_nt.resize(nblk);
  h_ioff.resize(nblk);
  h_roff.resize(nblk);
  int64_t iv = 0, r = 0;
  max_nt = 0;
  alg_rows = 0;
  for (int b = 0; b < nblk; ++b) {
    const int t = (sizes[b] + TILE - 1) / TILE;
    h_nt[b] = t;
    h_ioff[b] = iv;
    h_roff[b] = r;
    iv += int64_t(t) * TILE2;
    r += int64_t(t) * TILE;
    if (t > max_nt) max_nt = t;
    alg_rows += sizes[b];
  }
  i_elems = iv;
  nrows_pad = r;
  if (nblk == 0) return;
  nt.alloc(nblk);
  nb.alloc(nblk);
  ioff.alloc(nblk);
  roff.alloc(nblk);
  upload(nt.p, h_nt.data(), nblk * sizeof(int), alloc_stream());
  upload(nb.p, h_nb.data(), nblk * sizeof(int), alloc_stream());
  upload(ioff.p, h_ioff.data(), nblk * sizeof(int64_t), alloc_stream());
  upload(roff.p, h_roff.data(), nblk * sizeof(int64_t), alloc_stream());
}

namespace {

// sum over l in [A, B] of the number of rows r in [r0, min(U, l + bw)] (each term >= 0)
double band_rows(int64_t A, int64_t B, int64_t U, int64_t r0, int64_t bw) {
  A = std::max(A, r0 - bw);
  if (B < A || U < r0) return 0.0;
  const int64_t ls = U - bw;  // l <= ls: the column reaches row l + bw
  double s = 0.0;
  const int64_t b1 = std::min(B, ls);
  if (b1 >= A) {
    const double cnt = double(b1 - A + 1);
    s += cnt * double(A + b1) / 2.0 + cnt * double(bw - r0 + 1);
  }
  const int64_t a2 = std::max(A, ls + 1);
  if (B >= a2) s += double(B - a2 + 1) * double(U - r0 + 1);
  return s;
}

struct BandWork {
  std::vector<double> upd, pan, bytes;
  double tri = 0;
};

// Algorithmic work of the band Cholesky of an n-row block with element
// half-bandwidth bw, per tile column: updates from earlier tile columns and the
// diagonal tile's own factorisation, the panel solve below the diagonal tile,
// and every factor entry read and written once.
BandWork band_work(int n, int bw) {
  BandWork w;
  const int nt = (n + TILE - 1) / TILE;
  w.upd.assign(nt, 0.0);
  w.pan.assign(nt, 0.0);
  w.bytes.assign(nt, 0.0);
  for (int j = 0; j < nt; ++j) {
    const int64_t c0 = int64_t(j) * TILE, c1 = std::min<int64_t>(n, c0 + TILE);
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t e = std::min<int64_t>(bw, n - 1 - c) + 1;  // entries of column c
      const int64_t lo = std::max<int64_t>(0, c - bw);
      w.upd[j] += 2.0 * band_rows(lo, c0 - 1, n - 1, c, bw);
      w.upd[j] += 2.0 * band_rows(std::max(c0, lo), c - 1, c1 - 1, c, bw);
      w.pan[j] += 2.0 * band_rows(std::max(c0, lo), c - 1, n - 1, c1, bw);
      w.bytes[j] += 2.0 * e * sizeof(double);
      w.tri += double(e);
    }
  }
  return w;
}

}  // namespace

void TileLevel::layout_band(const std::vector<int>& bw) {
  h_bw.assign(nblk, 0);
  h_nbt.assign(nblk, 0);
  h_foff.assign(nblk, 0);
  int64_t f = 0;
  max_nbt = 0;
  alg_tri = alg_sq = 0;
  chol_upd_flops.assign(max_nt, 0.0);
  chol_pan_flops.assign(max_nt, 0.0);
  chol_bytes.assign(max_nt, 0.0);
  std::vector<std::pair<std::pair<int, int>, BandWork>> memo;  // work per distinct (rows, bandwidth)
  for (int b = 0; b < nblk; ++b) {
    const int n = h_nb[b];
    const int w = std::max(0, std::min(bw[b], n - 1));
    h_bw[b] = w;
    h_nbt[b] = band_tiles_for(n, w);
    h_foff[b] = f;
    f += band_col_off(h_nt[b], h_nbt[b], h_nt[b]) * TILE2;
    max_nbt = std::max(max_nbt, h_nbt[b]);
    const BandWork* bwk = nullptr;
    for (auto& m : memo)
      if (m.first.first == n && m.first.second == w) bwk = &m.second;
    if (!bwk) {
      memo.push_back({{n, w}, band_work(n, w)});
      bwk = &memo.back().second;
    }
    alg_tri += bwk->tri;
    for (int j = 0; j < h_nt[b]; ++j) {
      chol_upd_flops[j] += bwk->upd[j];
      chol_pan_flops[j] += bwk->pan[j];
      chol_bytes[j] += bwk->bytes[j];
    }
  }
  alg_sq = 2.0 * alg_tri - alg_rows;  // one triangular sweep per right-hand side
  f_elems = f;
  if (nblk == 0) return;
  nbt.alloc(nblk);
  foff.alloc(nblk);
  upload(nbt.p, h_nbt.data(), nblk * sizeof(int), alloc_stream());
  upload(foff.p, h_foff.data(), nblk * sizeof(int64_t), alloc_stream());
  L64.alloc(f_elems);
  Linv64.alloc(i_elems);
}

}  // namespace ns
