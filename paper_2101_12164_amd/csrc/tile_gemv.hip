// Single right-hand-side triangular solves with the interior Cholesky factors
// (the solves of the block LDL^T reduction and back-substitution, eq. A_LDLT)
// and explicit inverses of the small interface blocks used by the exact
// A_Gamma solve.
//
// The single-column sweeps are bandwidth bound: one 1024-thread workgroup per
// block keeps the block's solution in LDS and its 16 waves stream the factor
// tiles of the current tile column in parallel.  The forward sweep updates the
// rows below (tile (l, i) read column-major: lane r, coalesced); the backward
// sweep forms the dot products with a transposed copy of the same tiles so that
// its loads are coalesced as well.
#include "ns_internal.h"

namespace ns {
namespace {

constexpr int NW = 16;  // waves per workgroup
constexpr int NTH = NW * 64;
constexpr int LDT = TILE + 1;

// The sweeps walk the tile rows of a block in order; each step is a short chain of barriers, so the loads of
// step i + 1 (the diagonal inverse and the band tiles of the next tile column, which do not depend on the
// solution) are issued during step i and held in registers.  The nbt band tiles of a step are cut into
// (tile, 16-column chunk) items, one per wave (rounds of NW items when nbt > NW / 4), so every wave loads
// 16 + 4 values per step; partial sums are combined in a fixed order.
constexpr int CH = TILE / 4;  // columns (rows) of a band tile per item

// Forward: y = L^{-1} b (b, y in B with stride ldb, one column).
__global__ __launch_bounds__(NTH) void k_trsv_fwd(const int* __restrict__ nt_arr, const int* __restrict__ nbt_arr,
                                                  const int64_t* __restrict__ foff,
                                                  const int64_t* __restrict__ ioff, const int64_t* __restrict__ roff,
                                                  const double* __restrict__ L, const double* __restrict__ Linv,
                                                  double* __restrict__ B, int64_t ldb) {
  extern __shared__ double yv[];  // npad values of this block
  __shared__ double red[NW * 64];
  const int b = blockIdx.x;
  const int nt = nt_arr[b], nbt = nbt_arr[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* Bb = B + roff[b] * ldb;
  const double* Lb = L + foff[b];
  const double* Ib = Linv + ioff[b];
  for (int e = threadIdx.x; e < nt * TILE; e += NTH) yv[e] = Bb[int64_t(e) * ldb];
  // step i's operands of wave w: columns 4w .. 4w + 3 of Linv_ii (element (lane, c)) and item w of round 0:
  // tile L_{i+1+w/4, i}, columns 16 (w % 4) .. + 15
  double li[4], tt[CH];
  auto load_step = [&](int i, double* l4, double* t16) {
    const double* Li = Ib + int64_t(i) * TILE2;
#pragma unroll
    for (int c = 0; c < 4; ++c) l4[c] = Li[(4 * w + c) * TILE + lane];
    const int nl = min(nt - 1 - i, nbt);
    if (w < 4 * nl) {
      const double* T = Lb + (band_tile_index(nt, nbt, i, i) + 1 + (w >> 2)) * TILE2 + (CH * (w & 3)) * TILE;
#pragma unroll
      for (int c = 0; c < CH; ++c) t16[c] = T[c * TILE + lane];
    }
  };
  if (nt > 0) load_step(0, li, tt);
  __syncthreads();
  for (int i = 0; i < nt; ++i) {
    // y_i = Linv_ii * acc_i: wave w sums columns [4w, 4w + 4)
    double p = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) p += li[c] * yv[i * TILE + 4 * w + c];
    red[w * 64 + lane] = p;
    double lin[4], ttn[CH];
    if (i + 1 < nt) load_step(i + 1, lin, ttn);
    __syncthreads();
    if (threadIdx.x < 64) {
      double y = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) y += red[q * 64 + threadIdx.x];
      yv[i * TILE + threadIdx.x] = y;
    }
    __syncthreads();
    // acc_l -= L_li y_i for i < l <= i + nbt, NW items (4 tiles) per round
    const int nl = min(nt - 1 - i, nbt);
    for (int r0 = 0; r0 < 4 * nl; r0 += NW) {
      const int item = r0 + w;
      double s = 0.0;
      if (item < 4 * nl) {
        const double* yi = yv + i * TILE + CH * (item & 3);
        if (r0 == 0) {
#pragma unroll
          for (int c = 0; c < CH; ++c) s += tt[c] * yi[c];
        } else {
          const double* T =
              Lb + (band_tile_index(nt, nbt, i, i) + 1 + (item >> 2)) * TILE2 + (CH * (item & 3)) * TILE;
#pragma unroll
          for (int c = 0; c < CH; ++c) s += T[c * TILE + lane] * yi[c];
        }
      }
      red[w * 64 + lane] = s;
      __syncthreads();
      if (threadIdx.x < 4 * 64) {
        const int t = (r0 >> 2) + (threadIdx.x >> 6);
        if (t < nl) {
          const double* rq = red + (threadIdx.x >> 6) * 4 * 64 + lane;
          yv[(i + 1 + t) * TILE + lane] -= (rq[0] + rq[64]) + (rq[128] + rq[192]);
        }
      }
      __syncthreads();
    }
    if (i + 1 < nt) {
#pragma unroll
      for (int c = 0; c < 4; ++c) li[c] = lin[c];
#pragma unroll
      for (int c = 0; c < CH; ++c) tt[c] = ttn[c];
    }
  }
  for (int e = threadIdx.x; e < nt * TILE; e += NTH) Bb[int64_t(e) * ldb] = yv[e];
}

// Backward: x = L^{-T} y, dot products with the transposed tiles LT (row-major copies: element (r, c) of
// L_li at r * TILE + c), items (tile, 16-row chunk); x_i = Linv_ii^T t with wave w summing rows 4w .. 4w + 3.
__global__ __launch_bounds__(NTH) void k_trsv_bwd(const int* __restrict__ nt_arr, const int* __restrict__ nbt_arr,
                                                  const int64_t* __restrict__ foff,
                                                  const int64_t* __restrict__ ioff, const int64_t* __restrict__ roff,
                                                  const double* __restrict__ LT, const double* __restrict__ Linv,
                                                  double* __restrict__ B, int64_t ldb) {
  extern __shared__ double yv[];
  __shared__ double red[NW * 64];
  __shared__ double tv[TILE];
  const int b = blockIdx.x;
  const int nt = nt_arr[b], nbt = nbt_arr[b];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* Bb = B + roff[b] * ldb;
  const double* Lb = LT + foff[b];
  const double* Ib = Linv + ioff[b];
  for (int e = threadIdx.x; e < nt * TILE; e += NTH) yv[e] = Bb[int64_t(e) * ldb];
  // step i's operands of wave w: Linv_ii(4w + k, lane) for k < 4 and item w of round 0: rows
  // 16 (w % 4) .. + 15 of L_{i+1+w/4, i}
  double li[4], tt[CH];
  auto load_step = [&](int i, double* l4, double* t16) {
    const double* Li = Ib + int64_t(i) * TILE2;
#pragma unroll
    for (int k = 0; k < 4; ++k) l4[k] = Li[lane * TILE + 4 * w + k];
    const int nl = min(nt - 1 - i, nbt);
    if (w < 4 * nl) {
      const double* T = Lb + (band_tile_index(nt, nbt, i, i) + 1 + (w >> 2)) * TILE2 + (CH * (w & 3)) * TILE;
#pragma unroll
      for (int r = 0; r < CH; ++r) t16[r] = T[r * TILE + lane];
    }
  };
  if (nt > 0) load_step(nt - 1, li, tt);
  __syncthreads();
  for (int i = nt - 1; i >= 0; --i) {
    // t = y_i - sum_{l>i} L_li^T x_l, NW items per round, summed in item order by threads 0-63
    const int nl = min(nt - 1 - i, nbt);
    double lin[4], ttn[CH];
    if (i > 0) load_step(i - 1, lin, ttn);
    double tacc = 0.0;
    for (int r0 = 0; r0 < 4 * nl; r0 += NW) {
      const int item = r0 + w;
      double s = 0.0;
      if (item < 4 * nl) {
        const double* xl = yv + (i + 1 + (item >> 2)) * TILE + CH * (item & 3);
        if (r0 == 0) {
#pragma unroll
          for (int r = 0; r < CH; ++r) s += tt[r] * xl[r];
        } else {
          const double* T =
              Lb + (band_tile_index(nt, nbt, i, i) + 1 + (item >> 2)) * TILE2 + (CH * (item & 3)) * TILE;
#pragma unroll
          for (int r = 0; r < CH; ++r) s += T[r * TILE + lane] * xl[r];
        }
      }
      red[w * 64 + lane] = s;
      __syncthreads();
      if (threadIdx.x < 64) {
#pragma unroll
        for (int q = 0; q < NW; ++q) tacc += red[q * 64 + threadIdx.x];
      }
      __syncthreads();
    }
    if (threadIdx.x < 64) tv[threadIdx.x] = yv[i * TILE + threadIdx.x] - tacc;
    __syncthreads();
    // x_i = Linv_ii^T t : out[c] = sum_r Linv[r][c] t[r]
    double p = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) p += li[k] * tv[4 * w + k];
    red[w * 64 + lane] = p;
    __syncthreads();
    if (threadIdx.x < 64) {
      double x = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) x += red[q * 64 + threadIdx.x];
      yv[i * TILE + threadIdx.x] = x;
    }
    __syncthreads();
    if (i > 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) li[k] = lin[k];
#pragma unroll
      for (int r = 0; r < CH; ++r) tt[r] = ttn[r];
    }
  }
  for (int e = threadIdx.x; e < nt * TILE; e += NTH) Bb[int64_t(e) * ldb] = yv[e];
}

// LT = tile-wise transpose of L (every tile of the level).
__global__ __launch_bounds__(256) void k_transpose_tiles(int64_t ntiles, const double* __restrict__ L,
                                                         double* __restrict__ LT) {
  __shared__ double s[TILE * LDT];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const double* src = L + t * TILE2;
    double* dst = LT + t * TILE2;
    for (int e = threadIdx.x; e < TILE2; e += 256) s[(e >> 6) * LDT + (e & 63)] = src[e];  // (r = e&63, c = e>>6)
    __syncthreads();
    for (int e = threadIdx.x; e < TILE2; e += 256) dst[e] = s[(e & 63) * LDT + (e >> 6)];  // row-major (r = e>>6)
    __syncthreads();
  }
}

// Identity right-hand side for explicit inverses: E (rows x ld), block b rows
// roff_b .. + npad_b get e_{row - roff_b}.
__global__ void k_identity_blocks(const int* __restrict__ nt_arr, const int64_t* __restrict__ roff,
                                  double* __restrict__ E, int64_t ld) {
  const int b = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nt_arr[b] * TILE) E[(roff[b] + r) * ld + r] = 1.0;
}

__global__ void k_to_fp32_g(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = float(a[i]);
}

}  // namespace

bool trsv1_supported_size(const TileLevel& lv) { return size_t(lv.max_nt) * TILE * sizeof(double) <= 96 * 1024; }

bool trsv1_supported(const TileLevel& lv) { return lv.LT64.p != nullptr && trsv1_supported_size(lv); }

void tile_make_transposed(TileLevel& lv, hipStream_t st) {
  if (lv.nblk == 0) return;
  lv.LT64.alloc(lv.f_elems);
  const int64_t ntiles = lv.f_elems / TILE2;
  k_transpose_tiles<<<unsigned(std::min<int64_t>(ntiles, 8192)), 256, 0, st>>>(ntiles, lv.L64, lv.LT64);
  NS_LAUNCH_CHECK();
}

void tile_solve1(const TileLevel& lv, double* B, int64_t ldb, hipStream_t st) {
  const size_t lds = size_t(lv.max_nt) * TILE * sizeof(double);
  const double bytes = (lv.alg_tri + 2.0 * lv.alg_rows) * sizeof(double);
  const int fam = lv.role == 0 ? KF_TRSM_I64 : KF_TRSM_G64;
  {
    KScope ks(fam, st, bytes, lv.alg_sq);
    k_trsv_fwd<<<lv.nblk, NTH, lds, st>>>(lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, lv.L64, lv.Linv64, B, ldb);
    NS_LAUNCH_CHECK();
  }
  {
    KScope ks(fam, st, bytes, lv.alg_sq);
    k_trsv_bwd<<<lv.nblk, NTH, lds, st>>>(lv.nt, lv.nbt, lv.foff, lv.ioff, lv.roff, lv.LT64, lv.Linv64, B, ldb);
    NS_LAUNCH_CHECK();
  }
}

void tile_make_inverse(TileLevel& lv, bool fp32, hipStream_t st) {
  if (lv.nblk == 0) return;
  const int maxpad = lv.max_nt * TILE;
  lv.inv_ld = maxpad;
  std::vector<int64_t> aoff(lv.nblk), lda(lv.nblk, maxpad);
  std::vector<int> np(lv.nblk);
  for (int b = 0; b < lv.nblk; ++b) {
    aoff[b] = lv.h_roff[b] * maxpad;
    np[b] = lv.h_nt[b] * TILE;
  }
  lv.inv_off.alloc(lv.nblk);
  lv.inv_lda.alloc(lv.nblk);
  lv.npad_d.alloc(lv.nblk);
  upload(lv.inv_off.p, aoff.data(), lv.nblk * sizeof(int64_t), st);
  upload(lv.inv_lda.p, lda.data(), lv.nblk * sizeof(int64_t), st);
  upload(lv.npad_d.p, np.data(), lv.nblk * sizeof(int), st);
  // Y_b = L_b^{-1}: forward sweep on the identity.  Column chunk c is zero above tile row c * cw / TILE
  // and stays so, so its sweep starts there; narrower chunks when few blocks would leave the device idle.
  int cw = 64;
  while (cw > 16 && int64_t(lv.nblk) * ((maxpad + cw - 1) / cw) < 512) cw /= 2;
  const int nchunk = (maxpad + cw - 1) / cw;
  std::vector<int> ft(size_t(lv.nblk) * nchunk), kst(size_t(lv.nblk) * lv.max_nt);
  double fl_fwd = 0, fl_gram = 0;
  for (int b = 0; b < lv.nblk; ++b) {
    for (int c = 0; c < nchunk; ++c) ft[size_t(b) * nchunk + c] = c * cw / TILE;
    for (int t = 0; t < lv.max_nt; ++t) kst[size_t(b) * lv.max_nt + t] = t;
    const double n = np[b];
    fl_fwd += n * n * n / 3.0;   // column c of the identity: (n - c)^2 flops on a dense factor
    fl_gram += n * n * n / 3.0;  // lower half of Y^T Y over the nonzero rows
  }
  DBuf<int> ftd, kstd;
  ftd.alloc(ft.size());
  kstd.alloc(kst.size());
  upload(ftd.p, ft.data(), ft.size() * sizeof(int), st);
  upload(kstd.p, kst.data(), kst.size() * sizeof(int), st);
  DBuf<double> Y;
  Y.alloc(lv.nrows_pad * maxpad);
  NS_HIP(hipMemsetAsync(Y.p, 0, lv.nrows_pad * maxpad * sizeof(double), st));
  k_identity_blocks<<<dim3((maxpad + 255) / 256, lv.nblk), 256, 0, st>>>(lv.nt, lv.roff, Y.p, maxpad);
  NS_LAUNCH_CHECK();
  tile_solve_fwd<double>(lv, Y.p, maxpad, maxpad, cw, st, lv.npad_d.p, ftd.p, fl_fwd);
  // A_b^{-1} = L_b^{-T} L_b^{-1} = Y_b^T Y_b (lower tiles formed, mirrored)
  lv.Ainv64.alloc(lv.nrows_pad * maxpad);
  NS_HIP(hipMemsetAsync(lv.Ainv64.p, 0, lv.nrows_pad * maxpad * sizeof(double), st));
  tri_gram(lv, Y.p, lv.Ainv64.p, maxpad, kstd.p, lv.max_nt, fl_gram, st);
  std::vector<int> dims(lv.nblk);
  for (int b = 0; b < lv.nblk; ++b) dims[b] = lv.h_nt[b] * TILE;
  sym_pack(lv.inv_sym, dims, lv.Ainv64.p, lv.inv_off.p, lv.inv_lda.p, lv.roff.p, st);
  if (fp32) {
    lv.Ainv32.alloc(lv.Ainv64.n);
    k_to_fp32_g<<<2048, 256, 0, st>>>(lv.Ainv64, lv.Ainv32, lv.Ainv64.n);
    NS_LAUNCH_CHECK();
  }
}

}  // namespace ns
