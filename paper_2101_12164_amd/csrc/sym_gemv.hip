// Single-column products with symmetric blocks in packed lower tile storage.
// A workgroup takes one stored tile A_{ti,tj} (tj <= ti) of one block, stages
// it in LDS and forms both A_{ti,tj} x_tj (row sums) and, off the diagonal,
// A_{ti,tj}^T x_ti (column sums); the results go to a partial buffer indexed by
// (row tile, contributing tile) and a second kernel sums each row's partials in
// a fixed order.  Every stored entry is read from HBM once: half the bytes of a
// product with the full blocks.
#include <cmath>

#include "ns_internal.h"

namespace ns {
namespace {

constexpr int ST = 64;  // tile size

__device__ __forceinline__ void tile_of(int u, int& ti, int& tj) {
  int t = int((sqrt(8.0 * u + 1.0) - 1.0) * 0.5);
  while ((t + 1) * (t + 2) / 2 <= u) ++t;
  while (t * (t + 1) / 2 > u) --t;
  ti = t;
  tj = u - t * (t + 1) / 2;
}

__global__ __launch_bounds__(256) void k_sym_pack(const int* __restrict__ mt, const int* __restrict__ dim,
                                                  const int64_t* __restrict__ toff, const double* __restrict__ src,
                                                  const int64_t* __restrict__ soff, const int64_t* __restrict__ sld,
                                                  double* __restrict__ tiles) {
  const int b = blockIdx.y, u = blockIdx.x;
  const int m = mt[b];
  if (u >= m * (m + 1) / 2) return;
  int ti, tj;
  tile_of(u, ti, tj);
  const int n = dim[b];
  const double* a = src + soff[b];
  const int64_t ld = sld[b];
  double* t = tiles + (toff[b] + u) * int64_t(ST * ST);
  // all sixteen loads of a thread in flight together (clamped in-bounds addresses, zero outside the block)
  double v[ST * ST / 256];
#pragma unroll
  for (int q = 0; q < ST * ST / 256; ++q) {
    const int e = threadIdx.x + 256 * q, r = ST * ti + e / ST, c = ST * tj + e % ST;
    v[q] = a[int64_t(min(r, n - 1)) * ld + min(c, n - 1)];
  }
#pragma unroll
  for (int q = 0; q < ST * ST / 256; ++q) {
    const int e = threadIdx.x + 256 * q, r = ST * ti + e / ST, c = ST * tj + e % ST;
    t[e] = (r < n && c < n) ? v[q] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_sym_tiles(const int* __restrict__ mt, const int* __restrict__ dim,
                                                   const int64_t* __restrict__ toff,
                                                   const int64_t* __restrict__ pboff,
                                                   const int64_t* __restrict__ xoff, const double* __restrict__ tiles,
                                                   const double* __restrict__ x, const int32_t* __restrict__ xidx,
                                                   double* __restrict__ part) {
  __shared__ double s[ST * (ST + 1)];
  __shared__ double xi[ST], xj[ST];
  const int b = blockIdx.y, u = blockIdx.x;
  const int m = mt[b];
  if (u >= m * (m + 1) / 2) return;
  int ti, tj;
  tile_of(u, ti, tj);
  const int n = dim[b];
  const double* t = tiles + (toff[b] + u) * int64_t(ST * ST);
  // entry r of block b's vector: x[xoff_b + r], or x[xidx[xoff_b + r]] (-1: zero) when gathered by xidx.  The
  // gather index is requested before the tile and the value after it, so the three memory round trips overlap.
  const int tid = threadIdx.x;
  const int xr = tid < ST ? ST * ti + tid : ST * tj + (tid - ST);  // threads below 2 ST: x_ti, then x_tj
  const bool xin = tid < 2 * ST && xr < n;
  const int64_t xpos = xoff[b] + min(xr, n - 1);
  int32_t src = -1;
  if (xidx && xin) src = xidx[xpos];
  double v[ST * ST / 256];
#pragma unroll
  for (int q = 0; q < ST * ST / 256; ++q) v[q] = t[tid + 256 * q];
  double xv = 0.0;
  if (xin) {
    if (!xidx)
      xv = x[xpos];
    else if (src >= 0)
      xv = x[src];
  }
#pragma unroll
  for (int q = 0; q < ST * ST / 256; ++q) {
    const int e = tid + 256 * q;
    s[(e / ST) * (ST + 1) + e % ST] = v[q];
  }
  if (tid < ST)
    xi[tid] = xv;
  else if (tid < 2 * ST)
    xj[tid - ST] = xv;
  __syncthreads();
  double* pb = part + pboff[b];
  if (threadIdx.x < ST) {  // (A x_tj) rows of tile row ti
    const int r = threadIdx.x;
    double acc = 0.0;
#pragma unroll 16
    for (int c = 0; c < ST; ++c) acc += s[r * (ST + 1) + c] * xj[c];
    pb[(int64_t(ti) * m + tj) * ST + r] = acc;
  } else if (threadIdx.x < 2 * ST && ti != tj) {  // (A^T x_ti) rows of tile row tj
    const int c = threadIdx.x - ST;
    double acc = 0.0;
#pragma unroll 16
    for (int r = 0; r < ST; ++r) acc += s[r * (ST + 1) + c] * xi[r];
    pb[(int64_t(tj) * m + ti) * ST + c] = acc;
  }
}

__global__ __launch_bounds__(256) void k_sym_reduce(const int* __restrict__ mt, const int* __restrict__ dim,
                                                    const int64_t* __restrict__ pboff,
                                                    const int64_t* __restrict__ xoff, const double* __restrict__ part,
                                                    double* __restrict__ y) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= dim[b]) return;
  const int m = mt[b];
  const double* p = part + pboff[b] + int64_t(i / ST) * m * ST + i % ST;
  double acc = 0.0;
  constexpr int U = 8;  // partials per batch: their loads are issued together (clamped), then summed in order
  for (int t0 = 0; t0 < m; t0 += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = p[int64_t(min(t0 + u, m - 1)) * ST];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (t0 + u < m) acc += v[u];
  }
  y[xoff[b] + i] = acc;
}

}  // namespace

void sym_layout(SymPacked& sp, const std::vector<int>& dims, const int64_t* xoff, hipStream_t st) {
  const int nb = int(dims.size());
  sp.nblk = nb;
  sp.xoff = xoff;
  std::vector<int> hmt(nb);
  std::vector<int64_t> htoff(nb), hpb(nb);
  int64_t tt = 0, pp = 0;
  sp.max_tiles = 0;
  sp.max_mt = 0;
  sp.alg_bytes = sp.alg_flops = 0;
  for (int b = 0; b < nb; ++b) {
    const int m = (dims[b] + ST - 1) / ST;
    hmt[b] = m;
    htoff[b] = tt;
    hpb[b] = pp;
    tt += int64_t(m) * (m + 1) / 2;
    pp += int64_t(m) * m * ST;
    sp.max_tiles = std::max(sp.max_tiles, m * (m + 1) / 2);
    sp.max_mt = std::max(sp.max_mt, m);
    sp.alg_bytes += 0.5 * double(dims[b]) * (dims[b] + 1) * sizeof(double);
    sp.alg_flops += 2.0 * double(dims[b]) * dims[b];
  }
  sp.total_tiles = tt;
  if (nb == 0 || tt == 0) return;
  if (nb > 65535) fail(INVALID_ARG, "too many blocks for the packed symmetric product");
  sp.mt.alloc(nb);
  sp.dim.alloc(nb);
  sp.toff.alloc(nb);
  sp.pboff.alloc(nb);
  upload(sp.mt.p, hmt.data(), nb * sizeof(int), st);
  upload(sp.dim.p, dims.data(), nb * sizeof(int), st);
  upload(sp.toff.p, htoff.data(), nb * sizeof(int64_t), st);
  upload(sp.pboff.p, hpb.data(), nb * sizeof(int64_t), st);
  sp.tiles.alloc(size_t(tt) * ST * ST);
  sp.part.alloc(size_t(pp));
}

void sym_pack(SymPacked& sp, const std::vector<int>& dims, const double* src, const int64_t* src_off,
              const int64_t* src_ld, const int64_t* xoff, hipStream_t st) {
  sym_layout(sp, dims, xoff, st);
  if (sp.nblk == 0 || sp.total_tiles == 0) return;
  k_sym_pack<<<dim3(unsigned(sp.max_tiles), unsigned(sp.nblk)), 256, 0, st>>>(sp.mt, sp.dim, sp.toff, src, src_off,
                                                                              src_ld, sp.tiles);
  NS_LAUNCH_CHECK();
}

void sym_gemv(const SymPacked& sp, const double* x, double* y, hipStream_t st, const int32_t* xidx) {
  if (sp.nblk == 0 || sp.total_tiles == 0) return;
  k_sym_tiles<<<dim3(unsigned(sp.max_tiles), unsigned(sp.nblk)), 256, 0, st>>>(sp.mt, sp.dim, sp.toff, sp.pboff,
                                                                               sp.xoff, sp.tiles, x, xidx, sp.part);
  NS_LAUNCH_CHECK();
  k_sym_reduce<<<dim3(unsigned((sp.max_mt * ST + 255) / 256), unsigned(sp.nblk)), 256, 0, st>>>(
      sp.mt, sp.dim, sp.pboff, sp.xoff, sp.part, y);
  NS_LAUNCH_CHECK();
}

}  // namespace ns
