// Sparse and index kernels: the DBBD extraction of eq. (perm_A) on the device,
// the CSR products A_IGamma X, A_GammaI T, A_Gamma X, and the operators built
// from them: the Schur complement S_Gamma (eq. schur_complement), the exact
// A_Gamma solve through the interface split, and the interior solve A_I^{-1}.
#include "ns_handle.h"

namespace ns {
namespace {

constexpr int F_STRUCT = 0, F_NAN = 1, F_ASYM = 2, F_DBBD1 = 3, F_DBBD2 = 4;

// ----------------------------------------------------------------- products
// Threads per row (TPR) cover the columns of a row-major block.

template <class T, int TPR>
__global__ __launch_bounds__(256) void k_spmm(int64_t nrows, const int64_t* __restrict__ ptr,
                                              const int32_t* __restrict__ col, const T* __restrict__ val,
                                              const T* __restrict__ X, int64_t ldx, T* __restrict__ Y, int64_t ldy,
                                              int ncols) {
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  const int64_t e0 = ptr[row], e1 = ptr[row + 1];
  for (int c = lane; c < ncols; c += TPR) {
    T acc = T(0);
    for (int64_t e = e0; e < e1; ++e) acc += val[e] * X[int64_t(col[e]) * ldx + c];
    Y[row * ldy + c] = acc;
  }
}

// Y = A_Gamma X - A_GammaI Tb   (or Y = A_GammaI Tb when w_only)
template <class T, int TPR>
__global__ __launch_bounds__(256) void k_schur_epi(int64_t nrows, const int64_t* __restrict__ pG,
                                                   const int32_t* __restrict__ cG, const T* __restrict__ vG,
                                                   const T* __restrict__ X, int64_t ldx,
                                                   const int64_t* __restrict__ pI, const int32_t* __restrict__ cI,
                                                   const T* __restrict__ vI, const T* __restrict__ Tb, int64_t ldt,
                                                   T* __restrict__ Y, int64_t ldy, int ncols, int w_only) {
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  for (int c = lane; c < ncols; c += TPR) {
    T a = T(0), w = T(0);
    if (!w_only) csr_row_visit(pG[row], pG[row + 1], cG, vG, X, ldx, c, [&](T v, T x) { a += v * x; });
    csr_row_visit(pI[row], pI[row + 1], cI, vI, Tb, ldt, c, [&](T v, T x) { w += v * x; });
    Y[row * ldy + c] = w_only ? w : a - w;
  }
}

// Out[r] = (src[r] >= 0 ? R[src[r]] : 0) - sum_e val[e] X[col[e]]   (CSR optional)
template <class T, int TPR>
__global__ __launch_bounds__(256) void k_gather_sub(int64_t nrows, const int32_t* __restrict__ src,
                                                    const T* __restrict__ R, int64_t ldr,
                                                    const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                    const T* __restrict__ val, const T* __restrict__ X, int64_t ldx,
                                                    T* __restrict__ Out, int64_t ldo, int ncols) {
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  const int s = src ? src[row] : int(row);
  for (int c = lane; c < ncols; c += TPR) {
    T acc = s >= 0 ? R[int64_t(s) * ldr + c] : T(0);
    if (ptr) csr_row_visit(ptr[row], ptr[row + 1], col, val, X, ldx, c, [&](T v, T x) { acc -= v * x; });
    Out[row * ldo + c] = acc;
  }
}

// The same for 17..256 columns: one row per wave, lane l owns the columns l + 64 g (g < CPL); the row of R and
// each batch of four CSR entries issue all their loads before the first use.  Same sums in the same order.
template <class T, int CPL, int TPR = 64>
__global__ __launch_bounds__(256) void k_gather_sub_wide(int64_t nrows, const int32_t* __restrict__ src,
                                                         const T* __restrict__ R, int64_t ldr,
                                                         const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col, const T* __restrict__ val,
                                                         const T* __restrict__ X, int64_t ldx, T* __restrict__ Out,
                                                         int64_t ldo, int ncols) {
  // TPR threads per row (64 / TPR rows per wave: their chains of dependent loads overlap)
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  int cc[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) cc[g] = min(lane + TPR * g, ncols - 1);
  const int s = src ? src[row] : int(row);
  T acc[CPL];
  if (s >= 0) {
#pragma unroll
    for (int g = 0; g < CPL; ++g) acc[g] = R[int64_t(s) * ldr + cc[g]];
  } else {
#pragma unroll
    for (int g = 0; g < CPL; ++g) acc[g] = T(0);
  }
  if (ptr) {
    const int64_t e0 = ptr[row], e1 = ptr[row + 1];
    for (int64_t e = e0; e < e1; e += 4) {
      int j[4];
      T v[4], x[4][CPL];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t ek = e + k < e1 ? e + k : e;
        j[k] = col[ek];
        v[k] = val[ek];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int g = 0; g < CPL; ++g) x[k][g] = X[int64_t(j[k]) * ldx + cc[g]];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (e + k < e1)
#pragma unroll
          for (int g = 0; g < CPL; ++g) acc[g] -= v[k] * x[k][g];
    }
  }
#pragma unroll
  for (int g = 0; g < CPL; ++g) {
    const int c = lane + TPR * g;
    if (c < ncols) Out[row * ldo + c] = acc[g];
  }
}

// Out[dst[r]] = B[r] for dst[r] >= 0
template <class T, class U, int TPR>
__global__ __launch_bounds__(256) void k_scatter(int64_t nrows, const int32_t* __restrict__ dst,
                                                 const T* __restrict__ B, int64_t ldb, U* __restrict__ Out,
                                                 int64_t ldo, int ncols) {
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (row >= nrows) return;
  const int d = dst[row];
  if (d < 0) return;
  for (int c = lane; c < ncols; c += TPR) Out[int64_t(d) * ldo + c] = U(B[row * ldb + c]);
}

// Two scatters in one launch: rows [0, n1) of B1 through dst1, then rows [0, n2) of B2 through dst2
template <class T, int TPR>
__global__ __launch_bounds__(256) void k_scatter2(int64_t n1, const int32_t* __restrict__ dst1, const T* __restrict__ B1,
                                                  int64_t n2, const int32_t* __restrict__ dst2, const T* __restrict__ B2,
                                                  int64_t ldb, T* __restrict__ Out, int64_t ldo, int ncols) {
  int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  const int32_t* dst = dst1;
  const T* B = B1;
  if (row >= n1) {
    row -= n1;
    if (row >= n2) return;
    dst = dst2;
    B = B2;
  }
  const int d = dst[row];
  if (d < 0) return;
  for (int c = lane; c < ncols; c += TPR) Out[int64_t(d) * ldo + c] = B[row * ldb + c];
}

// C[q] = (A_sJ Y)[rows[q]] on the listed level-2 rows; TPR lanes per row, lane l holding the columns l + TPR g.
template <class T, int TPR, int CPL>
__global__ __launch_bounds__(256) void k_l2c_rows(int64_t nq, const int32_t* __restrict__ rows,
                                                  const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ Y, int64_t ldy,
                                                  T* __restrict__ C, int ncols) {
  const int64_t q = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  if (q >= nq) return;
  int cc[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) cc[g] = min(lane + TPR * g, ncols - 1);
  T acc[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) acc[g] = T(0);
  const int r = rows[q];
  for (int64_t e = ptr[r], e1 = ptr[r + 1]; e < e1; ++e) {
    const int64_t j = col[e];
    const T v = val[e];
#pragma unroll
    for (int g = 0; g < CPL; ++g) acc[g] += v * Y[j * ldy + cc[g]];
  }
#pragma unroll
  for (int g = 0; g < CPL; ++g) {
    const int c = lane + TPR * g;
    if (c < ncols) C[q * ncols + c] = acc[g];
  }
}

// The last step of an A_Gamma solve: Out[jsrc[i]] = yJ[i] on the junction rows and, on the level-2 rows,
// Out[l2src[r]] = xs[r] - sum over the listed rows k of r's block b of (A_b^{-1})(k, r) C[k], where xs is
// A_s^{-1} applied to the level-2 right-hand side alone and C = A_sJ y_J on the listed rows: by linearity
// A_s^{-1} (r_s - A_sJ y_J), with A_s^{-1} A_sJ y_J reduced to the few columns of A_s^{-1} that A_sJ reaches.
// The coefficients of row r sit at coef[r w + u] (k_l2c_coef), rinf[r] = (first listed row, count).  TPR lanes
// per row, lane l holding the columns l + TPR g; four listed rows at a time, their loads issued together.
template <class T, int TPR, int CPL>
__global__ __launch_bounds__(256) void k_scatter_l2c(int64_t nJ, const int32_t* __restrict__ jsrc,
                                                     const T* __restrict__ yJ, int64_t n2,
                                                     const int32_t* __restrict__ l2src, const T* __restrict__ xs,
                                                     const int2* __restrict__ rinf, const T* __restrict__ coef, int w,
                                                     const T* __restrict__ C, T* __restrict__ Out, int64_t ldo,
                                                     int ncols) {
  int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / TPR;
  const int lane = threadIdx.x % TPR;
  int cc[CPL];
#pragma unroll
  for (int g = 0; g < CPL; ++g) cc[g] = min(lane + TPR * g, ncols - 1);
  T v[CPL];
  int d;
  if (row < nJ) {
    d = jsrc[row];
#pragma unroll
    for (int g = 0; g < CPL; ++g) v[g] = yJ[row * ncols + cc[g]];
    if (d < 0) return;
  } else {
    row -= nJ;
    if (row >= n2) return;
    d = l2src[row];
    const int2 ri = rinf[row];
#pragma unroll
    for (int g = 0; g < CPL; ++g) v[g] = xs[row * ncols + cc[g]];
    if (d < 0) return;
    const T* cr = coef + row * w;
    for (int u = 0; u < ri.y; u += 4) {
      T a[4], cv[4][CPL];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int uk = u + k < ri.y ? u + k : u;
        a[k] = cr[uk];
#pragma unroll
        for (int g = 0; g < CPL; ++g) cv[k][g] = C[int64_t(ri.x + uk) * ncols + cc[g]];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (u + k < ri.y)
#pragma unroll
          for (int g = 0; g < CPL; ++g) v[g] -= a[k] * cv[k][g];
    }
  }
#pragma unroll
  for (int g = 0; g < CPL; ++g) {
    const int c = lane + TPR * g;
    if (c < ncols) Out[int64_t(d) * ldo + c] = v[g];
  }
}

// coef[r w + u] = (A_b^{-1})(k_u, r) for the listed rows k_u of the block b of padded level-2 row r (zero past
// their count), rinf[r] = (first listed row of b, count) when rinf is given.
template <class T>
__global__ void k_l2c_coef(int64_t n2, const int32_t* __restrict__ blk, const int64_t* __restrict__ roff,
                           const int64_t* __restrict__ inv_off, const int64_t* __restrict__ inv_lda,
                           const T* __restrict__ Ainv, const int32_t* __restrict__ off,
                           const int32_t* __restrict__ rows, int w, T* __restrict__ coef, int2* __restrict__ rinf) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n2) return;
  const int b = blk[r];
  const int64_t r0 = roff[b], m = r - r0;
  const int q0 = off[b], nq = off[b + 1] - q0;
  if (rinf) rinf[r] = make_int2(q0, nq);
  for (int u = 0; u < w; ++u)
    coef[r * w + u] = u < nq ? Ainv[inv_off[b] + (int64_t(rows[q0 + u]) - r0) * inv_lda[b] + m] : T(0);
}

template <int TPR>
inline int grid_rows(int64_t nrows) {
  return int((nrows * TPR + 255) / 256);
}

#define NS_TPR_DISPATCH(ncols, BODY)      \
  do {                                    \
    if ((ncols) == 1) {                   \
      constexpr int TPR = 1;              \
      BODY;                               \
    } else if ((ncols) <= 4) {            \
      constexpr int TPR = 4;              \
      BODY;                               \
    } else if ((ncols) <= 16) {           \
      constexpr int TPR = 16;             \
      BODY;                               \
    } else {                              \
      constexpr int TPR = 64;             \
      BODY;                               \
    }                                     \
  } while (0)

template <class T>
const T* csr_vals(const Csr& A) {
  if constexpr (sizeof(T) == 8)
    return A.val64.p;
  else
    return A.val32.p;
}

template <class T>
void spmm(const Csr& A, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, hipStream_t st) {
  if (A.nrows == 0 || ncols == 0) return;
  KScope ks(KF_SPMM, st);
  NS_TPR_DISPATCH(ncols, (k_spmm<T, TPR><<<grid_rows<TPR>(A.nrows), 256, 0, st>>>(
                              A.nrows, A.ptr, A.col, csr_vals<T>(A), X, ldx, Y, ldy, ncols)));
  NS_LAUNCH_CHECK();
}

template <class T>
void gather_sub(int64_t nrows, const int32_t* src, const T* R, int64_t ldr, const Csr* A, const T* X, int64_t ldx,
                T* Out, int64_t ldo, int ncols, hipStream_t st) {
  if (nrows == 0 || ncols == 0) return;
  const int64_t* p = A && A->nnz ? A->ptr.p : nullptr;
  const int32_t* c = A ? A->col.p : nullptr;
  const T* v = A ? csr_vals<T>(*A) : nullptr;
  if (ncols > 16 && ncols <= 256) {
    auto wide = [&](auto cpl, auto tpr) {
      constexpr int CPL = decltype(cpl)::value, TPR = decltype(tpr)::value;
      k_gather_sub_wide<T, CPL, TPR><<<grid_rows<TPR>(nrows), 256, 0, st>>>(nrows, src, R, ldr, p, c, v, X, ldx,
                                                                            Out, ldo, ncols);
    };
    using T64 = std::integral_constant<int, 64>;
    using T16 = std::integral_constant<int, 16>;
    const bool many = nrows >= 16384;  // four rows per wave (a few thousand rows keep one per wave)
    if (many && ncols <= 80)
      wide(std::integral_constant<int, 5>(), T16());
    else if (many && ncols <= 160)
      wide(std::integral_constant<int, 10>(), T16());
    else if (ncols <= 64)
      wide(std::integral_constant<int, 1>(), T64());
    else if (ncols <= 128)
      wide(std::integral_constant<int, 2>(), T64());
    else if (ncols <= 192)
      wide(std::integral_constant<int, 3>(), T64());
    else
      wide(std::integral_constant<int, 4>(), T64());
  } else {
    NS_TPR_DISPATCH(ncols, (k_gather_sub<T, TPR><<<grid_rows<TPR>(nrows), 256, 0, st>>>(
                                nrows, src, R, ldr, p, c, v, X, ldx, Out, ldo, ncols)));
  }
  NS_LAUNCH_CHECK();
}

template <class T, class U>
void scatter(int64_t nrows, const int32_t* dst, const T* B, int64_t ldb, U* Out, int64_t ldo, int ncols,
             hipStream_t st) {
  if (nrows == 0 || ncols == 0) return;
  NS_TPR_DISPATCH(ncols, (k_scatter<T, U, TPR><<<grid_rows<TPR>(nrows), 256, 0, st>>>(nrows, dst, B, ldb, Out, ldo,
                                                                                          ncols)));
  NS_LAUNCH_CHECK();
}

// ----------------------------------------------------------------- scan
// In-place inclusive scan of a[0..m) (int64), 4096 elements per workgroup.
__global__ __launch_bounds__(1024) void k_scan_local(int64_t* a, int64_t m, int64_t* bsum) {
  __shared__ int64_t s[1024];
  const int64_t base = int64_t(blockIdx.x) * 4096 + int64_t(threadIdx.x) * 4;
  int64_t v[4];
  int64_t run = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t idx = base + q;
    run += idx < m ? a[idx] : 0;
    v[q] = run;
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  const int64_t excl = threadIdx.x ? s[threadIdx.x - 1] : 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t idx = base + q;
    if (idx < m) a[idx] = v[q] + excl;
  }
  if (threadIdx.x == 1023 && bsum) bsum[blockIdx.x] = s[1023];
}

__global__ void k_scan_add(int64_t* a, int64_t m, const int64_t* bsum) {
  const int64_t idx = int64_t(blockIdx.x + 1) * 4096 + int64_t(threadIdx.x) * 4;  // blocks 1..
  const int64_t off = bsum[blockIdx.x];                                            // inclusive sum of blocks < this
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (idx + q < m) a[idx + q] += off;
}

}  // namespace

void scan_inclusive(int64_t* a, int64_t m, hipStream_t st) {
  if (m <= 0) return;
  const int64_t nb = (m + 4095) / 4096;
  DBuf<int64_t> bsum;
  bsum.alloc(nb);
  k_scan_local<<<int(nb), 1024, 0, st>>>(a, m, bsum);
  NS_LAUNCH_CHECK();
  if (nb > 1) {
    scan_inclusive(bsum.p, nb, st);
    k_scan_add<<<int(nb - 1), 1024, 0, st>>>(a, m, bsum);
    NS_LAUNCH_CHECK();
  }
}

namespace {

// ----------------------------------------------------------------- extraction

__global__ __launch_bounds__(256) void k_validate(int64_t n, int64_t nnz, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const int32_t* __restrict__ part, int* flags,
                                                  int* __restrict__ wg_minmax) {
  __shared__ int smax[4], smin[4];
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int pmax = INT32_MIN, pmin = INT32_MAX;
  if (i < n) {
    if (i == 0 && (ptr[0] != 0 || ptr[n] != nnz)) flags[F_STRUCT] = 1;
    const int64_t e0 = ptr[i], e1 = ptr[i + 1];
    if (e1 < e0 || e0 < 0 || e1 > nnz) {
      flags[F_STRUCT] = 1;
    } else {
      bool bad_idx = false, bad_val = false;
      for (int64_t e = e0; e < e1; e += 4) {  // four entries' loads in flight together (clamped positions)
        int32_t j[4];
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int64_t ek = e + k < e1 ? e + k : e;
          j[k] = col[ek];
          v[k] = val[ek];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          bad_idx |= j[k] < 0 || j[k] >= n;
          bad_val |= !(v[k] == v[k]) || v[k] - v[k] != 0.0;
        }
      }
      if (bad_idx) flags[F_STRUCT] = 1;
      if (bad_val) flags[F_NAN] = 1;
    }
    pmax = pmin = part[i];
  }
  // label range: wave-wide max / min, then the workgroup's, written per workgroup (k_minmax_final reduces)
  for (int o = 32; o > 0; o >>= 1) {
    pmax = max(pmax, __shfl_xor(pmax, o));
    pmin = min(pmin, __shfl_xor(pmin, o));
  }
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = pmax;
    smin[threadIdx.x >> 6] = pmin;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    wg_minmax[2 * blockIdx.x] = max(max(smax[0], smax[1]), max(smax[2], smax[3]));
    wg_minmax[2 * blockIdx.x + 1] = min(min(smin[0], smin[1]), min(smin[2], smin[3]));
  }
}

__global__ __launch_bounds__(1024) void k_minmax_final(int nwg, const int* __restrict__ wg_minmax,
                                                       int* __restrict__ minmax) {
  __shared__ int smax[1024], smin[1024];
  int pmax = INT32_MIN, pmin = INT32_MAX;
  for (int b = threadIdx.x; b < nwg; b += 1024) {
    pmax = max(pmax, wg_minmax[2 * b]);
    pmin = min(pmin, wg_minmax[2 * b + 1]);
  }
  smax[threadIdx.x] = pmax;
  smin[threadIdx.x] = pmin;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + o]);
      smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    minmax[0] = smax[0];
    minmax[1] = smin[0];
  }
}


// Every stored (i, j, v) must have its mirror (j, i, v).
__global__ void k_symcheck(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ val, int* flags) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
    const int32_t j = col[e];
    bool ok = false;
    for (int64_t f = ptr[j]; f < ptr[j + 1]; ++f)
      if (col[f] == i) {
        ok = val[f] == val[e];
        break;
      }
    if (!ok) flags[F_ASYM] = 1;
  }
}

// piece of node i: the q with node[q] <= i < node[q + 1]
__device__ __forceinline__ int piece_of(const int64_t* __restrict__ node, int P, int64_t i) {
  int lo = 0, hi = P - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (node[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Groups local to one piece (problem): its subdomains, then its level-2 blocks, then its junction set.
__global__ void k_group(int64_t n, const int32_t* __restrict__ part, int sub0, int nsub, int l20, int nl2,
                        int32_t* __restrict__ grp, int32_t* __restrict__ grp2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = part[i];
  grp[i] = p >= 0 ? p - sub0 : (p <= -2 ? nsub + (-2 - p - l20) : nsub + nl2);
  grp2[i] = p < 0 ? 1 : 0;
}

// Stable rank of each node inside its group: rank[i] = #{j < i : grp[j] == grp[i]}.
__global__ __launch_bounds__(1024) void k_chunk_hist(int64_t n, const int32_t* __restrict__ grp, int G,
                                                     int32_t* __restrict__ cnt) {
  extern __shared__ int hist[];
  for (int g = threadIdx.x; g < G; g += blockDim.x) hist[g] = 0;
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  if (i < n) atomicAdd(&hist[grp[i]], 1);
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += blockDim.x) cnt[int64_t(blockIdx.x) * G + g] = hist[g];
}

// Exclusive prefix over the chunks per group; the group's total goes to total[d] with d = the piece's
// destination of local group g (subdomains at d0 + g, level-2 blocks at d1 + g - nsub, the junction set at d2).
__global__ void k_chunk_offsets(int nchunk, int G, int32_t* __restrict__ cnt, int32_t* __restrict__ total, int nsub,
                                int nl2, int d0, int d1, int d2) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int run = 0;
  constexpr int B = 16;  // chunks per batch: their loads are issued together
  for (int c0 = 0; c0 < nchunk; c0 += B) {
    int v[B];
#pragma unroll
    for (int k = 0; k < B; ++k) v[k] = cnt[int64_t(min(c0 + k, nchunk - 1)) * G + g];  // clamped, in bounds
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (c0 + k < nchunk) {
        cnt[int64_t(c0 + k) * G + g] = run;
        run += v[k];
      }
  }
  const int d = g < nsub ? d0 + g : (g < nsub + nl2 ? d1 + g - nsub : d2);
  if (d >= 0) total[d] = run;
}

// interface index of every interface node: rank inside its piece + the piece's interface offset
__global__ void k_gidx_offset(int64_t n, const int32_t* __restrict__ part, const int64_t* __restrict__ node, int P,
                              const int64_t* __restrict__ goff, int32_t* __restrict__ gidx) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || part[i] >= 0) return;
  gidx[i] += int32_t(goff[piece_of(node, P, i)]);
}

__global__ __launch_bounds__(1024) void k_chunk_rank(int64_t n, const int32_t* __restrict__ grp, int G,
                                                     const int32_t* __restrict__ cnt, int32_t* __restrict__ rank) {
  __shared__ int sg[1024];
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  sg[threadIdx.x] = i < n ? grp[i] : -1;
  __syncthreads();
  if (i >= n) return;
  const int my = sg[threadIdx.x];
  int c = 0;
  for (int u = 0; u < int(threadIdx.x); ++u) c += sg[u] == my;
  rank[i] = cnt[int64_t(blockIdx.x) * G + my] + c;
}

struct NodeMaps {
  const int32_t* part;
  const int32_t* rank;   // rank inside (subdomain | level-2 block | junction set of the piece)
  const int32_t* gidx;   // interface index
  const int64_t* roff1;  // padded row offset of each subdomain block
  const int64_t* roff2;  // padded row offset of each level-2 block
  const int64_t* coff1;  // compact interior offset of each subdomain
  const int64_t* node;   // [P + 1] first node of each piece
  int P;
  const int64_t* roffJ;  // padded row offset of each piece's junction block
  const int* l2first;    // [P + 1] first level-2 block of each piece
};

__global__ void k_maps(int64_t n, NodeMaps m, int32_t* iperm, int32_t* icomp, int32_t* gperm, int32_t* l2src,
                       int32_t* jsrc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = m.part[i];
  const int r = m.rank[i];
  if (p >= 0) {
    const int64_t pos = m.roff1[p] + r;
    iperm[pos] = int32_t(i);
    icomp[pos] = int32_t(m.coff1[p] + r);
  } else {
    const int g = m.gidx[i];
    gperm[g] = int32_t(i);
    if (p <= -2)
      l2src[m.roff2[-2 - p] + r] = g;
    else
      jsrc[m.roffJ[piece_of(m.node, m.P, i)] + r] = g;
  }
}

// padded level-2 row -> first padded row of its piece's junction block (for the dense A_s^{-1} A_sJ)


struct Outs {
  int64_t *pIG, *pGI, *pGG, *psJ, *pJs;  // row pointers (counting pass: counts at [row+1])
  int32_t *cIG, *cGI, *cGG, *csJ, *cJs;
  double *vIG, *vGI, *vGG, *vsJ, *vJs;
  float *fIG, *fGI, *fGG, *fsJ, *fJs;
  double *L1, *L2, *LJ;
  const int *nt1, *nt2, *nbt1, *nbt2, *ntJ;
  const int64_t *foff1, *foff2, *foffJ;
  int *bw1, *bw2;  // counting pass: element half-bandwidth of every padded row's block row (row r: largest r - c)
};

// One thread per row.  FILL = false: count entries per CSR row and find the
// half-bandwidth of every diagonal block; FILL = true: write CSR entries and
// the lower triangles of the diagonal blocks (band tile storage).
template <bool FILL>
__global__ void k_extract(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                          const double* __restrict__ val, NodeMaps m, Outs o, int* flags) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int pi = m.part[i];
  const int ri = m.rank[i];
  int64_t nIG = 0, nGI = 0, nGG = 0, nsJ = 0, nJs = 0;
  int64_t rowIG = 0, rowG = 0, rowsJ = 0, rowJs = 0;
  int bw = 0;
  if (pi >= 0) {
    rowIG = m.roff1[pi] + ri;
  } else {
    rowG = m.gidx[i];
    if (pi <= -2) rowsJ = m.roff2[-2 - pi] + ri;
    if (pi == -1) rowJs = m.roffJ[piece_of(m.node, m.P, i)] + ri;
  }
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
    const int j = col[e];
    const int pj = m.part[j];
    const double v = val[e];
    const int rj = m.rank[j];
    if (pi >= 0) {
      if (pj >= 0) {
        if (pj != pi) {
          flags[F_DBBD1] = 1;
        } else if (!FILL) {
          bw = max(bw, ri - rj);
        } else if (ri >= rj) {
          o.L1[o.foff1[pi] + band_elem(o.nt1[pi], o.nbt1[pi], ri, rj)] = v;
        }
      } else {
        if (FILL) {
          const int64_t q = o.pIG[rowIG] + nIG;
          o.cIG[q] = m.gidx[j];
          o.vIG[q] = v;
          o.fIG[q] = float(v);
        }
        ++nIG;
      }
    } else {
      if (pj >= 0) {
        if (FILL) {
          const int64_t q = o.pGI[rowG] + nGI;
          o.cGI[q] = int32_t(m.roff1[pj] + rj);
          o.vGI[q] = v;
          o.fGI[q] = float(v);
        }
        ++nGI;
      } else {
        if (FILL) {
          const int64_t q = o.pGG[rowG] + nGG;
          o.cGG[q] = m.gidx[j];
          o.vGG[q] = v;
          o.fGG[q] = float(v);
        }
        ++nGG;
        if (pi <= -2) {
          if (pj <= -2) {
            if (pj != pi)
              flags[F_DBBD2] = 1;
            else if (!FILL)
              bw = max(bw, ri - rj);
            else if (ri >= rj)
              o.L2[o.foff2[-2 - pi] + band_elem(o.nt2[-2 - pi], o.nbt2[-2 - pi], ri, rj)] = v;
          } else {  // junction column
            if (FILL) {
              const int64_t q = o.psJ[rowsJ] + nsJ;
              o.csJ[q] = int32_t(m.roffJ[piece_of(m.node, m.P, j)] + rj);
              o.vsJ[q] = v;
              o.fsJ[q] = float(v);
            }
            ++nsJ;
          }
        } else {  // junction row
          if (pj <= -2) {
            if (FILL) {
              const int64_t q = o.pJs[rowJs] + nJs;
              o.cJs[q] = int32_t(m.roff2[-2 - pj] + rj);
              o.vJs[q] = v;
              o.fJs[q] = float(v);
            }
            ++nJs;
          } else if (FILL && ri >= rj) {
            const int q = piece_of(m.node, m.P, i);
            o.LJ[o.foffJ[q] + band_elem(o.ntJ[q], o.ntJ[q] - 1, ri, rj)] = v;
          }
        }
      }
    }
  }
  if (!FILL) {
    // per row (thousands of rows share a block: a per-block atomic maximum is a hot spot); k_block_max reduces
    if (pi >= 0) o.bw1[rowIG] = bw;
    if (pi <= -2) o.bw2[rowsJ] = bw;
    if (pi >= 0) {
      o.pIG[rowIG + 1] = nIG;
    } else {
      o.pGI[rowG + 1] = nGI;
      o.pGG[rowG + 1] = nGG;
      if (pi <= -2) o.psJ[rowsJ + 1] = nsJ;
      if (pi == -1) o.pJs[rowJs + 1] = nJs;
    }
  }
}

// Element half-bandwidth of every diagonal block of the two levels: the largest of its rows' values.
__global__ __launch_bounds__(256) void k_block_max(int nb1, const int64_t* __restrict__ roff1,
                                                   const int* __restrict__ rows1, const int* __restrict__ rbw1,
                                                   const int64_t* __restrict__ roff2, const int* __restrict__ rows2,
                                                   const int* __restrict__ rbw2, int* __restrict__ out) {
  __shared__ int red[256];
  const int b = blockIdx.x;
  const bool l1 = b < nb1;
  const int bb = l1 ? b : b - nb1;
  const int64_t r0 = l1 ? roff1[bb] : roff2[bb];
  const int cnt = l1 ? rows1[bb] : rows2[bb];
  const int* src = l1 ? rbw1 : rbw2;
  int m = 0;
  for (int r = threadIdx.x; r < cnt; r += 256) m = max(m, src[r0 + r]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

// Identity on the padded diagonal of every block.
__global__ void k_pad_identity(const int* __restrict__ nt_arr, const int* __restrict__ nbt_arr,
                               const int* __restrict__ nb_arr, const int64_t* __restrict__ foff,
                               double* __restrict__ L) {
  const int b = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int nt = nt_arr[b], nb = nb_arr[b];
  if (r < nb || r >= nt * TILE) return;
  L[foff[b] + band_elem(nt, nbt_arr[b], r, r)] = 1.0;
}

// Junction block q: S_J(ji, jj) -= sum_e A_Js(roffJ_q + ji, e) * E(col_e, jj) on the lower triangle,
// E(row, jj) = (A_s^{-1} A_sJ) with the junction column local to the piece of the level-2 row.
__global__ void k_junction_update(const int* __restrict__ nbJ, const int* __restrict__ ntJ,
                                  const int64_t* __restrict__ roffJ, const int64_t* __restrict__ foffJ,
                                  const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                  const double* __restrict__ val, const double* __restrict__ E, int64_t lde,
                                  double* __restrict__ LJ) {
  const int q = blockIdx.y;
  const int nJ = nbJ[q];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(nJ) * nJ) return;
  const int ji = int(idx / nJ), jj = int(idx % nJ);
  if (jj > ji) return;
  const int64_t row = roffJ[q] + ji;
  double acc = 0.0;
  for (int64_t e = ptr[row]; e < ptr[row + 1]; ++e) acc += val[e] * E[int64_t(col[e]) * lde + jj];
  LJ[foffJ[q] + band_elem(ntJ[q], ntJ[q] - 1, ji, jj)] -= acc;
}

// Row r of level-2 block b: E(roff2_b + r, c - roffJ_q) = A_sJ(roff2_b + r, c), q the problem of block b, and
// ft[b * nchunk + chunk of the column] = the smallest tile row of block b holding a nonzero of that chunk.
__global__ void k_sj_to_dense(int nl2, const int* __restrict__ nt2, const int64_t* __restrict__ roff2,
                              const int* __restrict__ l2first, int P, const int64_t* __restrict__ roffJ,
                              const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                              const double* __restrict__ val, double* __restrict__ E, int64_t lde, int nchunk,
                              int* __restrict__ ft) {
  const int b = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nt2[b] * TILE) return;
  int q = 0;
  while (q + 1 < P && l2first[q + 1] <= b) ++q;
  const int64_t row = roff2[b] + r, jb = roffJ[q];
  for (int64_t e = ptr[row]; e < ptr[row + 1]; ++e) {
    const int64_t c = col[e] - jb;
    E[row * lde + c] = val[e];
    atomicMin(&ft[int64_t(b) * nchunk + c / TILE], r / TILE);
  }
}

__global__ void k_fill_int(int64_t n, int v, int* __restrict__ a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

void pad_identity(TileLevel& lv, hipStream_t st) {
  if (lv.nblk == 0) return;
  dim3 g((lv.max_nt * TILE + 255) / 256, lv.nblk);
  k_pad_identity<<<g, 256, 0, st>>>(lv.nt, lv.nbt, lv.nb, lv.foff, lv.L64);
  NS_LAUNCH_CHECK();
}

void alloc_csr(Csr& A, int64_t nrows) {
  A.nrows = nrows;
  A.ptr.alloc(nrows + 1);
  NS_HIP(hipMemsetAsync(A.ptr.p, 0, (nrows + 1) * sizeof(int64_t), alloc_stream()));
}

// The level-2 rows with entries in A_sJ, block by block, and the padded row -> block map.  Kept only when every
// block has at most L2C_MAX such rows (box interfaces in two dimensions: the two ends of a separator segment);
// otherwise l2c_n stays 0 and the second level-2 solve runs in full.
constexpr int L2C_MAX = 16;
void build_l2_coupled_rows(Handle& h, const std::vector<int64_t>& ptr) {
  const TileLevel& lv = h.L2;
  h.l2c_n = 0;
  h.l2c_w = 0;
  if (lv.nblk == 0) return;
  std::vector<int32_t> rows, off(lv.nblk + 1, 0), blk(lv.nrows_pad, 0);
  for (int b = 0; b < lv.nblk; ++b) {
    const int64_t r0 = lv.h_roff[b], r1 = r0 + int64_t(lv.h_nt[b]) * TILE;
    for (int64_t r = r0; r < r1; ++r) {
      blk[r] = b;
      if (ptr[r + 1] > ptr[r]) rows.push_back(int32_t(r));
    }
    off[b + 1] = int32_t(rows.size());
    if (off[b + 1] - off[b] > L2C_MAX) return;
    h.l2c_w = std::max(h.l2c_w, off[b + 1] - off[b]);
  }
  if (rows.empty()) return;
  hipStream_t st = alloc_stream();
  h.l2c_rows.alloc(rows.size());
  h.l2c_off.alloc(off.size());
  h.l2c_blk.alloc(blk.size());
  upload(h.l2c_rows.p, rows.data(), rows.size() * sizeof(int32_t), st);
  upload(h.l2c_off.p, off.data(), off.size() * sizeof(int32_t), st);
  upload(h.l2c_blk.p, blk.data(), blk.size() * sizeof(int32_t), st);
  h.l2c_n = int64_t(rows.size());
}

}  // namespace

// The coefficients of the second level-2 solve (k_l2c_coef) from the explicit inverses of the level-2 blocks,
// FP64 and, when the FP32 inverses exist, FP32; without explicit inverses the path stays off.
void make_l2_coefs(Handle& h) {
  const TileLevel& lv = h.L2;
  if (!h.l2c_n || !lv.Ainv64.p) return;
  hipStream_t st = h.stream;
  const int64_t n2 = lv.nrows_pad;
  const unsigned grid = unsigned((n2 + 255) / 256);
  h.l2c_rinf.alloc(2 * n2);
  h.l2c_coef64.alloc(n2 * h.l2c_w);
  k_l2c_coef<double><<<grid, 256, 0, st>>>(n2, h.l2c_blk, lv.roff, lv.inv_off, lv.inv_lda, lv.Ainv64.p, h.l2c_off,
                                           h.l2c_rows, h.l2c_w, h.l2c_coef64.p,
                                           reinterpret_cast<int2*>(h.l2c_rinf.p));
  NS_LAUNCH_CHECK();
  if (lv.Ainv32.p) {
    h.l2c_coef32.alloc(n2 * h.l2c_w);
    k_l2c_coef<float><<<grid, 256, 0, st>>>(n2, h.l2c_blk, lv.roff, lv.inv_off, lv.inv_lda, lv.Ainv32.p, h.l2c_off,
                                            h.l2c_rows, h.l2c_w, h.l2c_coef32.p, nullptr);
    NS_LAUNCH_CHECK();
  }
}

namespace {

void finish_csr(Csr& A, hipStream_t st) {
  if (A.nrows == 0) return;
  scan_inclusive(A.ptr.p + 1, A.nrows, st);
  NS_HIP(hipMemcpyAsync(&A.nnz, A.ptr.p + A.nrows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  A.col.alloc(A.nnz > 0 ? A.nnz : 1);
  A.val64.alloc(A.nnz > 0 ? A.nnz : 1);
  A.val32.alloc(A.nnz > 0 ? A.nnz : 1);
}

}  // namespace

// ------------------------------------------------------------------------ API

void extract_dbbd(Handle& h, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const double* val,
                  const int32_t* part, const Pieces* pcs) {
  hipStream_t st = h.stream;
  h.n = n;
  h.nnz = nnz;
  int* flags = h.dflags.p;
  const int gn = int((n + 255) / 256);
  DBuf<int> minmax;
  minmax.alloc(2 + 2 * int64_t(gn));
  k_validate<<<gn, 256, 0, st>>>(n, nnz, row_ptr, col, val, part, flags, minmax.p + 2);
  NS_LAUNCH_CHECK();
  k_minmax_final<<<1, 1024, 0, st>>>(gn, minmax.p + 2, minmax.p);
  NS_LAUNCH_CHECK();
  int mm[2];
  NS_HIP(hipMemcpyAsync(mm, minmax.p, sizeof(mm), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(h.hflags, flags, 8 * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  if (h.hflags[F_STRUCT]) fail(INVALID_ARG, "CSR structure invalid (row_ptr/col_idx out of range)");
  if (h.hflags[F_NAN]) fail(INVALID_ARG, "matrix values contain NaN or Inf");
  k_symcheck<<<gn, 256, 0, st>>>(n, row_ptr, col, val, flags);
  NS_LAUNCH_CHECK();
  Pieces one;
  if (!pcs) {
    one.node = {0, n};
    one.sub = {0, mm[0] >= 0 ? mm[0] + 1 : 0};
    one.l2 = {0, mm[1] <= -2 ? -mm[1] - 1 : 0};
    pcs = &one;
  }
  const int P = int(pcs->node.size()) - 1;
  h.nsub = pcs->sub[P];
  h.nl2 = pcs->l2[P];
  if (mm[0] >= h.nsub || (mm[1] <= -2 && -mm[1] - 1 > h.nl2)) fail(INVALID_ARG, "part labels out of range");
  h.nprob = P;
  h.h_noff = pcs->node;
  h.h_sub = pcs->sub;

  // groups and stable ranks, piece by piece (groups never span two pieces)
  DBuf<int32_t> grp, grp2, rank, gidx, cnt, totall;
  grp.alloc(n);
  grp2.alloc(n);
  rank.alloc(n);
  gidx.alloc(n);
  const int ntot = h.nsub + h.nl2 + 2 * P;  // block sizes, junction counts, interface counts
  totall.alloc(ntot);
  NS_HIP(hipMemsetAsync(totall.p, 0, ntot * sizeof(int32_t), st));
  int64_t cmax = 2;
  for (int q = 0; q < P; ++q) {
    const int64_t nq = pcs->node[q + 1] - pcs->node[q];
    const int Gq = (pcs->sub[q + 1] - pcs->sub[q]) + (pcs->l2[q + 1] - pcs->l2[q]) + 1;
    if (Gq > 32768) fail(INVALID_ARG, "too many subdomains + interface blocks in one problem (limit 32767)");
    cmax = std::max(cmax, ((nq + 1023) / 1024) * std::max(Gq, 2));
  }
  cnt.alloc(cmax);
  for (int q = 0; q < P; ++q) {
    const int64_t a = pcs->node[q], nq = pcs->node[q + 1] - a;
    if (nq == 0) continue;
    const int nsq = pcs->sub[q + 1] - pcs->sub[q], nlq = pcs->l2[q + 1] - pcs->l2[q], Gq = nsq + nlq + 1;
    const int nch = int((nq + 1023) / 1024);
    k_group<<<unsigned((nq + 255) / 256), 256, 0, st>>>(nq, part + a, pcs->sub[q], nsq, pcs->l2[q], nlq, grp + a,
                                                        grp2 + a);
    NS_LAUNCH_CHECK();
    k_chunk_hist<<<nch, 1024, Gq * sizeof(int), st>>>(nq, grp + a, Gq, cnt);
    NS_LAUNCH_CHECK();
    k_chunk_offsets<<<(Gq + 255) / 256, 256, 0, st>>>(nch, Gq, cnt, totall, nsq, nlq, pcs->sub[q],
                                                       h.nsub + pcs->l2[q], h.nsub + h.nl2 + q);
    NS_LAUNCH_CHECK();
    k_chunk_rank<<<nch, 1024, 0, st>>>(nq, grp + a, Gq, cnt, rank + a);
    NS_LAUNCH_CHECK();
    k_chunk_hist<<<nch, 1024, 2 * sizeof(int), st>>>(nq, grp2 + a, 2, cnt);
    NS_LAUNCH_CHECK();
    k_chunk_offsets<<<1, 256, 0, st>>>(nch, 2, cnt, totall, 1, 0, -1, -1, h.nsub + h.nl2 + P + q);
    NS_LAUNCH_CHECK();
    k_chunk_rank<<<nch, 1024, 0, st>>>(nq, grp2 + a, 2, cnt, gidx + a);
    NS_LAUNCH_CHECK();
  }
  std::vector<int> tot(ntot);
  NS_HIP(hipMemcpyAsync(tot.data(), totall.p, ntot * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(h.hflags, flags, 8 * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  if (h.hflags[F_ASYM]) fail(INVALID_ARG, "A is not symmetric (pattern or values)");

  std::vector<int> nb1(tot.begin(), tot.begin() + h.nsub), nb2(tot.begin() + h.nsub, tot.begin() + h.nsub + h.nl2);
  std::vector<int> nJq(tot.begin() + h.nsub + h.nl2, tot.begin() + h.nsub + h.nl2 + P);
  h.h_goff.assign(P + 1, 0);
  for (int q = 0; q < P; ++q) h.h_goff[q + 1] = h.h_goff[q] + tot[h.nsub + h.nl2 + P + q];
  h.nJ = 0;
  for (int q = 0; q < P; ++q) h.nJ += nJq[q];
  std::vector<int64_t> coff(h.nsub + 1, 0);
  for (int b = 0; b < h.nsub; ++b) coff[b + 1] = coff[b] + nb1[b];
  h.nI = coff[h.nsub];
  h.nG = n - h.nI;
  if (h.nG != h.h_goff[P]) fail(INVALID_ARG, "interface count mismatch");
  for (int q = 0; q < P; ++q) {
    if (h.h_goff[q + 1] == h.h_goff[q]) fail(INVALID_ARG, "partition has no interface nodes");
    if (pcs->sub[q + 1] == pcs->sub[q]) fail(INVALID_ARG, "partition has no interior nodes");
  }
  if (h.nI <= 0) fail(INVALID_ARG, "partition has no interior nodes");
  h.pnode.alloc(P + 1);
  upload(h.pnode.p, pcs->node.data(), (P + 1) * sizeof(int64_t), st);
  h.l2first.alloc(P + 1);
  upload(h.l2first.p, pcs->l2.data(), (P + 1) * sizeof(int), st);
  if (P > 1) {
    DBuf<int64_t> goff;
    goff.alloc(P + 1);
    upload(goff.p, h.h_goff.data(), (P + 1) * sizeof(int64_t), st);
    k_gidx_offset<<<gn, 256, 0, st>>>(n, part, h.pnode, P, goff, gidx);
    NS_LAUNCH_CHECK();
    NS_HIP(hipStreamSynchronize(st));
  }
  h.L1.layout(nb1);
  h.L2.layout(nb2);
  h.L2.role = 1;
  h.LJ.role = 1;
  h.LJ.layout(h.nJ > 0 ? nJq : std::vector<int>{});
  DBuf<int64_t> coff1;
  coff1.alloc(h.nsub > 0 ? h.nsub : 1);
  if (h.nsub) upload(coff1.p, coff.data(), h.nsub * sizeof(int64_t), st);

  // maps
  const int64_t nIpad = h.L1.nrows_pad, n2pad = h.L2.nrows_pad, nJpad = h.LJ.nrows_pad;
  h.iperm.alloc(nIpad > 0 ? nIpad : 1);
  h.icomp.alloc(nIpad > 0 ? nIpad : 1);
  h.gperm.alloc(h.nG);
  h.l2src.alloc(n2pad > 0 ? n2pad : 1);
  h.jsrc.alloc(nJpad > 0 ? nJpad : 1);
  NS_HIP(hipMemsetAsync(h.iperm.p, 0xFF, h.iperm.n * sizeof(int32_t), st));
  NS_HIP(hipMemsetAsync(h.icomp.p, 0xFF, h.icomp.n * sizeof(int32_t), st));
  NS_HIP(hipMemsetAsync(h.l2src.p, 0xFF, h.l2src.n * sizeof(int32_t), st));
  NS_HIP(hipMemsetAsync(h.jsrc.p, 0xFF, h.jsrc.n * sizeof(int32_t), st));
  NodeMaps m{part, rank, gidx, h.L1.roff.p, h.L2.roff.p, coff1.p, h.pnode.p, P, h.LJ.roff.p, h.l2first.p};
  k_maps<<<gn, 256, 0, st>>>(n, m, h.iperm, h.icomp, h.gperm, h.l2src, h.jsrc);
  NS_LAUNCH_CHECK();

  // counting pass
  alloc_csr(h.AIG, nIpad);
  alloc_csr(h.AGI, h.nG);
  alloc_csr(h.AGG, h.nG);
  alloc_csr(h.AsJ, n2pad);
  alloc_csr(h.AJs, nJpad);
  Outs o{};
  o.pIG = h.AIG.ptr;
  o.pGI = h.AGI.ptr;
  o.pGG = h.AGG.ptr;
  o.psJ = h.AsJ.ptr;
  o.pJs = h.AJs.ptr;
  DBuf<int> bwd, rbw;
  bwd.alloc(h.nsub + h.nl2 + 1);
  rbw.alloc(nIpad + n2pad + 1);
  NS_HIP(hipMemsetAsync(bwd.p, 0, bwd.n * sizeof(int), st));
  NS_HIP(hipMemsetAsync(rbw.p, 0, rbw.n * sizeof(int), st));
  o.bw1 = rbw.p;
  o.bw2 = rbw.p + nIpad;
  k_extract<false><<<gn, 256, 0, st>>>(n, row_ptr, col, val, m, o, flags);
  NS_LAUNCH_CHECK();
  if (h.nsub + h.nl2 > 0) {
    k_block_max<<<h.nsub + h.nl2, 256, 0, st>>>(h.nsub, h.L1.roff, h.L1.nb, o.bw1, h.L2.roff, h.L2.nb, o.bw2, bwd);
    NS_LAUNCH_CHECK();
  }
  std::vector<int> bwh(bwd.n);
  NS_HIP(hipMemcpyAsync(bwh.data(), bwd.p, bwd.n * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipMemcpyAsync(h.hflags, flags, 8 * sizeof(int), hipMemcpyDeviceToHost, st));
  NS_HIP(hipStreamSynchronize(st));
  if (h.hflags[F_DBBD1]) fail(INVALID_ARG, "partition is not DBBD: interior nodes of different subdomains are coupled");
  if (h.hflags[F_DBBD2]) fail(INVALID_ARG, "interface split invalid: nodes of different interface blocks are coupled");
  // band storage of the diagonal blocks (the junction block is dense)
  h.L1.layout_band(std::vector<int>(bwh.begin(), bwh.begin() + h.nsub));
  h.L2.layout_band(std::vector<int>(bwh.begin() + h.nsub, bwh.begin() + h.nsub + h.nl2));
  {
    std::vector<int> bwJ;
    if (h.nJ > 0)
      for (int q = 0; q < P; ++q) bwJ.push_back(std::max(nJq[q] - 1, 0));
    h.LJ.layout_band(bwJ);  // dense junction blocks
  }
  o.nt1 = h.L1.nt;
  o.nt2 = h.L2.nt;
  o.nbt1 = h.L1.nbt;
  o.nbt2 = h.L2.nbt;
  o.foff1 = h.L1.foff;
  o.foff2 = h.L2.foff;
  o.ntJ = h.LJ.nt;
  o.foffJ = h.LJ.foff;
  finish_csr(h.AIG, st);
  finish_csr(h.AGI, st);
  finish_csr(h.AGG, st);
  finish_csr(h.AsJ, st);
  std::vector<int64_t> sjp;
  if (n2pad > 0 && nJpad > 0) {  // read once the junction coupling of finish_csr(AJs) has synchronised
    sjp.resize(n2pad + 1);
    NS_HIP(hipMemcpyAsync(sjp.data(), h.AsJ.ptr.p, (n2pad + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  }
  finish_csr(h.AJs, st);
  if (!sjp.empty()) {
    NS_HIP(hipStreamSynchronize(st));
    build_l2_coupled_rows(h, sjp);
  }
  // fill pass
  if (h.L1.f_elems) NS_HIP(hipMemsetAsync(h.L1.L64.p, 0, h.L1.f_elems * sizeof(double), st));
  if (h.L2.f_elems) NS_HIP(hipMemsetAsync(h.L2.L64.p, 0, h.L2.f_elems * sizeof(double), st));
  if (h.LJ.f_elems) NS_HIP(hipMemsetAsync(h.LJ.L64.p, 0, h.LJ.f_elems * sizeof(double), st));
  o.cIG = h.AIG.col;
  o.vIG = h.AIG.val64;
  o.fIG = h.AIG.val32;
  o.cGI = h.AGI.col;
  o.vGI = h.AGI.val64;
  o.fGI = h.AGI.val32;
  o.cGG = h.AGG.col;
  o.vGG = h.AGG.val64;
  o.fGG = h.AGG.val32;
  o.csJ = h.AsJ.col;
  o.vsJ = h.AsJ.val64;
  o.fsJ = h.AsJ.val32;
  o.cJs = h.AJs.col;
  o.vJs = h.AJs.val64;
  o.fJs = h.AJs.val32;
  o.L1 = h.L1.L64;
  o.L2 = h.L2.L64;
  o.LJ = h.LJ.L64;
  k_extract<true><<<gn, 256, 0, st>>>(n, row_ptr, col, val, m, o, flags);
  NS_LAUNCH_CHECK();
  pad_identity(h.L1, st);
  pad_identity(h.L2, st);
  pad_identity(h.LJ, st);
  // keep the original matrix for the true residual
  h.Aorig.nrows = n;
  h.Aorig.nnz = nnz;
  h.Aorig.ptr.alloc(n + 1);
  h.Aorig.col.alloc(nnz > 0 ? nnz : 1);
  h.Aorig.val64.alloc(nnz > 0 ? nnz : 1);
  NS_HIP(hipMemcpyAsync(h.Aorig.ptr.p, row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  if (nnz) {
    NS_HIP(hipMemcpyAsync(h.Aorig.col.p, col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    NS_HIP(hipMemcpyAsync(h.Aorig.val64.p, val, nnz * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
}

void assemble_junction(Handle& h) {
  hipStream_t st = h.stream;
  if (h.nJ == 0 || h.L2.nblk == 0) return;
  const int64_t n2pad = h.L2.nrows_pad;
  const int ldE = h.LJ.max_nt * TILE;  // junction columns of the level-2 rows' own piece
  int maxJ = 0;
  for (int q = 0; q < h.LJ.nblk; ++q) maxJ = std::max(maxJ, h.LJ.h_nb[q]);
  DBuf<double> E;
  DBuf<int> ft;
  E.alloc(n2pad * ldE);
  const int nchunk = ldE / TILE;
  const int64_t nft = int64_t(h.L2.nblk) * nchunk;
  ft.alloc(nft);
  NS_HIP(hipMemsetAsync(E.p, 0, n2pad * ldE * sizeof(double), st));
  k_fill_int<<<unsigned((nft + 255) / 256), 256, 0, st>>>(nft, INT32_MAX, ft);  // no nonzero yet
  NS_LAUNCH_CHECK();
  k_sj_to_dense<<<dim3((h.L2.max_nt * TILE + 255) / 256, h.L2.nblk), 256, 0, st>>>(
      h.nl2, h.L2.nt, h.L2.roff, h.l2first, h.nprob, h.LJ.roff, h.AsJ.ptr, h.AsJ.col, h.AsJ.val64, E, ldE, nchunk, ft);
  NS_LAUNCH_CHECK();
  // E = A_s^{-1} A_sJ: a patch touches few junction nodes, so most column chunks of a block are zero and
  // both sweeps skip them (the forward one also starts each chunk at its first nonzero tile row)
  tile_solve_chunks(h.L2, E.p, ldE, maxJ, ft, st);
  k_junction_update<<<dim3(unsigned((int64_t(maxJ) * maxJ + 255) / 256), h.LJ.nblk), 256, 0, st>>>(
      h.LJ.nb, h.LJ.nt, h.LJ.roff, h.LJ.foff, h.AJs.ptr, h.AJs.col, h.AJs.val64, E, ldE, h.LJ.L64);
  NS_LAUNCH_CHECK();
}

template <class T>
static T* ws_ptr(DBuf<double>& a, DBuf<float>& b) {
  if constexpr (sizeof(T) == 8)
    return a.p;
  else
    return b.p;
}

void ensure_workspace(Handle& h, int64_t ncols) {
  if (ncols <= h.ws_cols) return;
  const int64_t c = ncols;
  auto grow = [&](auto& buf, int64_t rows) { buf.alloc(rows > 0 ? rows * c : 1); };
  grow(h.wsB64, h.L2.nrows_pad);
  grow(h.wsJ64, h.LJ.nrows_pad);
  grow(h.wsC64, h.l2c_n);
  grow(h.wsB64b, h.L2.nrows_pad);
  grow(h.wsJ64b, h.LJ.nrows_pad);
  if (h.prec_inner) {
    grow(h.wsB32, h.L2.nrows_pad);
    grow(h.wsJ32, h.LJ.nrows_pad);
    grow(h.wsC32, h.l2c_n);
    grow(h.wsB32b, h.L2.nrows_pad);
    grow(h.wsJ32b, h.LJ.nrows_pad);
  }
  h.ws_cols = c;
}

// Padded interior right-hand side (rows L1.nrows_pad, ncols columns), made on first use: the local
// Schur blocks leave it unused in the inner solve.
template <class T>
static T* interior_ws(Handle& h, int64_t ncols) {
  if constexpr (sizeof(T) == 8) {
    if (ncols > h.wsT64_cols) {
      h.wsT64.alloc(std::max<int64_t>(h.L1.nrows_pad * ncols, 1));
      h.wsT64_cols = ncols;
    }
    return h.wsT64.p;
  } else {
    if (ncols > h.wsT32_cols) {
      h.wsT32.alloc(std::max<int64_t>(h.L1.nrows_pad * ncols, 1));
      h.wsT32_cols = ncols;
    }
    return h.wsT32.p;
  }
}

template <class T>
void op_schur(Handle& h, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, bool w_only) {
  if (h.LS.built)
    op_schur_local<T>(h, X, ldx, Y, ldy, ncols, w_only);
  else
    op_schur_tri<T>(h, X, ldx, Y, ldy, ncols, w_only);
}

// FP32 interior factors are made on first use when the local Schur blocks
// replaced them inside the inner solve.
template <class T>
static void need_l1(Handle& h) {
  if constexpr (sizeof(T) == 4)
    if (!h.L1.L32.p) tile_make_fp32(h.L1, h.stream);
}

template <class T>
void op_schur_tri(Handle& h, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, bool w_only) {
  hipStream_t st = h.stream;
  need_l1<T>(h);
  ensure_workspace(h, ncols);
  T* Tb = interior_ws<T>(h, ncols);
  spmm<T>(h.AIG, X, ldx, Tb, ncols, ncols, st);
  tile_solve<T>(h.L1, Tb, ncols, ncols, h.trsm_cols, st);
  if (h.nG == 0) return;
  KScope ks(KF_SCHUR_EPI, st);
  NS_TPR_DISPATCH(ncols, (k_schur_epi<T, TPR><<<grid_rows<TPR>(h.nG), 256, 0, st>>>(
                              h.nG, h.AGG.ptr, h.AGG.col, csr_vals<T>(h.AGG), X, ldx, h.AGI.ptr, h.AGI.col,
                              csr_vals<T>(h.AGI), Tb, ncols, Y, ldy, ncols, w_only ? 1 : 0)));
  NS_LAUNCH_CHECK();
}

// Approximate A_Gamma^{-1} R of the recursive construction: the block LDL^T solve of A_Gamma split by the
// level-2 labels (its interior s = the interface blocks, its interface J = the junction nodes), handled by the
// level-below handle g whose "original" rows are this handle's interface rows, with M_J = g's preconditioner
// in place of S_J^{-1}:
//   u_s = A_s^{-1} r_s,  y_J = M_J (r_J - A_Js u_s),  z_s = A_s^{-1} (r_s - A_sJ y_J),  z_J = y_J.
void gamma_solve_recursive(Handle& h, const double* R, int64_t ldr, double* Out, int64_t ldo, int ncols) {
  hipStream_t st = h.stream;
  Handle& g = *h.sub;
  g.stream = st;  // the level below follows this handle's stream (which a graph capture swaps)
  const int64_t nIp = g.L1.nrows_pad, nJ = g.nG;
  if (ncols > h.rec_cols) {
    h.recU.alloc(size_t(std::max<int64_t>(nIp, 1)) * ncols);
    h.recT.alloc(size_t(std::max<int64_t>(nJ, 1)) * ncols);
    h.recY.alloc(size_t(std::max<int64_t>(nJ, 1)) * ncols);
    h.rec_cols = ncols;
  }
  double* u = h.recU.p;
  double* t = h.recT.p;
  double* y = h.recY.p;
  gather_sub<double>(nIp, g.iperm, R, ldr, nullptr, static_cast<const double*>(nullptr), 0, u, ncols, ncols, st);
  tile_solve<double>(g.L1, u, ncols, ncols, h.trsm_cols, st);                   // u_s = A_s^{-1} r_s
  gather_sub<double>(nJ, g.gperm, R, ldr, &g.AGI, u, ncols, t, ncols, ncols, st);  // r_J - A_Js u_s
  sub_apply(g, t, ncols, y, ncols, ncols);                                        // y_J = M_J (...)
  gather_sub<double>(nIp, g.iperm, R, ldr, &g.AIG, y, ncols, u, ncols, ncols, st);  // r_s - A_sJ y_J
  tile_solve<double>(g.L1, u, ncols, ncols, h.trsm_cols, st);                   // z_s
  NS_TPR_DISPATCH(ncols, (k_scatter2<double, TPR><<<grid_rows<TPR>(nJ + nIp), 256, 0, st>>>(
                             nJ, g.gperm, y, nIp, g.iperm, u, ncols, Out, ldo, ncols)));
  NS_LAUNCH_CHECK();
}

template <class T>
void op_gamma_solve(Handle& h, const T* R, int64_t ldr, T* Out, int64_t ldo, int ncols) {
  hipStream_t st = h.stream;
  if (h.sub) {
    if constexpr (sizeof(T) == 8) {
      gamma_solve_recursive(h, R, ldr, Out, ldo, ncols);
      return;
    } else {
      fail(INVALID_ARG, "the recursive A_Gamma solve runs in FP64 only");
    }
  }
  ensure_workspace(h, ncols);
  T* Bp = ws_ptr<T>(h.wsB64, h.wsB32);
  T* Bq = ws_ptr<T>(h.wsB64b, h.wsB32b);
  T* Gj = ws_ptr<T>(h.wsJ64, h.wsJ32);
  T* Gk = ws_ptr<T>(h.wsJ64b, h.wsJ32b);
  const int64_t n2pad = h.L2.nrows_pad, nJpad = h.LJ.nrows_pad;
  // interface blocks: explicit inverses when built, else the two triangular sweeps (in place)
  auto solve = [&](const TileLevel& lv, T* in, T* out) -> T* {
    if (lv.Ainv64.p && (sizeof(T) == 8 || lv.Ainv32.p)) {
      tile_apply_inverse<T>(lv, in, out, ncols, st, nullptr, h.op_bf16 != 0);
      return out;
    }
    tile_solve<T>(lv, in, ncols, ncols, h.trsm_cols, st);
    return in;
  };
  T* xs = nullptr;
  if (n2pad) {
    if (sizeof(T) == 8 && ncols == 1 && ldr == 1 && h.L2.Ainv64.p && h.L2.inv_sym.built()) {
      // one column: the packed product reads its input through l2src (no separate gather)
      tile_apply_inverse<T>(h.L2, R, Bq, 1, st, h.l2src);
      xs = Bq;
    } else {
      gather_sub<T>(n2pad, h.l2src, R, ldr, nullptr, static_cast<const T*>(nullptr), 0, Bp, ncols, ncols, st);
      xs = solve(h.L2, Bp, Bq);
    }
  }
  if (nJpad) {
    gather_sub<T>(nJpad, h.jsrc, R, ldr, n2pad ? &h.AJs : nullptr, xs, ncols, Gj, ncols, ncols, st);
    T* xj = solve(h.LJ, Gj, Gk);
    // the second level-2 solve through the few columns of the explicit inverses that A_sJ reaches
    const T* coef = ws_ptr<T>(h.l2c_coef64, h.l2c_coef32);
    if (n2pad && h.l2c_n && coef && !h.op_bf16 && ncols <= 256) {
      T* C = ws_ptr<T>(h.wsC64, h.wsC32);
      const T* vsJ = ws_ptr<T>(h.AsJ.val64, h.AsJ.val32);
      auto run = [&](auto tpr, auto cpl) {
        constexpr int TPR = decltype(tpr)::value, CPL = decltype(cpl)::value;
        k_l2c_rows<T, TPR, CPL><<<grid_rows<TPR>(h.l2c_n), 256, 0, st>>>(h.l2c_n, h.l2c_rows, h.AsJ.ptr, h.AsJ.col,
                                                                         vsJ, xj, ncols, C, ncols);
        NS_LAUNCH_CHECK();
        k_scatter_l2c<T, TPR, CPL><<<grid_rows<TPR>(nJpad + n2pad), 256, 0, st>>>(
            nJpad, h.jsrc, xj, n2pad, h.l2src, xs, reinterpret_cast<const int2*>(h.l2c_rinf.p), coef, h.l2c_w, C,
            Out, ldo, ncols);
        NS_LAUNCH_CHECK();
      };
      using I = std::integral_constant<int, 1>;
      if (ncols == 1)
        run(I(), I());
      else if (ncols <= 16)
        run(std::integral_constant<int, 16>(), I());
      else if (ncols <= 64)
        run(std::integral_constant<int, 64>(), I());
      else if (ncols <= 80)  // four rows per wave: their dependent loads overlap
        run(std::integral_constant<int, 16>(), std::integral_constant<int, 5>());
      else if (ncols <= 128)
        run(std::integral_constant<int, 64>(), std::integral_constant<int, 2>());
      else if (ncols <= 160)
        run(std::integral_constant<int, 16>(), std::integral_constant<int, 10>());
      else if (ncols <= 192)
        run(std::integral_constant<int, 64>(), std::integral_constant<int, 3>());
      else
        run(std::integral_constant<int, 64>(), std::integral_constant<int, 4>());
      return;
    }
    if (n2pad) {
      gather_sub<T>(n2pad, h.l2src, R, ldr, &h.AsJ, xj, ncols, Bp, ncols, ncols, st);
      xs = solve(h.L2, Bp, Bq);
    }
    // both levels' results back into the interface rows in one launch
    const int64_t n2 = n2pad ? n2pad : 0;
    NS_TPR_DISPATCH(ncols, (k_scatter2<T, TPR><<<grid_rows<TPR>(nJpad + n2), 256, 0, st>>>(
                               nJpad, h.jsrc, xj, n2, h.l2src, xs, ncols, Out, ldo, ncols)));
    NS_LAUNCH_CHECK();
    return;
  }
  if (n2pad) scatter<T, T>(n2pad, h.l2src, xs, ncols, Out, ldo, ncols, st);
}

template <class T>
void op_interior_solve(Handle& h, const T* X, T* Y, int ncols) {
  hipStream_t st = h.stream;
  need_l1<T>(h);
  T* Tb = interior_ws<T>(h, ncols);
  gather_sub<T>(h.L1.nrows_pad, h.icomp, X, ncols, nullptr, static_cast<const T*>(nullptr), 0, Tb, ncols, ncols, st);
  tile_solve<T>(h.L1, Tb, ncols, ncols, h.trsm_cols, st);
  scatter<T, T>(h.L1.nrows_pad, h.icomp, Tb, ncols, Y, ncols, ncols, st);
}

// explicit instantiations
template void op_schur<double>(Handle&, const double*, int64_t, double*, int64_t, int, bool);
template void op_schur<float>(Handle&, const float*, int64_t, float*, int64_t, int, bool);
template void op_schur_tri<double>(Handle&, const double*, int64_t, double*, int64_t, int, bool);
template void op_schur_tri<float>(Handle&, const float*, int64_t, float*, int64_t, int, bool);
template void op_gamma_solve<double>(Handle&, const double*, int64_t, double*, int64_t, int);
template void op_gamma_solve<float>(Handle&, const float*, int64_t, float*, int64_t, int);
template void op_interior_solve<double>(Handle&, const double*, double*, int);
template void op_interior_solve<float>(Handle&, const float*, float*, int);

// generic helpers used by the solver
template <class T>
void gather_rows(int64_t nrows, const int32_t* src, const T* R, int64_t ldr, T* Out, int64_t ldo, int ncols,
                 hipStream_t st) {
  gather_sub<T>(nrows, src, R, ldr, nullptr, static_cast<const T*>(nullptr), 0, Out, ldo, ncols, st);
}
template <class T, class U>
void scatter_rows(int64_t nrows, const int32_t* dst, const T* B, int64_t ldb, U* Out, int64_t ldo, int ncols,
                  hipStream_t st) {
  scatter<T, U>(nrows, dst, B, ldb, Out, ldo, ncols, st);
}
template <class T>
void csr_mult(const Csr& A, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, hipStream_t st) {
  spmm<T>(A, X, ldx, Y, ldy, ncols, st);
}
template void gather_rows<double>(int64_t, const int32_t*, const double*, int64_t, double*, int64_t, int, hipStream_t);
template void gather_rows<float>(int64_t, const int32_t*, const float*, int64_t, float*, int64_t, int, hipStream_t);
template void scatter_rows<double, double>(int64_t, const int32_t*, const double*, int64_t, double*, int64_t, int,
                                           hipStream_t);
template void csr_mult<double>(const Csr&, const double*, int64_t, double*, int64_t, int, hipStream_t);
template void csr_mult<float>(const Csr&, const float*, int64_t, float*, int64_t, int, hipStream_t);

}  // namespace ns
