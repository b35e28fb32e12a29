// Tall-skinny block-vector kernels: Gram products X^T Y with a deterministic
// two-stage reduction, block updates Out = beta Out + X M (+ X2 M2), column
// norms, dot products and the fused vector updates of PCG.
#include "ns_vec.h"

namespace ns {
namespace {

constexpr int GRAM_CHUNKS = 240;  // fixed partial count: bitwise-reproducible reductions
constexpr int GRAM_RB = 16;       // rows staged per LDS batch
constexpr int GRAM_MAXQ = 32;     // outputs per thread (1024 threads): up to 32768 entries

template <class TA, class TB>
__global__ __launch_bounds__(1024) void k_gram_partial(int64_t n, const TA* __restrict__ A, int64_t lda, int ra,
                                                       const TB* __restrict__ B, int64_t ldb, int rb,
                                                       double* __restrict__ part) {
  extern __shared__ double sm[];
  double* sA = sm;                    // GRAM_RB x ra
  double* sB = sm + GRAM_RB * ra;     // GRAM_RB x rb
  const int nout = ra * rb;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = int64_t(blockIdx.x) * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  double acc[GRAM_MAXQ];
#pragma unroll
  for (int q = 0; q < GRAM_MAXQ; ++q) acc[q] = 0.0;
  for (int64_t rs = r0; rs < r1; rs += GRAM_RB) {
    const int nr = int(r1 - rs < GRAM_RB ? r1 - rs : GRAM_RB);
    __syncthreads();
    for (int e = threadIdx.x; e < GRAM_RB * ra; e += blockDim.x) {
      const int rr = e / ra, c = e % ra;
      sA[e] = rr < nr ? double(A[(rs + rr) * lda + c]) : 0.0;
    }
    for (int e = threadIdx.x; e < GRAM_RB * rb; e += blockDim.x) {
      const int rr = e / rb, c = e % rb;
      sB[e] = rr < nr ? double(B[(rs + rr) * ldb + c]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GRAM_MAXQ; ++q) {
      const int o = threadIdx.x + q * 1024;
      if (o < nout) {
        const int a = o / rb, b = o % rb;
        double s = acc[q];
        for (int rr = 0; rr < GRAM_RB; ++rr) s += sA[rr * ra + a] * sB[rr * rb + b];
        acc[q] = s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < GRAM_MAXQ; ++q) {
    const int o = threadIdx.x + q * 1024;
    if (o < nout) part[int64_t(blockIdx.x) * nout + o] = acc[q];
  }
}

__global__ void k_gram_final(int nchunk, int nout, const double* __restrict__ part, double* __restrict__ G,
                             double alpha, double beta) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int c = 0;
  for (; c + 8 <= nchunk; c += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += part[int64_t(c + u) * nout + o];
  for (; c < nchunk; ++c) s[0] += part[int64_t(c) * nout + o];
  const double t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  G[o] = alpha * t + (beta != 0.0 ? beta * G[o] : 0.0);
}

// Out[r, c] = beta * Out[r, c] + sum_m X[r, m] M[m, c] + sum_m X2[r, m] M2[m, c]
template <class T>
__global__ __launch_bounds__(256) void k_ts_update(int64_t n, int ncols, T* __restrict__ Out, int64_t ldo,
                                                   double beta, double gamma, const T* __restrict__ X,
                                                   int64_t ldx, int rm,
                                                   const double* __restrict__ M, int64_t ldm,
                                                   const T* __restrict__ X2, int64_t ldx2, int rm2,
                                                   const double* __restrict__ M2, int64_t ldm2) {
  extern __shared__ double sm[];
  double* sM = sm;             // rm x 32
  double* sM2 = sm + rm * 32;  // rm2 x 32
  const int c0 = blockIdx.y * 32;
  for (int e = threadIdx.x; e < rm * 32; e += blockDim.x) {
    const int m = e / 32, c = e % 32;
    sM[e] = (c0 + c < ncols) ? M[int64_t(m) * ldm + c0 + c] : 0.0;
  }
  for (int e = threadIdx.x; e < rm2 * 32; e += blockDim.x) {
    const int m = e / 32, c = e % 32;
    sM2[e] = (c0 + c < ncols) ? M2[int64_t(m) * ldm2 + c0 + c] : 0.0;
  }
  __syncthreads();
  const int c = threadIdx.x & 31;
  if (c0 + c >= ncols) return;
  const int64_t rbase = int64_t(blockIdx.x) * 64;
  for (int rr = threadIdx.x >> 5; rr < 64; rr += 8) {
    const int64_t r = rbase + rr;
    if (r >= n) break;
    double acc = 0.0;
    const T* xr = X + r * ldx;
    for (int m = 0; m < rm; ++m) acc += double(xr[m]) * sM[m * 32 + c];
    if (rm2) {
      const T* x2 = X2 + r * ldx2;
      for (int m = 0; m < rm2; ++m) acc += double(x2[m]) * sM2[m * 32 + c];
    }
    acc *= gamma;
    if (beta != 0.0) acc += beta * double(Out[r * ldo + c0 + c]);
    Out[r * ldo + c0 + c] = T(acc);
  }
}

template <class T, class U>
__global__ void k_convert(int64_t n, int ncols, const T* __restrict__ X, int64_t ldx, U* __restrict__ Y, int64_t ldy) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t r = idx / ncols;
  const int c = int(idx % ncols);
  Y[r * ldy + c] = U(X[r * ldx + c]);
}

// PCG vector updates; scalars live in device memory: sc[4 it + 0] = rho_it,
// sc[4 it + 1] = p^T q, sc[4 it + 2] = ||r||^2 after the update.
__global__ __launch_bounds__(256) void k_pcg_wr(int64_t n, const double* __restrict__ sc, int it,
                                                double* __restrict__ w, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                double* __restrict__ part) {
  __shared__ double red[256];
  const double alpha = sc[4 * it] / sc[4 * it + 1];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    w[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    s += x[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_final(int np, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// p = z + (rho_{it+1} / rho_it) p
__global__ void k_pcg_p(int64_t n, const double* __restrict__ sc, int it, const double* __restrict__ z,
                        double* __restrict__ p) {
  const double beta = sc[4 * (it + 1)] / sc[4 * it];
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = a * x[i] + (b != 0.0 ? b * y[i] : 0.0);
}

// Column sums of squares of a row-major block, in two deterministic stages.
template <class T>
__global__ __launch_bounds__(256) void k_colsq_partial(int64_t n, int ncols, const T* __restrict__ X, int64_t ldx,
                                                       double* __restrict__ part) {
  // thread t: column t % 64 chunk..., rows strided over the grid
  __shared__ double red[256];
  for (int c0 = 0; c0 < ncols; c0 += 64) {
    const int c = c0 + (threadIdx.x & 63);
    double s = 0.0;
    if (c < ncols)
      for (int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); r < n; r += int64_t(gridDim.x) * 4) {
        const double v = double(X[r * ldx + c]);
        s += v * v;
      }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < 64 && c < ncols)
      part[int64_t(blockIdx.x) * ncols + c] =
          red[threadIdx.x] + red[threadIdx.x + 64] + red[threadIdx.x + 128] + red[threadIdx.x + 192];
    __syncthreads();
  }
}

}  // namespace

template <class TA, class TB>
void gram(int64_t n, const TA* A, int64_t lda, int ra, const TB* B, int64_t ldb, int rb, double* G, double alpha,
          double beta, double* work, hipStream_t st) {
  const int nout = ra * rb;
  if (nout == 0) return;
  if (nout > 1024 * GRAM_MAXQ) fail(INVALID_ARG, "Gram product too wide");
  const size_t lds = size_t(GRAM_RB) * (ra + rb) * sizeof(double);
  k_gram_partial<TA, TB><<<GRAM_CHUNKS, 1024, lds, st>>>(n, A, lda, ra, B, ldb, rb, work);
  NS_LAUNCH_CHECK();
  k_gram_final<<<(nout + 255) / 256, 256, 0, st>>>(GRAM_CHUNKS, nout, work, G, alpha, beta);
  NS_LAUNCH_CHECK();
}

size_t gram_work_elems(int maxw) { return size_t(GRAM_CHUNKS) * maxw * maxw; }

template <class T>
void ts_update(int64_t n, int ncols, T* Out, int64_t ldo, double beta, double gamma, const T* X, int64_t ldx, int rm,
               const double* M, int64_t ldm, const T* X2, int64_t ldx2, int rm2, const double* M2, int64_t ldm2,
               hipStream_t st) {
  if (n == 0 || ncols == 0) return;
  dim3 g(unsigned((n + 63) / 64), unsigned((ncols + 31) / 32));
  const size_t lds = size_t(rm + rm2) * 32 * sizeof(double);
  k_ts_update<T><<<g, 256, lds, st>>>(n, ncols, Out, ldo, beta, gamma, X, ldx, rm, M, ldm, X2, ldx2, rm2, M2, ldm2);
  NS_LAUNCH_CHECK();
}

template <class T, class U>
void convert_block(int64_t n, int ncols, const T* X, int64_t ldx, U* Y, int64_t ldy, hipStream_t st) {
  if (n == 0 || ncols == 0) return;
  const int64_t tot = n * ncols;
  k_convert<T, U><<<unsigned((tot + 255) / 256), 256, 0, st>>>(n, ncols, X, ldx, Y, ldy);
  NS_LAUNCH_CHECK();
}

template <class T>
void col_sumsq(int64_t n, int ncols, const T* X, int64_t ldx, double* out, double* work, hipStream_t st) {
  if (ncols == 0) return;
  const int nb = 240;
  k_colsq_partial<T><<<nb, 256, 0, st>>>(n, ncols, X, ldx, work);
  NS_LAUNCH_CHECK();
  k_gram_final<<<(ncols + 255) / 256, 256, 0, st>>>(nb, ncols, work, out, 1.0, 0.0);
  NS_LAUNCH_CHECK();
}

constexpr int VEC_BLOCKS = 480;

void dot(int64_t n, const double* x, const double* y, double* out, double* work, hipStream_t st) {
  k_dot_partial<<<VEC_BLOCKS, 256, 0, st>>>(n, x, y, work);
  NS_LAUNCH_CHECK();
  k_sum_final<<<1, 256, 0, st>>>(VEC_BLOCKS, work, out);
  NS_LAUNCH_CHECK();
}

void pcg_update_wr(int64_t n, const double* sc, int it, double* w, double* r, const double* p, const double* q,
                   double* rn2_out, double* work, hipStream_t st) {
  k_pcg_wr<<<VEC_BLOCKS, 256, 0, st>>>(n, sc, it, w, r, p, q, work);
  NS_LAUNCH_CHECK();
  k_sum_final<<<1, 256, 0, st>>>(VEC_BLOCKS, work, rn2_out);
  NS_LAUNCH_CHECK();
}

void pcg_update_p(int64_t n, const double* sc, int it, const double* z, double* p, hipStream_t st) {
  k_pcg_p<<<VEC_BLOCKS, 256, 0, st>>>(n, sc, it, z, p);
  NS_LAUNCH_CHECK();
}

void axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
  k_axpby<<<VEC_BLOCKS, 256, 0, st>>>(n, a, x, b, y);
  NS_LAUNCH_CHECK();
}

template void gram<double, double>(int64_t, const double*, int64_t, int, const double*, int64_t, int, double*, double,
                                   double, double*, hipStream_t);
template void gram<float, float>(int64_t, const float*, int64_t, int, const float*, int64_t, int, double*, double,
                                 double, double*, hipStream_t);
template void ts_update<double>(int64_t, int, double*, int64_t, double, double, const double*, int64_t, int,
                                const double*, int64_t, const double*, int64_t, int, const double*, int64_t,
                                hipStream_t);
template void ts_update<float>(int64_t, int, float*, int64_t, double, double, const float*, int64_t, int,
                               const double*, int64_t, const float*, int64_t, int, const double*, int64_t,
                               hipStream_t);
template void convert_block<double, float>(int64_t, int, const double*, int64_t, float*, int64_t, hipStream_t);
template void convert_block<float, double>(int64_t, int, const float*, int64_t, double*, int64_t, hipStream_t);
template void convert_block<double, double>(int64_t, int, const double*, int64_t, double*, int64_t, hipStream_t);
template void col_sumsq<double>(int64_t, int, const double*, int64_t, double*, double*, hipStream_t);
template void col_sumsq<float>(int64_t, int, const float*, int64_t, double*, double*, hipStream_t);

}  // namespace ns
