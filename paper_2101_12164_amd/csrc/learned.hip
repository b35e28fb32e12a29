// Learned starting subspace for the deflation: interface-node features, a
// three-layer MLP (d_in -> h -> h -> k, ReLU hidden layers) with BF16 operands
// on MFMA and FP32 accumulation, its backward pass, the subspace loss
//   L = 1 - tr(G^{-1} Z0^T U U^T Z0) / k,  G = Z0^T Z0,
// with dL/dZ0 = -(2/k) (I - Z0 G^{-1} Z0^T) U U^T Z0 G^{-1}, and Adam on FP32
// master weights.  The proposal Z0 feeds the adapted deflation (eqs.
// adapted_deflation_prec, deflation_comp_from_low_rank) through setup, which
// judges it by Rayleigh-Ritz.
#include <cmath>
#include <cstring>

#include "ns_handle.h"
#include "ns_vec.h"

namespace ns {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int D_FEAT = 16;

__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// ------------------------------------------------------------------ features
// Per interface node (interface index a = gidx[i]): the row-local features and s0 = log A_ii.
__global__ void k_feat_rows(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, const int32_t* __restrict__ part,
                            const int64_t* __restrict__ gpos, const double* __restrict__ coords,
                            double* __restrict__ F, double* __restrict__ s0, int* __restrict__ deg) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || part[i] >= 0) return;
  const int64_t a = gpos[i] - 1;
  double diag = 0.0, lsum = 0.0, lmin = 0.0, lmax = 0.0, s_int = 0.0, s_gam = 0.0;
  int nl = 0, ng = 0;
  int subs[16];
  int nsub = 0;
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
    const int j = col[e];
    if (j < 0 || j >= n) continue;  // the CSR is not validated by this entry point
    const double v = val[e];
    if (j == i) {
      diag = v;
      continue;
    }
    if (v != 0.0) {
      const double lv = log(fabs(v));
      lmin = nl ? fmin(lmin, lv) : lv;
      lmax = nl ? fmax(lmax, lv) : lv;
      lsum += lv;
      ++nl;
    }
    const int pj = part[j];
    if (pj >= 0) {
      s_int += fabs(v);
      bool seen = false;
      for (int t = 0; t < nsub; ++t) seen = seen || subs[t] == pj;
      if (!seen && nsub < 16) subs[nsub++] = pj;
    } else {
      s_gam += fabs(v);
      ++ng;
    }
  }
  double* f = F + a * D_FEAT;
  for (int c = 0; c < 3; ++c) f[c] = coords ? coords[i * 3 + c] : 0.0;
  f[3] = log(diag);
  f[4] = nl ? lsum / nl : 0.0;
  f[5] = nl ? lmin : 0.0;
  f[6] = nl ? lmax : 0.0;
  f[7] = log(1e-30 + s_int);
  f[8] = log(1e-30 + s_gam);
  f[9] = part[i] == -1 ? 1.0 : 0.0;
  f[10] = nsub / 4.0;
  f[14] = ng / 8.0;
  f[15] = 1.0;
  s0[a] = f[3];
  deg[a] = ng;
}

// one averaging step of s over the interface graph: t_a = (s_a + sum_{interface neighbours} s_b) / (1 + deg_a)
__global__ void k_feat_smooth(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                              const int32_t* __restrict__ part, const int64_t* __restrict__ gpos,
                              const int* __restrict__ deg, const double* __restrict__ s, double* __restrict__ t) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || part[i] >= 0) return;
  const int64_t a = gpos[i] - 1;
  double acc = 0.0;
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
    const int j = col[e];
    if (j >= 0 && j < n && j != i && part[j] < 0) acc += s[gpos[j] - 1];
  }
  t[a] = (s[a] + acc) / (1.0 + deg[a]);
}

__global__ void k_flag_interface(int64_t n, const int32_t* __restrict__ part, int64_t* __restrict__ g) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) g[i] = part[i] < 0 ? 1 : 0;
}

__global__ void k_feat_out(int64_t ng, const double* __restrict__ F, const double* __restrict__ s1,
                           const double* __restrict__ s2, const double* __restrict__ s4, float* __restrict__ X) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= ng) return;
  for (int c = 0; c < D_FEAT; ++c) {
    double v = F[a * D_FEAT + c];
    if (c == 11) v = s1[a];
    if (c == 12) v = s2[a];
    if (c == 13) v = s4[a];
    X[a * D_FEAT + c] = float(v);
  }
}

// ------------------------------------------------------------------ BF16 GEMM on MFMA
// C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn] (BF16).
// One workgroup: 64 x 64 output tile, wave w rows [16 w, 16 w + 16), four 16 x 16 MFMA blocks.
// gfx950 MFMA 16x16x32 BF16 operands: lane l holds A(l % 16, 8 (l / 16) + t) and B(8 (l / 16) + t, l % 16),
// t = 0..7; the FP32 result element v of lane l is C(4 (l / 16) + v, l % 16).
// OUT 0: BF16 out = act(acc + bias); OUT 2: FP64 out = acc + bias.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8 bf16x8_of(const uint16_t (&u)[8]) {
  bf16x8 r;
#pragma unroll
  for (int t = 0; t < 8; ++t) r[t] = __builtin_bit_cast(__bf16, u[t]);
  return r;
}
template <int OUT>
__global__ __launch_bounds__(256) void k_bgemm(int M, int N, int K, const uint16_t* __restrict__ A, int64_t sam,
                                               int64_t sak, const uint16_t* __restrict__ B, int64_t sbk,
                                               int64_t sbn, const float* __restrict__ bias, int relu,
                                               const uint16_t* __restrict__ mask, int64_t ldm, void* Cv,
                                               int64_t ldc, int kchunk) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + 16 * w, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int li = lane & 15, lk = 8 * (lane >> 4), lr = 4 * (lane >> 4);
  f4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
  const int am = m0 + li;
  // operands are loaded unconditionally from clamped in-bounds positions and zeroed afterwards, so the forty
  // loads of a k-step are in flight together (a load under a per-lane condition waits behind its own branch)
  const int amc = min(am, M - 1);
  for (int k0 = kb; k0 < ke; k0 += 32) {
    uint16_t av[8], bv[4][8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kc = min(k0 + lk + t, ke - 1);
      av[t] = A[int64_t(amc) * sam + int64_t(kc) * sak];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q][t] = B[int64_t(kc) * sbk + int64_t(min(n0 + 16 * q + li, N - 1)) * sbn];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (!(am < M && k0 + lk + t < ke)) av[t] = 0;
    const bf16x8 a = bf16x8_of(av);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int bn = n0 + 16 * q + li;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (!(bn < N && k0 + lk + t < ke)) bv[q][t] = 0;
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bf16x8_of(bv[q]), acc[q], 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cn = n0 + 16 * q + li;
    if (cn >= N) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cm = m0 + lr + v;
      if (cm >= M) continue;
      float x = acc[q][v];
      if constexpr (OUT == 0) {
        if (bias) x += bias[cn];
        if (relu) x = fmaxf(x, 0.f);
        static_cast<uint16_t*>(Cv)[int64_t(cm) * ldc + cn] = f2bf(x);
      } else {
        static_cast<double*>(Cv)[int64_t(cm) * ldc + cn] = double(x) + (bias ? double(bias[cn]) : 0.0);
      }
    }
  }
}

// FP32 GEMM on MFMA (16x16x4 f32) for the backward pass: operands are FP32 or BF16 (converted on load),
// C(m, n) = sum_k A(m, k) B(k, n) with the same strided addressing and tiling as k_bgemm.
// 16x16x4 f32 operands: lane l holds A(l % 16, l / 16) and B(l / 16, l % 16); result as for k_bgemm.
// OUT 1: FP32 partial per k chunk (grid.z); OUT 3: FP32 out * (mask > 0).
template <class T>
__device__ __forceinline__ float ldf(const T* p, int64_t i) {
  if constexpr (sizeof(T) == 2)
    return bf2f(p[i]);
  else
    return p[i];
}

template <class TA, class TB, int OUT>
__global__ __launch_bounds__(256) void k_fgemm(int M, int N, int K, const TA* __restrict__ A, int64_t sam,
                                               int64_t sak, const TB* __restrict__ B, int64_t sbk, int64_t sbn,
                                               const uint16_t* __restrict__ mask, int64_t ldm,
                                               float* __restrict__ C, int64_t ldc, int kchunk) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + 16 * w, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int li = lane & 15, lk = lane >> 4;
  f4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
  const int am = m0 + li, amc = min(am, M - 1);
  // four k-steps per batch, every operand loaded unconditionally from a clamped in-bounds position (zeroed
  // afterwards), so the twenty loads of a batch are in flight together
  constexpr int U = 4;
  for (int k0 = kb; k0 < ke; k0 += 4 * U) {
    float av[U], bv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kc = min(k0 + 4 * u + lk, ke - 1);
      av[u] = ldf(A, int64_t(amc) * sam + int64_t(kc) * sak);
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[u][q] = ldf(B, int64_t(kc) * sbk + int64_t(min(n0 + 16 * q + li, N - 1)) * sbn);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool kin = k0 + 4 * u + lk < ke;
      const float a = (am < M && kin) ? av[u] : 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float b = (n0 + 16 * q + li < N && kin) ? bv[u][q] : 0.f;
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cn = n0 + 16 * q + li;
    if (cn >= N) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int cm = m0 + 4 * lk + v;
      if (cm >= M) continue;
      float x = acc[q][v];
      if constexpr (OUT == 1) {
        C[(int64_t(blockIdx.z) * M + cm) * ldc + cn] = x;
      } else {
        if (mask && !(bf2f(mask[int64_t(cm) * ldm + cn]) > 0.f)) x = 0.f;
        C[int64_t(cm) * ldc + cn] = x;
      }
    }
  }
}

// out[e] = sum_z part[z * MN + e] (fixed order)
__global__ void k_sum_partials(int64_t MN, int nz, const float* __restrict__ part, float* __restrict__ out) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= MN) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += part[int64_t(z) * MN + e];
  out[e] = s;
}

// column sums of an FP32 n x N matrix (bias gradients): stage 1 sums rows [z * RC, (z + 1) * RC) per column
// (grid.y = z), stage 2 adds the partials in a fixed order
constexpr int COLSUM_ROWS = 256;
__global__ void k_colsum_part(int64_t n, int N, const float* __restrict__ X, float* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int64_t r0 = int64_t(blockIdx.y) * COLSUM_ROWS, r1 = min(n, r0 + COLSUM_ROWS);
  float s = 0.f;
  for (int64_t r = r0; r < r1; ++r) s += X[r * N + c];
  part[int64_t(blockIdx.y) * N + c] = s;
}

__global__ void k_to_bf(int64_t m, const float* __restrict__ x, uint16_t* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) y[i] = f2bf(x[i]);
}
__global__ void k_d_to_f(int64_t m, const double* __restrict__ x, float* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) y[i] = float(x[i]);
}

// loss = 1 - sum_ij X_ij M_ij / k with X = G^{-1} M; P1 = -(2/k) X^T, P2 = (2/k) X X^T
__global__ void k_loss_mats(int k, const double* __restrict__ X, const double* __restrict__ Mm, double* __restrict__ P1,
                            double* __restrict__ P2, double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int i = e / k, j = e % k;
    s += X[e] * Mm[e];
    P1[e] = -(2.0 / k) * X[j * k + i];
    double t = 0.0;
    for (int c = 0; c < k; ++c) t += X[i * k + c] * X[j * k + c];
    P2[e] = (2.0 / k) * t;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = 1.0 - red[0] / k;
}

__global__ void k_adam(int64_t m, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ mo,
                       float* __restrict__ vo, float lr, float b1, float b2, float c1, float c2, float eps) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float gi = g[i];
  const float a = b1 * mo[i] + (1.f - b1) * gi;
  const float b = b2 * vo[i] + (1.f - b2) * gi * gi;
  mo[i] = a;
  vo[i] = b;
  p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

unsigned blocks(int64_t m) { return unsigned((m + 255) / 256); }

}  // namespace
}  // namespace ns

using namespace ns;

// The network: FP32 master parameters (flat: W1 d_in x h, b1, W2 h x h, b2, W3 h x k, b3; weights row-major
// in x out), BF16 copies of the weights, Adam moments, the gradient and the activation workspaces.
struct ns_mlp_s {
  int d_in = 0, h = 0, k = 0;
  int64_t np = 0;          // parameters
  int64_t off[6] = {};     // offsets of W1, b1, W2, b2, W3, b3
  DBuf<float> p, g, m1, m2;
  DBuf<uint16_t> wb;       // BF16 weights, same layout (biases unused)
  int64_t steps = 0;
  int64_t cap = 0;         // rows the workspaces hold
  DBuf<uint16_t> Xb, H1, H2;
  DBuf<float> dZf, dH1, dH2;
  DBuf<double> Z0, dZ;
  DBuf<float> part, cpart;
  // loss workspaces, sized for `cap` rows
  SegBuf seg;
  int64_t seg_rows = -1;
  DBuf<double> small, work, gs;
  SmallWs gsw;
  DBuf<int> flag;
  DBuf<double> lossd;
  std::string last_error;
  hipEvent_t ev = nullptr;       // recorded at the end of every call
  hipStream_t last = nullptr;    // stream of the previous call
  hipStream_t own = nullptr;     // the network's own stream (initialisation, parameter copies)
};

namespace ns {
namespace {

void mlp_layout(ns_mlp_s& m) {
  const int64_t sz[6] = {int64_t(m.d_in) * m.h, m.h, int64_t(m.h) * m.h, m.h, int64_t(m.h) * m.k, m.k};
  int64_t o = 0;
  for (int t = 0; t < 6; ++t) {
    m.off[t] = o;
    o += sz[t];
  }
  m.np = o;
}

void mlp_refresh_bf(ns_mlp_s& m, hipStream_t st) {
  k_to_bf<<<blocks(m.np), 256, 0, st>>>(m.np, m.p, m.wb);
  NS_LAUNCH_CHECK();
}

void mlp_workspace(ns_mlp_s& m, int64_t n) {
  if (n <= m.cap) return;
  m.Xb.alloc(n * m.d_in);
  m.H1.alloc(n * m.h);
  m.H2.alloc(n * m.h);
  m.dH1.alloc(n * m.h);
  m.dH2.alloc(n * m.h);
  m.dZf.alloc(n * m.k);
  m.Z0.alloc(n * m.k);
  m.dZ.alloc(n * m.k);
  m.cap = n;
}

template <int OUT>
void bgemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
           int64_t sbn, const float* bias, int relu, const uint16_t* mask, int64_t ldm, void* C, int64_t ldc,
           int kchunk, hipStream_t st) {
  // algorithmic work: 2 M N K flops; operands read once, the output written once
  KScope ks(KF_MLP_FWD, st, (double(M) * K + double(K) * N) * 2.0 + double(M) * N * (OUT == 2 ? 8.0 : 2.0),
            2.0 * M * N * double(K));
  const int nz = (K + kchunk - 1) / kchunk;
  dim3 grid((N + 63) / 64, (M + 63) / 64, nz);
  k_bgemm<OUT><<<grid, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, bias, relu, mask, ldm, C, ldc, kchunk);
  NS_LAUNCH_CHECK();
}

// forward: Xb, H1, H2 (BF16), Z0 (FP64)
void mlp_forward(ns_mlp_s& m, const float* X, int64_t n, hipStream_t st) {
  mlp_workspace(m, n);
  const int din = m.d_in, h = m.h, k = m.k;
  k_to_bf<<<blocks(n * din), 256, 0, st>>>(n * din, X, m.Xb);
  NS_LAUNCH_CHECK();
  const uint16_t* W = m.wb.p;
  const float* P = m.p.p;
  bgemm<0>(int(n), h, din, m.Xb, din, 1, W + m.off[0], h, 1, P + m.off[1], 1, nullptr, 0, m.H1, h, din, st);
  bgemm<0>(int(n), h, h, m.H1, h, 1, W + m.off[2], h, 1, P + m.off[3], 1, nullptr, 0, m.H2, h, h, st);
  bgemm<2>(int(n), k, h, m.H2, h, 1, W + m.off[4], k, 1, P + m.off[5], 0, nullptr, 0, m.Z0, k, h, st);
}

template <class TA, class TB, int OUT>
void fgemm(int M, int N, int K, const TA* A, int64_t sam, int64_t sak, const TB* B, int64_t sbk, int64_t sbn,
           const uint16_t* mask, int64_t ldm, float* C, int64_t ldc, int kchunk, hipStream_t st) {
  KScope ks(KF_MLP_BWD, st, double(M) * K * sizeof(TA) + double(K) * N * sizeof(TB) + double(M) * N * 4.0,
            2.0 * M * N * double(K));
  const int nz = (K + kchunk - 1) / kchunk;
  dim3 grid((N + 63) / 64, (M + 63) / 64, nz);
  k_fgemm<TA, TB, OUT><<<grid, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, mask, ldm, C, ldc, kchunk);
  NS_LAUNCH_CHECK();
}

// Gradient of the parameters for dZ (FP64, n x k) into m.g: the exact gradient of the network as evaluated
// (BF16 inputs, weights and activations), with FP32 backward products on MFMA.
void mlp_backward(ns_mlp_s& m, int64_t n, hipStream_t st) {
  const int din = m.d_in, h = m.h, k = m.k;
  const uint16_t* W = m.wb.p;
  float* G = m.g.p;
  constexpr int KC = 1024;  // rows per partial of the weight gradients
  const int nz = int((n + KC - 1) / KC);
  const size_t need = size_t(nz) * std::max<int64_t>(int64_t(h) * h, int64_t(h) * std::max(k, din));
  if (m.part.n < need) m.part.alloc(need);
  k_d_to_f<<<blocks(n * k), 256, 0, st>>>(n * k, m.dZ, m.dZf);
  NS_LAUNCH_CHECK();
  const int nzc = int((n + COLSUM_ROWS - 1) / COLSUM_ROWS);
  const size_t needc = size_t(nzc) * std::max(h, k);
  if (m.cpart.n < needc) m.cpart.alloc(needc);
  auto colsum = [&](const float* X, int N, float* out) {
    k_colsum_part<<<dim3(blocks(N), nzc), 256, 0, st>>>(n, N, X, m.cpart);
    NS_LAUNCH_CHECK();
    k_sum_partials<<<blocks(N), 256, 0, st>>>(N, nzc, m.cpart, out);
    NS_LAUNCH_CHECK();
  };
  auto wgrad = [&](const uint16_t* A, int a_cols, const float* B, int b_cols, float* out) {
    // out (a_cols x b_cols) = A^T B over the n rows, in fixed row chunks
    fgemm<uint16_t, float, 1>(a_cols, b_cols, int(n), A, 1, a_cols, B, b_cols, 1, nullptr, 0, m.part, b_cols, KC,
                              st);
    k_sum_partials<<<blocks(int64_t(a_cols) * b_cols), 256, 0, st>>>(int64_t(a_cols) * b_cols, nz, m.part, out);
    NS_LAUNCH_CHECK();
  };
  // layer 3
  wgrad(m.H2, h, m.dZf, k, G + m.off[4]);
  colsum(m.dZf, k, G + m.off[5]);
  // dH2 = (dZ W3^T) * 1[H2 > 0]
  fgemm<float, uint16_t, 3>(int(n), h, k, m.dZf, k, 1, W + m.off[4], 1, k, m.H2, h, m.dH2, h, k, st);
  wgrad(m.H1, h, m.dH2, h, G + m.off[2]);
  colsum(m.dH2, h, G + m.off[3]);
  // dH1 = (dH2 W2^T) * 1[H1 > 0]
  fgemm<float, uint16_t, 3>(int(n), h, h, m.dH2, h, 1, W + m.off[2], 1, h, m.H1, h, m.dH1, h, h, st);
  wgrad(m.Xb, din, m.dH1, h, G + m.off[0]);
  colsum(m.dH1, h, G + m.off[1]);
}

thread_local std::string g_mlp_error = "no error";

// Calls may come on different streams: a call on another stream than the previous one first waits (on the
// device) for the previous call's work, so buffers that are reused or freed in stream order stay safe.
struct MlpCall {
  ns_mlp_s& m;
  hipStream_t st;
  StreamScope ss;
  MlpCall(ns_mlp_s& m_, hipStream_t s) : m(m_), st(s), ss(s) {
    if (m.ev && s != m.last) NS_HIP(hipStreamWaitEvent(s, m.ev, 0));
  }
  ~MlpCall() {
    if (m.ev) (void)hipEventRecord(m.ev, st);
    m.last = st;
  }
};

ns_status mlp_fail(ns_mlp_s* m, const Error& e) {
  g_mlp_error = e.msg;
  if (m) m->last_error = e.msg;
  return ns_status(e.status);
}

}  // namespace
}  // namespace ns

extern "C" {

ns_status nystrom_schur_features(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                                 const double* val, const int32_t* part, const double* coords, float* X,
                                 int64_t* n_gamma, void* stream) {
  try {
    if (n <= 0 || nnz < 0 || !row_ptr || !col_idx || !val || !part || !X || !n_gamma)
      fail(INVALID_ARG, "bad features arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope ss(st);
    DBuf<int64_t> gpos;
    gpos.alloc(n);
    k_flag_interface<<<blocks(n), 256, 0, st>>>(n, part, gpos);
    NS_LAUNCH_CHECK();
    scan_inclusive(gpos.p, n, st);  // gpos[i] - 1 = interface index of node i
    int64_t ng = 0;
    NS_HIP(hipMemcpyAsync(&ng, gpos.p + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    NS_HIP(hipStreamSynchronize(st));
    *n_gamma = ng;
    if (ng == 0) return NS_OK;
    DBuf<double> F, s0, s1, s2, s3, s4;
    DBuf<int> deg;
    F.alloc(ng * D_FEAT);
    for (DBuf<double>* b : {&s0, &s1, &s2, &s3, &s4}) b->alloc(ng);
    deg.alloc(ng);
    k_feat_rows<<<blocks(n), 256, 0, st>>>(n, row_ptr, col_idx, val, part, gpos, coords, F, s0, deg);
    NS_LAUNCH_CHECK();
    k_feat_smooth<<<blocks(n), 256, 0, st>>>(n, row_ptr, col_idx, part, gpos, deg, s0, s1);
    k_feat_smooth<<<blocks(n), 256, 0, st>>>(n, row_ptr, col_idx, part, gpos, deg, s1, s2);
    k_feat_smooth<<<blocks(n), 256, 0, st>>>(n, row_ptr, col_idx, part, gpos, deg, s2, s3);
    k_feat_smooth<<<blocks(n), 256, 0, st>>>(n, row_ptr, col_idx, part, gpos, deg, s3, s4);
    NS_LAUNCH_CHECK();
    k_feat_out<<<blocks(ng), 256, 0, st>>>(ng, F, s1, s2, s4, X);
    NS_LAUNCH_CHECK();
    NS_HIP(hipStreamSynchronize(st));
    return NS_OK;
  } catch (const Error& e) {
    return mlp_fail(nullptr, e);
  }
}

ns_status nystrom_schur_mlp_create(int32_t d_in, int32_t hidden, int32_t d_out, const float* params, ns_mlp* out) {
  if (out) *out = nullptr;
  ns_mlp_s* m = nullptr;
  try {
    if (!out || !params || d_in < 1 || hidden < 1 || d_out < 1 || d_in > 4096 || hidden > 4096 || d_out > 1024)
      fail(INVALID_ARG, "bad MLP sizes or NULL parameters");
    m = new ns_mlp_s();
    m->d_in = d_in;
    m->h = hidden;
    m->k = d_out;
    mlp_layout(*m);
    // initialisation on a private stream, synchronised alone (no device-wide synchronisation); later calls on
    // any stream wait for it through the network's event
    NS_HIP(hipStreamCreateWithFlags(&m->own, hipStreamNonBlocking));
    StreamScope ss(m->own);
    m->p.alloc(m->np);
    m->g.alloc(m->np);
    m->m1.alloc(m->np);
    m->m2.alloc(m->np);
    m->wb.alloc(m->np);
    NS_HIP(hipEventCreateWithFlags(&m->ev, hipEventDisableTiming));
    NS_HIP(hipMemcpyAsync(m->p.p, params, m->np * sizeof(float), hipMemcpyHostToDevice, m->own));
    NS_HIP(hipMemsetAsync(m->g.p, 0, m->np * sizeof(float), m->own));
    NS_HIP(hipMemsetAsync(m->m1.p, 0, m->np * sizeof(float), m->own));
    NS_HIP(hipMemsetAsync(m->m2.p, 0, m->np * sizeof(float), m->own));
    mlp_refresh_bf(*m, m->own);
    NS_HIP(hipEventRecord(m->ev, m->own));
    m->last = m->own;
    NS_HIP(hipStreamSynchronize(m->own));
    *out = m;
    return NS_OK;
  } catch (const Error& e) {
    ns_status s = mlp_fail(m, e);
    nystrom_schur_mlp_destroy(m);
    return s;
  }
}

ns_status nystrom_schur_mlp_get_params(ns_mlp m, float* params, float* grad) {
  if (!m) return mlp_fail(nullptr, Error{INVALID_ARG, "NULL network"});
  try {
    // after the network's last call (its event), on the network's own stream
    NS_HIP(hipStreamWaitEvent(m->own, m->ev, 0));
    if (params) NS_HIP(hipMemcpyAsync(params, m->p.p, m->np * sizeof(float), hipMemcpyDeviceToHost, m->own));
    if (grad) NS_HIP(hipMemcpyAsync(grad, m->g.p, m->np * sizeof(float), hipMemcpyDeviceToHost, m->own));
    NS_HIP(hipStreamSynchronize(m->own));
    return NS_OK;
  } catch (const Error& e) {
    return mlp_fail(m, e);
  }
}

ns_status nystrom_schur_mlp_forward(ns_mlp m, const float* X, int64_t n, double* Z0, void* stream) {
  if (!m) return mlp_fail(nullptr, Error{INVALID_ARG, "NULL network"});
  try {
    if (!X || !Z0 || n < 1 || n > (int64_t(1) << 30)) fail(INVALID_ARG, "bad forward arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MlpCall call(*m, st);
    mlp_forward(*m, X, n, st);
    NS_HIP(hipMemcpyAsync(Z0, m->Z0.p, n * m->k * sizeof(double), hipMemcpyDeviceToDevice, st));
    NS_HIP(hipStreamSynchronize(st));
    return NS_OK;
  } catch (const Error& e) {
    return mlp_fail(m, e);
  }
}

ns_status nystrom_schur_mlp_loss_grad(ns_mlp m, const float* X, const double* U, int64_t n, double* loss,
                                      void* stream) {
  if (!m) return mlp_fail(nullptr, Error{INVALID_ARG, "NULL network"});
  try {
    if (!X || !U || !loss || n < m->k || n > (int64_t(1) << 30)) fail(INVALID_ARG, "bad loss_grad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MlpCall call(*m, st);
    const int k = m->k;
    mlp_forward(*m, X, n, st);
    if (m->seg_rows != n) {  // loss workspaces for this row count (kept for the next calls)
      m->seg.build({0, n}, st);
      m->seg_rows = n;
      m->work.alloc(gram_work_elems(m->seg.view, k));
    }
    if (!m->small.p) {
      m->small.alloc(size_t(k) * k * 5 + 8);
      m->gsw = small_ws(m->gs, 1, k, k);
      m->flag.alloc(1);
      m->lossd.alloc(1);
    }
    const Seg& sg = m->seg.view;
    double* Gm = m->small.p;
    double* Mm = Gm + k * k;
    double* Xs = Mm + k * k;
    double* P1 = Xs + k * k;
    double* P2 = P1 + k * k;
    double* dl = m->lossd.p;
    NS_HIP(hipMemsetAsync(m->flag.p, 0, sizeof(int), st));
    gram<double, double>(sg, m->Z0.p, k, k, m->Z0.p, k, k, Gm, k * k, 1.0, 0.0, m->work, st);  // G = Z0^T Z0
    gram<double, double>(sg, m->Z0.p, k, k, U, k, k, Mm, k * k, 1.0, 0.0, m->work, st);        // M = Z0^T U
    small_chol_solve(Batch{1, nullptr}, k, Gm, k * k, Mm, k, k * k, Xs, k, k * k, k, k, 1.0, m->flag, m->gsw, st);
    k_loss_mats<<<1, 256, 0, st>>>(k, Xs, Mm, P1, P2, dl);
    NS_LAUNCH_CHECK();
    // dZ = U P1 + Z0 P2
    ts_update<double>(sg, k, m->dZ.p, k, 0.0, 1.0, U, k, k, P1, k, 0, m->Z0.p, k, k, P2, k, 0, st);
    mlp_backward(*m, n, st);
    int fl = 0;
    NS_HIP(hipMemcpyAsync(&fl, m->flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    NS_HIP(hipMemcpyAsync(loss, dl, sizeof(double), hipMemcpyDeviceToHost, st));
    NS_HIP(hipStreamSynchronize(st));
    if (fl) fail(BREAKDOWN, "the proposal Z0 is rank deficient (Z0^T Z0 not positive definite)");
    return NS_OK;
  } catch (const Error& e) {
    return mlp_fail(m, e);
  }
}

ns_status nystrom_schur_mlp_adam_step(ns_mlp m, double lr, void* stream) {
  if (!m) return mlp_fail(nullptr, Error{INVALID_ARG, "NULL network"});
  try {
    if (!(lr > 0.0)) fail(INVALID_ARG, "learning rate must be positive");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MlpCall call(*m, st);
    const float b1 = 0.9f, b2 = 0.999f;
    ++m->steps;
    const float c1 = 1.f - std::pow(b1, float(m->steps)), c2 = 1.f - std::pow(b2, float(m->steps));
    k_adam<<<blocks(m->np), 256, 0, st>>>(m->np, m->p, m->g, m->m1, m->m2, float(lr), b1, b2, c1, c2, 1e-8f);
    NS_LAUNCH_CHECK();
    mlp_refresh_bf(*m, st);  // stream-ordered: the next forward on this stream sees the new weights
    return NS_OK;
  } catch (const Error& e) {
    return mlp_fail(m, e);
  }
}

void nystrom_schur_mlp_destroy(ns_mlp m) {
  if (!m) return;
  // every call waits for the previous one (the network's event), so the last event covers them all
  if (m->ev) (void)hipEventSynchronize(m->ev);
  if (m->own) (void)hipStreamSynchronize(m->own);
  {
    StreamScope ss(m->own);
    hipStream_t own = m->own;
    hipEvent_t ev = m->ev;
    delete m;  // buffers return to the allocator behind the completed work
    if (ev) (void)hipEventDestroy(ev);
    if (own) (void)hipStreamDestroy(own);
  }
}

const char* nystrom_schur_mlp_last_error(ns_mlp m) { return m ? m->last_error.c_str() : g_mlp_error.c_str(); }

}  // extern "C"
