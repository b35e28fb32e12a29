// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace ns {

// Dense blocks are stored as TILE x TILE tiles.
constexpr int TILE = 64;
constexpr int TILE2 = TILE * TILE;

// Status codes (mirror ns_status of the public header).
enum Status { OK = 0, INVALID_ARG = 1, NOT_SPD = 2, OOM = 3, HIP = 4, NOT_CONVERGED = 5, BREAKDOWN = 6 };

struct Error {
  int status;
  std::string msg;
};

[[noreturn]] void fail(int status, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define NS_HIP(call) ::ns::hip_check((call), #call, __FILE__, __LINE__)
#define NS_LAUNCH_CHECK() ::ns::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// Device memory comes from a per-device cache of blocks: every library call
// sets the stream its buffers are allocated and freed on (StreamScope); a
// freed block is reused at once by later allocations on the same stream (work
// already queued on it still reads the block before any new work) and by other
// streams once an event recorded at the free has completed.  Blocks are
// obtained with hipMalloc on a miss and kept until the process ends (or an
// allocation fails, which first returns the idle blocks to the driver).
hipStream_t& alloc_stream();  // thread-local; the null stream outside a call
struct StreamScope {
  hipStream_t prev;
  // Every library call opens one: an error code left by an earlier call whose result was deliberately
  // ignored (an event query) is cleared so that the launch checks of this call report only its own launches.
  explicit StreamScope(hipStream_t s) : prev(alloc_stream()) {
    alloc_stream() = s;
    (void)hipGetLastError();
  }
  ~StreamScope() { alloc_stream() = prev; }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};
void* dev_alloc(size_t bytes);  // throws OOM
void dev_free(void* p);         // back to the cache, ordered on alloc_stream()
// Host-to-device copy ordered on st that returns at once: the bytes are first
// copied into a pinned staging area of the calling thread (src may be freed on
// return).  A staging area is reused only after the copies from it completed.
void upload(void* dst, const void* src, size_t bytes, hipStream_t st);
// Tells the staging area that stream st has been synchronised.
void stream_idle(hipStream_t st);
// A small pinned host buffer of the calling thread (at most 4 KiB; allocated on first use and kept until the
// process ends) for device-to-host copies the host waits for through an event.
void* pinned_scratch(size_t bytes);

// Owning device buffer.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    p = static_cast<T*>(dev_alloc(count * sizeof(T)));
    n = count;
  }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  operator T*() const { return p; }
};

// Tile band storage.  A block of nt tile rows whose nonzeros lie within nbt
// tile diagonals below the main one (0 <= nbt <= nt - 1; nbt = nt - 1 is the
// full lower tile triangle) stores, tile column by tile column, the tiles
// (j, j), (j + 1, j), ..., (min(nt - 1, j + nbt), j).  The Cholesky factor of
// a band matrix keeps the band, so the factor lives in the same storage.
// Visit the entries e0 .. e1-1 of a CSR row in index order as f(value, X[col[e] * ldx + c]) (value 1 when val
// is null).  The index, value and X loads of four entries are issued together from clamped in-bounds positions
// (a row's entries are otherwise a chain of dependent loads, each waiting for the last); entries past the row
// end are loaded but not visited.
template <class T, class F>
__device__ __forceinline__ void csr_row_visit(int64_t e0, int64_t e1, const int32_t* __restrict__ col,
                                              const T* __restrict__ val, const T* __restrict__ X, int64_t ldx, int c,
                                              F&& f) {
  for (int64_t e = e0; e < e1; e += 4) {
    int j[4];
    T v[4], x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t ek = e + k < e1 ? e + k : e;
      j[k] = col[ek];
      v[k] = val ? val[ek] : T(1);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = X[int64_t(j[k]) * ldx + c];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (e + k < e1) f(v[k], x[k]);
  }
}

__host__ __device__ inline int64_t band_col_off(int nt, int nbt, int j) {
  const int a = nt - nbt;  // tile columns that hold nbt + 1 tiles
  if (j <= a) return int64_t(j) * (nbt + 1);
  const int64_t m = j - a;
  return int64_t(a) * (nbt + 1) + m * nt - m * (a + j - 1) / 2;
}
__host__ __device__ inline int64_t band_tile_index(int nt, int nbt, int i, int j) {  // tile (i, j), 0 <= i - j <= nbt
  return band_col_off(nt, nbt, j) + (i - j);
}
// Element (r, c), r >= c, of a band tile block (tiles TILE x TILE column-major).
__host__ __device__ inline int64_t band_elem(int nt, int nbt, int r, int c) {
  return band_tile_index(nt, nbt, r >> 6, c >> 6) * TILE2 + (c & 63) * TILE + (r & 63);
}
// Tile half-bandwidth that holds an element half-bandwidth bw of an n-row block.
inline int band_tiles_for(int n, int bw) {
  const int nt = (n + TILE - 1) / TILE;
  return nt == 0 ? 0 : std::min(nt - 1, (bw + TILE - 1) / TILE);
}

// A batch of SPD blocks in band tile storage.
//   Block b has nb[b] rows, padded to nt[b] * TILE; padding rows carry an
//   identity diagonal so the padded block stays SPD and leaves padded
//   right-hand-side rows at zero.  bw[b] is the element half-bandwidth of the
//   block (largest r - c of a nonzero) and nbt[b] the tile half-bandwidth.
//   Factor tiles: band storage above, block b's first tile at element foff[b].
//   Inverse diagonal tiles: nt[b] tiles from element ioff[b].
//   Padded rows of block b start at row roff[b] of a padded right-hand side.
// layout() sets the row layout; layout_band() the band and the factor storage.
// Symmetric blocks in packed lower tile storage for single-column products
// y_b = A_b x_b: block b (dimension dim_b, mt_b = ceil(dim_b / 64) tile rows)
// keeps the tiles (ti, tj), tj <= ti, row-major 64 x 64 each, at tile index
// toff_b + ti (ti + 1) / 2 + tj (zero beyond dim_b).  Each tile is read once
// and serves both A_{ti,tj} x_tj and A_{ti,tj}^T x_ti; the per-tile partial
// results are summed in a fixed order.  x_b and y_b start at row xoff_b of x
// and y (device offsets owned by the caller's structure).
struct SymPacked {
  int nblk = 0, max_tiles = 0, max_mt = 0;
  int64_t total_tiles = 0;
  DBuf<int> mt, dim;
  DBuf<int64_t> toff, pboff;
  const int64_t* xoff = nullptr;
  DBuf<double> tiles, part;
  double alg_bytes = 0, alg_flops = 0;  // per product: distinct entries read, 2 dim^2 flops
  bool built() const { return tiles.p != nullptr; }
};
// Pack block b of src (dim_b x dim_b at src + src_off[b], leading dimension src_ld[b]; device arrays).
void sym_pack(SymPacked& sp, const std::vector<int>& dims, const double* src, const int64_t* src_off,
              const int64_t* src_ld, const int64_t* xoff, hipStream_t st);
// The layout and storage of sym_pack without filling the tiles (a producer writes them: tile (ti, tj) of block b,
// row-major, at tile index toff_b + ti (ti + 1) / 2 + tj, zero beyond dim_b).
void sym_layout(SymPacked& sp, const std::vector<int>& dims, const int64_t* xoff, hipStream_t st);
// y_b = A_b x_b for every block (one column).
// y = S x per block; block b's vector is x[xoff_b ..], or with xidx gathered as x[xidx[xoff_b + r]] (-1: 0).
void sym_gemv(const SymPacked& sp, const double* x, double* y, hipStream_t st, const int32_t* xidx = nullptr);

struct TileLevel {
  int role = 0;  // 0: interior blocks, 1: interface blocks (timing family)
  int nblk = 0;
  int max_nt = 0, max_nbt = 0;
  std::vector<int> h_nb, h_nt, h_bw, h_nbt;
  std::vector<int64_t> h_foff, h_ioff, h_roff;
  int64_t nrows_pad = 0, f_elems = 0, i_elems = 0;
  DBuf<int> nt, nb, nbt;
  DBuf<int64_t> foff, ioff, roff;
  DBuf<double> L64, Linv64;
  DBuf<float> L32, Linv32;
  DBuf<double> LT64;  // tile-wise transposed factor (single-column backward sweeps)
  // explicit inverses of the (small) blocks: rows nrows_pad x inv_ld, block b at row roff_b
  DBuf<double> Ainv64;
  DBuf<float> Ainv32;
  DBuf<uint16_t> Ainv16;  // BF16 copy (NS_BF16 inner operators)
  DBuf<int64_t> inv_off, inv_lda;
  DBuf<int> npad_d;
  int64_t inv_ld = 0;
  SymPacked inv_sym;  // the FP64 inverses packed for single-column applies
  // algorithmic work: factor entries (band lower triangle), flops of one
  // triangular sweep per right-hand side, rows; per tile column of the
  // factorisation: update flops, panel flops, bytes
  double alg_tri = 0, alg_sq = 0, alg_rows = 0;
  std::vector<double> chol_upd_flops, chol_pan_flops, chol_bytes;
  void layout(const std::vector<int>& sizes);   // host: row layout + index arrays
  void layout_band(const std::vector<int>& bw);  // host: band, factor storage (allocates L64, Linv64)
};

// ---------------------------------------------------------------- tuned settings
// The tuned value of an automatic setting (kernel: "trsm_cols", "pcg_graph_iters", "bcg_graph_iters",
// "ls_gemm_cols"; prec: "f64", "f32", "bf16") for a size, from the table beside the library, else fallback.
int tuned(const char* kernel, const char* prec, int64_t size, int fallback);

// ---------------------------------------------------------------- kernel timing
// Families of launches that can be timed with HIP events (opt-in, ABI
// nystrom_schur_kernel_timing / nystrom_schur_kernel_stats).
enum KFamily {
  KF_CHOL_UPDATE = 0,
  KF_CHOL_PANEL,
  KF_TRSM_I64,  // interior blocks, FP64
  KF_TRSM_I32,  // interior blocks, FP32
  KF_TRSM_G64,  // interface blocks (level 2 and junction), FP64
  KF_TRSM_G32,
  KF_SCHUR_EPI,
  KF_SPMM,
  KF_LS_FORM,     // local Schur blocks: S_j = W_j^T W_j
  KF_LS_APPLY64,  // local Schur blocks applied (batched GEMM), FP64
  KF_LS_APPLY32,
  KF_INV64,  // explicit interface-block inverses applied, FP64
  KF_INV32,
  KF_MLP_FWD,  // learned proposal: network forward GEMMs (BF16 MFMA)
  KF_MLP_BWD,  // learned proposal: backward GEMMs (FP32 MFMA)
  KF_LS_APPLY16,  // local Schur blocks applied with BF16 operands (FP32 accumulation)
  KF_INV16,       // interface-block inverses applied with BF16 operands
  KF_GRAM,        // Gram products A^T B of block vectors, both sides wider than 16 columns (block CG, Nystrom)
  KF_BLOCK_UPDATE,  // block updates Out = beta Out + gamma X M of more than 16 columns (block CG, Nystrom)
  KF_SMALL,       // one-workgroup dense kernels on the s x s matrices
  KF_GRAM_NARROW,          // Gram products with one side of at most 16 columns (Z^T r of the PCG apply)
  KF_BLOCK_UPDATE_NARROW,  // block updates of at most 16 output columns (Z c of the PCG apply)
  KF_LS_APPLY64_NARROW,    // local Schur blocks applied to at most 16 FP64 columns (the PCG's S_Gamma p)
  KF_INV64_NARROW,         // interface-block inverses applied to at most 16 FP64 columns (the PCG's M r)
  KF_COUNT
};
// Brackets one launch when timing is on; bytes / flops are the algorithmic
// work of the launch (what the method must move / compute, no padding).
// True while kernel timing covers a family that runs inside the block-CG (pcg false) or the PCG (pcg true)
// iterations: that loop then uses plain launches (launches recorded into a graph cannot be timed one by one).
bool kernel_timing_in_loops(bool pcg);
struct KScope {
  int fam;
  hipStream_t st;
  double bytes, flops;
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  KScope(int fam, hipStream_t st, double bytes = 0.0, double flops = 0.0);
  ~KScope();
};
// Adds work to a family's totals when timing is on (work known only after its launches were queued).
void kscope_add_work(int fam, double bytes, double flops);

// ---------------------------------------------------------------- dense tiles
// Batched Cholesky of all blocks of a level (FP64, in place), with inverted
// diagonal tiles.  err[0..2] = (flag, block, column) of the first pivot <= 0.
void tile_cholesky(TileLevel& lv, int* d_err, hipStream_t st);
// Convert the FP64 factor of a level to FP32 (allocates L32/Linv32).
void tile_make_fp32(TileLevel& lv, hipStream_t st);
// In-place solve (L L^T) X = B on a padded right-hand side (rows lv.nrows_pad,
// row-major with leading dimension ldb, ncols columns).
template <class T>
void tile_solve(const TileLevel& lv, T* B, int64_t ldb, int ncols, int cw, hipStream_t st);
// Forward sweep only: B <- L^{-1} B.
// ncols_blk: optional per-block column count (chunks beyond it are skipped);
// first_tile: optional [block * nchunks + chunk] first tile row with a nonzero
// right-hand side (rows above stay zero); alg_flops >= 0 overrides the timing work.
// Blocks b0 .. b1-1 only (b1 < 0: all), with B holding the padded rows from row0 on.
// A right-hand side given by columns of at most SPARSE_RHS_CAP entries: column c of block b (b counted from
// b0, c < ld) has cnt[b * ld + c] entries, local row row[(b * ld + c) * CAP + e] and value val[...]; every
// other entry is zero.  With it the sweep reads no right-hand side from B and writes every tile row from the
// chunk's first tile on (rows above are left as they are: callers do not read them).
constexpr int SPARSE_RHS_CAP = 4;
struct SparseRhs {
  const int* cnt = nullptr;
  const int* row = nullptr;
  const double* val = nullptr;
  int64_t ld = 0;
};
template <class T>
void tile_solve_fwd(const TileLevel& lv, T* B, int64_t ldb, int ncols, int cw, hipStream_t st,
                    const int* ncols_blk = nullptr, const int* first_tile = nullptr, double alg_flops = -1.0,
                    int b0 = 0, int b1 = -1, int64_t row0 = 0, int family = -1,  // -1: by the level's role
                    const SparseRhs* sparse = nullptr);
// Backward sweep only: B <- L^{-T} B (every block, padded rows).
template <class T>
void tile_solve_bwd(const TileLevel& lv, T* B, int64_t ldb, int ncols, int cw, hipStream_t st);
// The FP64 64-column forward sweep of every block of lv can take a SparseRhs (band of at most 4 tiles).
bool tile_sparse_rhs_ok(const TileLevel& lv);
// Single right-hand side sweeps (FP64) with 16-wave workgroups; need LT64.
bool trsv1_supported(const TileLevel& lv);
bool trsv1_supported_size(const TileLevel& lv);  // the block size allows the single-column sweeps
void tile_make_transposed(TileLevel& lv, hipStream_t st);
void tile_solve1(const TileLevel& lv, double* B, int64_t ldb, hipStream_t st);
// Explicit inverses (L L^T)^{-1} of every block of a level (FP64, optional FP32 copy).
void tile_make_inverse(TileLevel& lv, bool fp32, hipStream_t st);
// B = A^{-1} B (forward and backward sweeps, 64-column chunks) for a right-hand side whose chunk c of block b
// is zero above tile row first_tile[b * chunks + c] (a value >= the block's tile count: the chunk is zero).
void tile_solve_chunks(const TileLevel& lv, double* B, int64_t ldb, int ncols, const int* first_tile,
                       hipStream_t st);
// C_b = Y_b^T Y_b for the lower triangular Y_b of every block of lv (stacked at the offsets inv_off, leading
// dimension ld; kstart[b * kstride + t]: first tile row holding a nonzero of column tile t): the tiles on
// and below the diagonal are formed from that row on and mirrored.
void tri_gram(const TileLevel& lv, const double* Y, double* C, int64_t ld, const int* kstart, int kstride,
              double alg_flops, hipStream_t st);
// C = A^{-1} B for every block with the explicit inverses; B, C padded rhs (ld ncols).
template <class T>
void tile_apply_inverse(const TileLevel& lv, const T* B, T* C, int ncols, hipStream_t st,
                        const int32_t* bidx = nullptr,  // bidx: B gathered per row (one column, FP64 packed path)
                        bool bf16 = false);             // FP32 data: BF16 operands of the inverses (Ainv16)
// BF16 copy of the FP32 inverses (round to nearest even), for the BF16 inner operators.
void tile_make_bf16_inverse(TileLevel& lv, hipStream_t st);
// Expand the factor of one block to a dense nb x nb column-major lower matrix.
void tile_export(const TileLevel& lv, int block, double* out, hipStream_t st);

// ---------------------------------------------------------------- sparse
// In-place inclusive scan of a[0..m) (int64).  Synchronises st.
void scan_inclusive(int64_t* a, int64_t m, hipStream_t st);

struct Csr {
  int64_t nrows = 0, nnz = 0;
  DBuf<int64_t> ptr;
  DBuf<int32_t> col;
  DBuf<double> val64;
  DBuf<float> val32;
};

}  // namespace ns
