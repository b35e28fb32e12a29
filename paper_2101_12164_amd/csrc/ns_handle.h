// The solver handle and the host-side operator entry points that the C ABI uses.
#pragma once

#include "../../include/nystrom_schur.h"
#include "ns_internal.h"
#include "ns_vec.h"

namespace ns {

// Explicit local Schur complements S_j = (L_j^{-1} B_j)^T (L_j^{-1} B_j), one
// dense m_j x m_j block per subdomain (m_j = interface nodes coupled to it).
// Structure of the local Schur formation handed from its symbolic pass (which reads sizes back to the host)
// to its numeric pass.
struct LocalSchurPlan {
  DBuf<int32_t> rblk, cidx;  // padded interior row -> block; (block, interface index) -> column of B_j
  DBuf<int64_t> gbase_d;     // first interface row of each block's problem
  int64_t ldf = 1, ldw = 1;  // interface rows of the largest problem; columns of the stacked W
  std::vector<int> Kv;       // padded rows of every block
  bool sparse_rhs = false;   // every column of A_{I_j Gamma_j} has at most SPARSE_RHS_CAP entries
};

struct LocalSchur {
  bool built = false;
  LocalSchurPlan plan;
  int nblk = 0, max_m = 0;
  int64_t npos = 0, s_elems = 0;  // stacked (padded) interface rows, S elements
  std::vector<int> h_m;
  DBuf<int> M, K, Kg;                          // per block: m_j, padded rows, m_j
  DBuf<int64_t> goff, soff, sld, wld;          // stacked offsets / leading dimensions
  DBuf<int32_t> glist;                         // stacked position -> interface index (-1 pad)
  DBuf<double> S64;
  DBuf<float> S32;
  DBuf<uint16_t> S16;  // BF16 copy (NS_BF16 inner operators)
  Csr contrib;  // interface row -> stacked positions (values 1)
  DBuf<double> wsX64, wsY64;
  DBuf<float> wsX32, wsY32;
  int64_t ws_cols = 0;
  double alg_bytes = 0, alg_flops = 0;  // per apply and column: sum m_j^2 entries, 2 sum m_j^2 flops
  SymPacked sym;                         // S_j packed for single-column FP64 applies
  DBuf<int> xperm;                       // [8][xplen] blocks of each XCD in the batched applies
  int xplen = 0;
};

}  // namespace ns

struct ns_handle_s {
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;  // second stream of the setup (interface levels), created on first use
  std::string last_error;

  // sizes (a batch of problems is one block-diagonal matrix: totals over the problems)
  int64_t n = 0, nnz = 0, nI = 0, nG = 0, nJ = 0;
  int nsub = 0, nl2 = 0;
  int k = 0, p = 0, s = 0, k_eff = 0;  // k_eff: largest over the problems
  // problems: original rows [h_noff[q], h_noff[q + 1]), interface rows [h_goff[q], h_goff[q + 1])
  int nprob = 1;
  std::vector<int64_t> h_noff, h_goff;
  std::vector<int> h_sub;   // first subdomain of each problem
  ns::DBuf<int64_t> pnode;  // device copy of h_noff
  ns::DBuf<int> l2first;    // first level-2 block of each problem
  ns::SegBuf segG, segN;    // interface rows / original rows by problem
  std::vector<int> h_keff;  // k_eff of each problem
  ns::DBuf<int> keff_d;
  // per-problem inner solve results
  std::vector<int> it_inner, conv_inner;
  std::vector<double> relres_inner;
  int prec_inner = 0, apply_mode = 0, trsm_cols = 0, schur_mode = 0, pcg_graph = 0;
  int variant = 0, power = 0, outer = 0;  // ns_variant, power iterations of the sketch, ns_outer
  int bcg_graph = 0;                       // block-CG iterations per replayed graph (0 auto, -1 plain)
  int bf16 = 0;     // NS_BF16 inner operators built (BF16 copies of S_j and of the interface inverses)
  int op_bf16 = 0;  // FP32 operator applications currently use the BF16 copies
  int bf16_schur = 1;  // the BF16 copies of S_j are used (cleared after a block-CG breakdown on them)
  ns::SegBuf segI;                         // padded interior rows (one problem): the rows of variant M_3
  // recursive level (NS_LEVEL2_NYSTROM): A_Gamma as a DBBD matrix of its own, preconditioned by a handle of
  // its own (interior = interface blocks, interface = junction nodes), which this handle owns
  int inner_form = 0;  // ns_inner_form
  int level2 = 0, level2_k = 0, level2_p = 0;
  double level2_tol = 0.0;
  const double* level2_omega = nullptr;
  ns_handle_s* sub = nullptr;
  ns::DBuf<double> recU, recT, recY;  // workspaces of the recursive A_Gamma solve (sized by columns)
  int64_t rec_cols = 0;
  ns::DBuf<double> subW, subC1, subC2;  // workspaces of the low-rank term when this handle is the level below
  int64_t sub_cols = 0;
  double tol_inner = 0.1, eig_rel = 1e-10, drop_rel = 1e-6;
  int max_inner = 500;

  // original matrix (for the true residual)
  ns::Csr Aorig;

  // index maps
  ns::DBuf<int32_t> iperm;  // padded interior row -> original node, -1 on padding
  ns::DBuf<int32_t> icomp;  // padded interior row -> compact interior index, -1 on padding
  ns::DBuf<int32_t> gperm;  // interface index -> original node
  ns::DBuf<int32_t> l2src;  // padded level-2 row -> interface index, -1 on padding
  ns::DBuf<int32_t> jsrc;   // padded junction row -> interface index, -1 on padding

  // level-1 couplings and blocks
  ns::Csr AIG;  // rows: padded interior rows; cols: interface index
  ns::Csr AGI;  // rows: interface index;      cols: padded interior rows
  ns::Csr AGG;  // rows: interface index;      cols: interface index
  ns::TileLevel L1;
  ns::LocalSchur LS;
  // level-2 (exact A_Gamma solve)
  ns::Csr AsJ;  // rows: padded level-2 rows;  cols: junction rows
  ns::Csr AJs;  // rows: padded junction rows; cols: padded level-2 rows
  ns::TileLevel L2, LJ;
  // level-2 rows coupled to junction nodes (the rows of A_sJ with entries), listed block by block: the second
  // level-2 solve of an A_Gamma solve only changes by A_s^{-1} restricted to these columns (see
  // op_gamma_solve); l2c_n = 0 turns that path off
  ns::DBuf<int32_t> l2c_rows, l2c_off, l2c_blk;  // row list, per-block offsets (nblk + 1), padded row -> block
  int64_t l2c_n = 0;
  int l2c_w = 0;                   // most listed rows of one block
  ns::DBuf<int32_t> l2c_rinf;      // per padded level-2 row: first listed row of its block, their count
  ns::DBuf<double> l2c_coef64;     // per padded level-2 row r: (A_b^{-1})(k, r) for the listed rows k of its block
  ns::DBuf<float> l2c_coef32;

  // low-rank term (FP64): Z n_G x k (ld = k; columns >= k_eff of a problem are zero), Sigma k per problem
  ns::DBuf<double> Z, Sigma;
  // adapted deflation: SZ = S Z, chol(E) (k x k lower, ld = k, per problem)
  ns::DBuf<double> SZ, Echol;
  // Nystrom basis U (n_G x k, before the A_Gamma^{-1} of Z = A_Gamma^{-1} U), kept for export
  ns::DBuf<double> U;
  // learned starting subspace: caller's n_G x k proposal, eigen-residual threshold, outcome
  const double* proposal = nullptr;
  double accept_tol = 0.2;
  int proposal_accepted = 0;
  double proposal_rho = 0.0;  // largest eigen-residual over the ceil(k/2) smallest Ritz values

  // error flags written by kernels and their host copy
  ns::DBuf<int> dflags;
  int hflags[16] = {};

  // workspaces (sized at setup)
  ns::DBuf<double> wsT64, wsB64, wsJ64, wsB64b, wsJ64b;  // interior rhs, level-2 rhs, junction rhs, outputs
  ns::DBuf<float> wsT32, wsB32, wsJ32, wsB32b, wsJ32b;
  ns::DBuf<double> wsC64;  // A_sJ y_J on the listed level-2 rows
  ns::DBuf<float> wsC32;
  ns::DBuf<double> red;    // reduction partials
  ns::DBuf<double> small;  // small dense scratch (per problem), described by sws
  ns::SmallWs sws;
  int64_t ws_cols = 0;     // column capacity of the workspaces
  int64_t wsT64_cols = 0, wsT32_cols = 0;  // column capacity of the interior workspaces

};

namespace ns {

using Handle = ns_handle_s;

enum SchurMode { SCHUR_AUTO = 0, SCHUR_TRIANGULAR = 1, SCHUR_LOCAL = 2 };

// Workspace management: make sure every per-apply buffer holds ncols columns.
void ensure_workspace(Handle& h, int64_t ncols);
void ensure_local_workspace(Handle& h, int64_t ncols);

// Operators on FP64 or FP32 data (blocks row-major, ld = leading dimension).
// op_schur uses the local Schur blocks when they were built, else the
// triangular solves with the interior factors (op_schur_tri).
template <class T>
void op_schur(Handle& h, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, bool w_only);
template <class T>
void op_schur_tri(Handle& h, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, bool w_only);
template <class T>
void op_schur_local(Handle& h, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, bool w_only);
template <class T>
void op_gamma_solve(Handle& h, const T* R, int64_t ldr, T* Out, int64_t ldo, int ncols);
template <class T>
void op_interior_solve(Handle& h, const T* X, T* Y, int ncols);  // X, Y: n_I x ncols interior order
// The preconditioner of a level-below handle g on its interface rows: z = M_g r (FP64, row-major, ncols
// columns; its workspaces grow on first use and are reused afterwards, so calls inside a captured graph
// allocate nothing once a call of the same width has run).
void sub_apply(Handle& g, const double* r, int64_t ldr, double* z, int64_t ldz, int ncols);

// Setup pieces.
// Problems of a batch laid side by side in one matrix: piece q owns nodes [node[q], node[q + 1]),
// subdomain labels [sub[q], sub[q + 1]) and level-2 labels [l2[q], l2[q + 1]); its junction nodes form
// junction block q.  pieces == nullptr: one problem, labels as given.
struct Pieces {
  std::vector<int64_t> node;
  std::vector<int> sub, l2;
};
void extract_dbbd(Handle& h, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                  const double* val, const int32_t* part, const Pieces* pieces = nullptr);
void assemble_junction(Handle& h);
// the second level-2 solve's coefficients from the explicit level-2 inverses (after they are made)
void make_l2_coefs(Handle& h);
// Symbolic pass (interface lists, layouts; waits for the device) and numeric pass (needs the interior factor).
void local_schur_plan(Handle& h);
void local_schur_form(Handle& h);
void local_schur_make_bf16(Handle& h);  // BF16 copy of the FP32 local Schur blocks

// Generic row gather / scatter and CSR products (row-major blocks).
template <class T>
void gather_rows(int64_t nrows, const int32_t* src, const T* R, int64_t ldr, T* Out, int64_t ldo, int ncols,
                 hipStream_t st);
template <class T, class U>
void scatter_rows(int64_t nrows, const int32_t* dst, const T* B, int64_t ldb, U* Out, int64_t ldo, int ncols,
                  hipStream_t st);
template <class T>
void csr_mult(const Csr& A, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, hipStream_t st);

}  // namespace ns
