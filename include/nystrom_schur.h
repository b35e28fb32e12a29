/*
 * nystrom_schur.h -- C ABI of the MI355X (gfx950) Nystrom-Schur solver library.
 *
 * Method: H. Al Daas, T. Rees, J. Scott, "Two-level Nystrom-Schur
 * Preconditioner for Sparse Symmetric Positive Definite Matrices",
 * arXiv:2101.12164.  The library takes a sparse SPD matrix A in CSR form and a
 * partition of its nodes into subdomains (interior nodes) and an interface,
 * i.e. the doubly bordered block diagonal (DBBD) form of eq. (perm_A).  It
 * builds the two-level preconditioner M_2 = A_Gamma^{-1} + Z Sigma Z^T of
 * eq. (left_prec_mat) with Algorithm alg:prec1 and solves A x = b through the
 * block LDL^T factorisation of eq. (A_LDLT): PCG on the Schur complement
 * system S_Gamma w = f of eq. (Sx=b), then back-substitution.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer (memory of the current HIP
 *    device, e.g. a torch CUDA tensor's data_ptr()), except the info structs
 *    and the options struct, which live in HOST memory.
 *  - Sizes are element counts.  Floating point data is IEEE double.
 *  - Dense blocks of vectors are ROW-MAJOR: element (i, c) of an m x ncols
 *    block is at [i * ncols + c].
 *  - "Interface order": the interface nodes (part[i] < 0) sorted by ascending
 *    original node index.  Vectors on the interface (length n_gamma) and the
 *    sketch Omega use this order.
 *  - "Interior order": interior nodes sorted by (subdomain id, original node
 *    index).
 *  - The caller owns every buffer it passes.  setup() copies what it needs, so
 *    A, part and omega may be freed after it returns.  The handle owns all
 *    internal device memory (factors, low-rank term, workspaces) and releases it
 *    in nystrom_schur_destroy().
 *  - Work is ordered on opt->stream (a hipStream_t; NULL = the null stream).
 *    Entry points synchronise that stream before returning status; they never
 *    synchronise the whole device.  A handle must not be used from two threads
 *    at once.
 *  - Errors are reported through the returned status only.  On failure of
 *    setup(), *out is set to NULL and nothing leaks.  nystrom_schur_last_error()
 *    returns a human-readable message for the last failure on a handle (or on
 *    the calling thread when the handle is NULL).
 */
#ifndef NYSTROM_SCHUR_H
#define NYSTROM_SCHUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_handle_s* ns_handle;

typedef enum {
  NS_OK = 0,
  NS_ERR_INVALID_ARG = 1,   /* bad sizes, NaN input, A not symmetric, partition not DBBD      */
  NS_ERR_NOT_SPD = 2,       /* a Cholesky pivot was <= 0: info->bad_block / bad_col say where */
  NS_ERR_OOM = 3,           /* device allocation failed                                       */
  NS_ERR_HIP = 4,           /* a HIP runtime call failed                                      */
  NS_ERR_NOT_CONVERGED = 5, /* maxit reached; the last iterate is still written               */
  NS_ERR_BREAKDOWN = 6      /* block CG lost every search direction / zero curvature          */
} ns_status;

/*
 * Precision of the inner block CG (the loose-tolerance solve of Algorithm alg:prec1 step 3):
 *   NS_FP64: everything FP64;
 *   NS_FP32: FP32 factors, local Schur blocks, interface inverses and block vectors, MFMA f32;
 *   NS_BF16: FP32 block vectors; the local Schur blocks and the interface-level inverses are applied as
 *            BF16 operands (round to nearest even) of 16x16x32 BF16 MFMA with FP32 accumulation (needs the
 *            local Schur operator and explicit interface inverses; otherwise those applications run in FP32).
 *            If the block CG breaks down on the BF16 Schur operator, it is run again with FP32 Schur operands
 *            (ns_setup_info.inner_bf16_schur says which ran).
 * The Nystrom core, the coarse deflation solve and the outer PCG (operator and residual) stay FP64.
 */
typedef enum { NS_FP64 = 0, NS_FP32 = 1, NS_BF16 = 2 } ns_prec;

typedef enum {
  NS_APPLY_M2 = 0,    /* z = A_Gamma^{-1} r + Z (Sigma o Z^T r)            eq. (left_prec_mat)  */
  NS_APPLY_ADEF2 = 1  /* z = t + Z E^{-1} (Z^T r - (S Z)^T t), t = A_G^{-1} r, E = Z^T S Z;
                         adapted deflation, eqs. (adapted_deflation_prec),
                         (deflation_comp_from_low_rank); PCG starts at w_0 = Z E^{-1} Z^T f */
} ns_apply_mode;

/*
 * Which matrix Nystrom approximates and how the low-rank basis Z is formed (the
 * variants of the preconditioner section; apply_mode then selects the additive
 * form A_Gamma^{-1} + Z Sigma Z^T or the adapted deflation built from Z):
 *   NS_VARIANT_M2: A_GammaI S_I^{-1} A_IGamma, Z = A_Gamma^{-1} U
 *                  (eqs. internal_term_lr_approximation_1, left_prec_mat);
 *   NS_VARIANT_M1: R_Gamma^{-T} A_GammaI S_I^{-1} A_IGamma R_Gamma^{-1}, Z = R_Gamma^{-1} U
 *                  (eqs. lr_approximation_S-1_A-I, prec1S, our_two_level_preconditioner), with
 *                  A_Gamma = R_Gamma^T R_Gamma the Cholesky factor of A_Gamma in the order of the
 *                  interface split (interface blocks in label order, then the junction nodes);
 *   NS_VARIANT_M3: S_I^{-1} on the interior space, Z = A_Gamma^{-1} A_GammaI U
 *                  (eqs. internal_term_lr_approximation_2, left_prec_mat2); the sketch omega is then
 *                  n_interior x (k+p) in interior order.  One problem per handle.
 */
typedef enum { NS_VARIANT_M2 = 0, NS_VARIANT_M1 = 1, NS_VARIANT_M3 = 2 } ns_variant;

/*
 * The outer iteration of pcg_solve:
 *   NS_OUTER_SCHUR: PCG on S_Gamma w = f (eq. Sx=b), then back-substitution;
 *   NS_OUTER_FULL:  PCG on A x = b preconditioned by the approximate block LDL^T factorisation with
 *                   S~^{-1} = M (eq. M_inv_A; spectrum Lambda(M S_Gamma) u {1}).  Needs
 *                   apply_mode NS_APPLY_M2 (a symmetric M).
 */
typedef enum { NS_OUTER_SCHUR = 0, NS_OUTER_FULL = 1 } ns_outer;

/*
 * How every solve with A_Gamma is made (the first level of M, the inner block CG's preconditioner, Z):
 *   NS_LEVEL2_EXACT:    exactly, through the interface split given by the labels (interface blocks, then
 *                       the junction Schur complement S_J = A_J - A_Js A_s^{-1} A_sJ, factorised);
 *   NS_LEVEL2_NYSTROM:  the recursive construction the conclusions name as future work: A_Gamma, taken as
 *                       a DBBD matrix of its own (interface blocks = its interior, junction nodes = its
 *                       interface), is preconditioned by its block LDL^T (eq. A_LDLT, the preconditioner
 *                       M^{-1} of the Schur-complement section) with S_J^{-1} replaced by the
 *                       Nystrom-Schur preconditioner M_J = A_J^{-1} + Z_J Sigma_J Z_J^T of S_J (Algorithm
 *                       alg:prec1 one level down, rank level2_k, sketch level2_omega, tolerance
 *                       level2_tol_inner, preconditioned by A_J^{-1}).  Only the interface blocks and A_J
 *                       are factorised.  One problem per handle; FP64 inner work; not with
 *                       NS_VARIANT_M1 (which needs an exact factor of A_Gamma) or a learned proposal;
 *                       the labels must give at least one interface block and one junction node.
 */
typedef enum { NS_LEVEL2_EXACT = 0, NS_LEVEL2_NYSTROM = 1 } ns_level2;

/*
 * The inner system of the construction:
 *   NS_INNER_SHIFTED: S_Gamma D = W G preconditioned by A_Gamma^{-1}, then B G = A_Gamma D (by eq. S-1 the
 *                     product of Algorithm alg:prec1 steps 2-4; n_gamma rows);
 *   NS_INNER_FORM_A:  the steps as printed: S_I X = A_IGamma G preconditioned by A_I^{-1} (eq. SI), then
 *                     B G = A_GammaI X (NS_VARIANT_M3: S_I X = G, B G = X); block vectors of n_interior rows.
 *                     One problem per handle; FP64 inner work; NS_VARIANT_M2 or NS_VARIANT_M3.
 */
typedef enum { NS_INNER_SHIFTED = 0, NS_INNER_FORM_A = 1 } ns_inner_form;

/*
 * Options of setup().  Zero-initialise and set what you need; a value of 0 in
 * tol_inner, eig_thresh_rel, orth_drop_rel or max_inner_iters selects the
 * default given in brackets.
 */
typedef struct {
  int32_t k;                 /* rank of the low-rank term, 0 <= k; k = 0 gives M = A_Gamma^{-1}  */
  int32_t p;                 /* oversampling, 0 <= p, k + p <= n_gamma                            */
  double tol_inner;          /* eps_SI: block-CG relative tolerance (max over columns) [0.1]     */
  double eig_thresh_rel;     /* Nystrom threshold on eig(C) relative to its largest [1e-10]      */
  double orth_drop_rel;      /* block-CG drop tolerance on singular values rel. to the largest
                                [1e-6 with FP64 inner work, 1e-5 with FP32]                      */
  int32_t max_inner_iters;   /* block-CG iteration cap [500]                                      */
  int32_t prec_inner;        /* ns_prec of the inner block CG (factors, block vectors) [NS_FP64] */
  int32_t apply_mode;        /* ns_apply_mode [NS_APPLY_M2]                                       */
  int32_t trsm_cols;         /* columns per workgroup in the batched triangular solves, 16/32/64;
                                0 = automatic                                                     */
  int32_t schur_mode;        /* how S_Gamma X is applied: 0 = automatic (local blocks), 1 =
                                A_Gamma X - A_GammaI (L L^T)^{-1} A_IGamma X with the interior
                                Cholesky factors (two triangular sweeps per apply), 2 = explicit
                                local Schur blocks S_j = (L_j^{-1} B_j)^T (L_j^{-1} B_j), one dense
                                block per subdomain over the interface nodes it touches, applied
                                as one batched GEMM                                              */
  const double* omega;       /* DEVICE, n_gamma x (k+p) row-major Gaussian sketch in interface
                                order (Algorithm alg:prec1 step 1); n_interior x (k+p) in
                                interior order for NS_VARIANT_M3.  Required when k > 0.           */
  const double* proposal;    /* DEVICE, optional n_gamma x k starting subspace (learned); NULL =
                                plain Nystrom.  Accepted subspaces run in NS_APPLY_ADEF2 mode.   */
  double accept_tol;         /* eigen-residual threshold for accepting `proposal` [0.2]          */
  void* stream;              /* hipStream_t for all work; NULL = null stream                      */
  int32_t pcg_graph_iters;   /* PCG iterations recorded per HIP graph and replayed between the
                                host's stopping checks: 0 = automatic (1 for one problem, 4 for
                                a batch), -1 = plain launches, m > 0 = m iterations per graph.
                                Results are the same in every mode.                              */
  int32_t variant;           /* ns_variant [NS_VARIANT_M2]                                        */
  int32_t power_iters;       /* q of eq. power: the sketch becomes B^q Omega, orthonormalised after
                                every product with B (each product is one inner block solve;
                                it_inner counts them all) [0]                                     */
  int32_t outer;             /* ns_outer [NS_OUTER_SCHUR]                                         */
  int32_t bcg_graph_iters;   /* block-CG iterations recorded per HIP graph and replayed between the
                                host's stopping checks (rounded up to an even count): 0 = automatic
                                (2), -1 = plain launches.  Results are the same in every mode.   */
  int32_t level2;            /* ns_level2 [NS_LEVEL2_EXACT]                                       */
  int32_t level2_k;          /* NS_LEVEL2_NYSTROM: rank k_2 of M_J, 0 <= k_2 (0: M_J = A_J^{-1})  */
  int32_t level2_p;          /* NS_LEVEL2_NYSTROM: oversampling p_2, k_2 + p_2 <= n_junction      */
  double level2_tol_inner;   /* NS_LEVEL2_NYSTROM: block-CG tolerance of level 2 [tol_inner]      */
  const double* level2_omega;/* NS_LEVEL2_NYSTROM: DEVICE, n_junction x (k_2 + p_2) row-major
                                sketch, junction nodes in interface order.  Required when k_2 > 0. */
  int32_t inner_form;        /* ns_inner_form [NS_INNER_SHIFTED]                                  */
} ns_options;

/* Outputs of setup(), HOST memory. Times are seconds measured with hipEvents. */
typedef struct {
  int64_t n, n_interior, n_gamma, n_junction;
  int32_t n_sub, n_level2_blocks;
  int32_t k_eff;             /* rank actually kept: min(k, rank of thresholded C)                 */
  int32_t it_inner;          /* block-CG iterations (it_SI)                                       */
  int32_t inner_converged;   /* 1 if eps_SI was reached                                           */
  int32_t proposal_accepted; /* 1 if the learned subspace was accepted                            */
  int32_t bad_block, bad_col;/* location of a non-positive pivot (NS_ERR_NOT_SPD), else -1        */
  double inner_relres;       /* final max column relative residual of block CG                    */
  double t_extract, t_factor, t_inner, t_nystrom, t_total;
  int32_t inner_bf16_schur;  /* NS_BF16: 1 if the Schur operator of the inner block CG ran on BF16 operands
                                to the end; 0 if the block CG broke down with them (P^T S P not positive
                                definite: S_Gamma's small eigenvalues below BF16 resolution) and was run again
                                with FP32 Schur operands (the preconditioner keeps its BF16 operands)      */
  int32_t level2_it_inner;   /* NS_LEVEL2_NYSTROM: block-CG iterations of level 2, else 0         */
  int32_t level2_k_eff;      /* NS_LEVEL2_NYSTROM: rank kept by M_J, else 0                       */
} ns_setup_info;

/* Outputs of pcg_solve(), HOST memory. */
typedef struct {
  int32_t it_pcg;            /* outer PCG iterations (applications of S_Gamma in the loop)        */
  int32_t converged;
  double relres_schur;       /* recurrence residual ||r|| / ||f|| at exit (NS_OUTER_FULL: ||r|| / ||b||
                                of the full-system recurrence)                                   */
  double relres_true;        /* ||b - A x|| / ||b|| of the returned x                             */
  double t_solve;            /* seconds, hipEvents                                                */
  double* res_hist;          /* optional HOST array receiving ||r_j|| / ||f||, j = 0..it_pcg      */
  int32_t res_hist_cap;      /* capacity of res_hist (0 = do not record)                          */
} ns_solve_info;

/*
 * Build the preconditioner (Algorithm alg:prec1) for the n x n SPD matrix A.
 *   row_ptr [n+1] int64, col_idx [nnz] int32, val [nnz] double: CSR of A with
 *     both triangles stored; A must be exactly symmetric.
 *   part [n] int32: partition labels.  part[i] >= 0: interior node of
 *     subdomain part[i] (ids 0..n_sub-1, every id used); part[i] == -1:
 *     interface node that is a junction of the interface split; part[i] <= -2:
 *     interface node of interface block (-2 - part[i]).  Interior nodes of
 *     distinct subdomains must not be coupled (eq. perm_A), and interface nodes
 *     of distinct interface blocks must not be coupled (the same form applied to
 *     A_Gamma, which the library uses for its exact A_Gamma solves).  Labelling
 *     every interface node -1 is always valid (A_Gamma is then factorised as
 *     one dense block).
 *   opt: options (HOST).  info: HOST, may be NULL.
 * Steps on the device: DBBD extraction; batched dense Cholesky of the interior
 * blocks and of the interface blocks; the junction Schur complement and its
 * Cholesky; block PCG on S_Gamma D = W Omega with W = A_Gamma - S_Gamma,
 * preconditioned by A_Gamma^{-1}, to tol_inner; Y = A_Gamma D (which equals
 * A_GammaI S_I^{-1} A_IGamma Omega by eq. S-1); the Nystrom core (QR of Y,
 * EVDs of C = Omega^T Y and T); Z = A_Gamma^{-1} U.
 * Errors: NS_ERR_INVALID_ARG (sizes, labels, asymmetry, DBBD violation, NaN),
 * NS_ERR_NOT_SPD (info->bad_block, bad_col: subdomain block -- or, for
 * bad_block <= -2, interface block -2-bad_block, or -1 for the junction
 * complement -- and its column), NS_ERR_OOM, NS_ERR_HIP, NS_ERR_BREAKDOWN.
 * A block CG that reaches max_inner_iters is not an error (info says so).
 */
ns_status nystrom_schur_setup(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                              const double* val, const int32_t* part, const ns_options* opt, ns_handle* out,
                              ns_setup_info* info);

/*
 * z = M r for ncols vectors (Algorithm alg:prec1 step 12, or the adapted
 * deflation form).  r_gamma, z_gamma: DEVICE, n_gamma x ncols row-major in
 * interface order; they must not overlap.  1 <= ncols <= 1024.
 */
ns_status nystrom_schur_apply(ns_handle h, const double* r_gamma, double* z_gamma, int32_t ncols);

/*
 * nystrom_schur_apply without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments and results as
 * nystrom_schur_apply; its scratch (Gram partials, coefficient blocks, small dense workspace) is a
 * file-scope device array of 4 MiB that every GPU the library runs on holds until the process ends, and the
 * handle's own operator workspaces (sized at setup for k + p columns) are used as they are.
 * NS_ERR_INVALID_ARG when the call would need more than the 4 MiB (its need grows with k x ncols x the
 * number of reduction chunks, about n_gamma / 128 up to 240 per problem) or more columns than the handle's
 * workspaces hold, and for handles built with NS_LEVEL2_NYSTROM.  Calls on one GPU share the array: calls that overlap on one GPU (two streams, two
 * threads) race and must not be made.
 */
ns_status nystrom_schur_apply_noalloc(ns_handle h, const double* r_gamma, double* z_gamma, int32_t ncols);

/*
 * Solve A x = b (eq. A_LDLT): f = b_Gamma - A_GammaI A_I^{-1} b_I; PCG with M on
 * S_Gamma w = f until ||r_j|| / ||f|| <= rtol (eq. Sx=b); x_I = A_I^{-1}(b_I -
 * A_IGamma w), x_Gamma = w.  b, x: DEVICE, length n, ORIGINAL node order; they
 * must not overlap.  Returns NS_ERR_NOT_CONVERGED (x still written) when maxit
 * iterations do not reach rtol; NS_ERR_INVALID_ARG for NaN/Inf in b.
 */
ns_status nystrom_schur_pcg_solve(ns_handle h, const double* b, double* x, double rtol, int32_t maxit,
                                  ns_solve_info* info);

/*
 * Batched setup: nprob independent problems set up together, as the diagonal
 * blocks of one block-diagonal matrix (Algorithm alg:prec1 for each of them).
 * Every launch of the extraction, the factorisations, the Schur operator and
 * the A_Gamma solves covers the subdomain and interface blocks of all problems;
 * block CG, the Nystrom core and PCG keep separate scalars, Gram matrices,
 * ranks and stopping tests per problem, and every reduction is taken per
 * problem over a fixed number of row chunks that depends only on that
 * problem's size, so each problem's results equal those of the problem set up
 * alone with nystrom_schur_setup (same options).
 *   n[q], nnz[q]: HOST arrays; row_ptr[q], col_idx[q], val[q], part[q]: HOST
 *     arrays of DEVICE pointers, each problem as in nystrom_schur_setup (labels
 *     local to the problem); omega[q]: DEVICE n_gamma(q) x (k+p) sketch of
 *     problem q (HOST array of pointers; may be NULL when k == 0).
 *   opt: shared options (opt->omega is ignored).  info: HOST array of nprob
 *     entries (times are those of the whole batch), may be NULL.
 * The handle serves nystrom_schur_pcg_solve_batched and nystrom_schur_apply
 * (on the problems' interface vectors stacked in problem order).
 * Errors as nystrom_schur_setup; a failure in any problem fails the batch; opt->level2 must be
 * NS_LEVEL2_EXACT.
 */
ns_status nystrom_schur_setup_batched(int32_t nprob, const int64_t* n, const int64_t* nnz,
                                      const int64_t* const* row_ptr, const int32_t* const* col_idx,
                                      const double* const* val, const int32_t* const* part,
                                      const double* const* omega, const ns_options* opt, ns_handle* out,
                                      ns_setup_info* info);

/*
 * Solve A_q x_q = b_q for every problem of a batched handle (eqs. A_LDLT and
 * Sx=b): one PCG over all problems with per-problem scalars; a problem that
 * meets rtol is frozen (its iterate no longer changes) while the others go on,
 * so each problem stops at the same iteration as alone.  b[q], x[q]: HOST
 * arrays of DEVICE pointers (length n[q], the problem's own node order).
 * info: HOST array of nprob entries (t_solve: the whole batch), may be NULL.
 * NS_ERR_NOT_CONVERGED when some problem does not reach rtol (all x written).
 */
ns_status nystrom_schur_pcg_solve_batched(ns_handle h, const double* const* b, double* const* x, double rtol,
                                          int32_t maxit, ns_solve_info* info);

/* Operator access (the building blocks of the two calls above), for testing and
 * composition.  All blocks are DEVICE, row-major, ncols columns (1..1024).    */

/* Y = S_Gamma X = A_Gamma X - A_GammaI A_I^{-1} A_IGamma X (eq. schur_complement);
 * X, Y: n_gamma x ncols, interface order.  prec selects the FP64 operator or
 * the FP32 one used inside the inner block CG (inputs/outputs stay double). */
ns_status nystrom_schur_schur_apply(ns_handle h, const double* X, double* Y, int32_t ncols, int32_t prec);

/* Y = A_Gamma^{-1} X (the first-level preconditioner of eq. S1); interface order.  With NS_LEVEL2_NYSTROM,
 * the recursive approximation of A_Gamma^{-1} that the handle uses (FP64 only). */
ns_status nystrom_schur_interface_solve(ns_handle h, const double* X, double* Y, int32_t ncols, int32_t prec);

/* Y = A_I^{-1} X; X, Y: n_interior x ncols in interior order. */
ns_status nystrom_schur_interior_solve(ns_handle h, const double* X, double* Y, int32_t ncols, int32_t prec);

/* Copy the dense lower Cholesky factor of interior block `block` (FP64) into
 * L (DEVICE, nb x nb column-major, nb = size of the block; upper part zeroed). */
ns_status nystrom_schur_export_factor(ns_handle h, int32_t block, double* L);

/* Sizes: out[0..7] = n, n_interior, n_gamma, n_sub, n_junction,
 * n_level2_blocks, k_eff, number of problems (totals over the problems of a
 * batched handle; k_eff is then the largest).  HOST array.                  */
ns_status nystrom_schur_get_sizes(ns_handle h, int64_t* out);

/* Copy the low-rank term: Z (DEVICE, n_gamma x k_eff row-major, interface
 * order) and Sigma (DEVICE, k_eff).  Either pointer may be NULL.
 * NS_ERR_INVALID_ARG for a batched handle. */
ns_status nystrom_schur_get_lowrank(ns_handle h, double* Z, double* Sigma);

/* Copy the Nystrom basis U (the orthonormal n_gamma x k_eff factor of Algorithm
 * alg:nystrom before Z = A_Gamma^{-1} U; DEVICE, row-major, interface order) and
 * the eigen-residual of the judged proposal (HOST, may be NULL; 0 when no
 * proposal was given).  NS_ERR_INVALID_ARG for a batched handle, or for U when
 * an accepted proposal replaced the Nystrom step. */
ns_status nystrom_schur_get_basis(ns_handle h, double* U, double* rho);

/* ---------------------------------------------------------------------------
 * Learned starting subspace.  The adapted deflation (eqs.
 * adapted_deflation_prec, deflation_comp_from_low_rank) works with any
 * full-rank basis; a small network over interface nodes proposes one
 * (ns_options.proposal), setup judges it by Rayleigh-Ritz on the pencil
 * (S_Gamma, A_Gamma) and uses it, or falls back to plain Nystrom.
 * ------------------------------------------------------------------------- */

/* Interface-node features, 16 per node, rows in interface order (ascending node
 * index among part < 0): coordinates (coords: DEVICE n x 3 or NULL -> 0), log A_ii,
 * mean/min/max log|A_ij| off the diagonal, log of the summed |A_ij| to interior
 * and to interface neighbours, junction flag, distinct neighbouring subdomains/4,
 * log A_ii averaged over the interface graph 1, 2 and 4 times, interface
 * degree/8, 1.  X: DEVICE float, at least n_gamma x 16; *n_gamma (HOST) receives
 * the row count.  CSR as in nystrom_schur_setup (not validated here).
 * Synchronises `stream`. */
ns_status nystrom_schur_features(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                                 const double* val, const int32_t* part, const double* coords, float* X,
                                 int64_t* n_gamma, void* stream);

/* The network: d_in -> hidden -> hidden -> d_out, ReLU hidden layers, linear
 * output; BF16 operands on 16x16x32 MFMA with FP32 accumulation; FP32 master
 * weights.  params: HOST float array, in order W1 (d_in x hidden, row-major in x
 * out), b1, W2 (hidden x hidden), b2, W3 (hidden x d_out), b3; the library copies
 * it.  Every call is ordered on its stream and after the network's previous call
 * (whatever its stream); create, get_params and destroy use the network's own
 * stream and synchronise only that (no device-wide synchronisation). */
typedef struct ns_mlp_s* ns_mlp;
ns_status nystrom_schur_mlp_create(int32_t d_in, int32_t hidden, int32_t d_out, const float* params, ns_mlp* out);
/* HOST copies of the parameters and of the last gradient (either may be NULL). */
ns_status nystrom_schur_mlp_get_params(ns_mlp m, float* params, float* grad);
/* Z0 (DEVICE double, n x d_out) = network(X) for X (DEVICE float, n x d_in). */
ns_status nystrom_schur_mlp_forward(ns_mlp m, const float* X, int64_t n, double* Z0, void* stream);
/* Forward, the subspace loss L = 1 - tr(G^{-1} Z0^T U U^T Z0) / k (G = Z0^T Z0,
 * U: DEVICE n x d_out with orthonormal columns) into *loss (HOST), and its
 * gradient with respect to the parameters (kept in the network for the next
 * adam_step).  NS_ERR_BREAKDOWN when Z0 is rank deficient. */
ns_status nystrom_schur_mlp_loss_grad(ns_mlp m, const float* X, const double* U, int64_t n, double* loss,
                                      void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the last gradient. */
ns_status nystrom_schur_mlp_adam_step(ns_mlp m, double lr, void* stream);
void nystrom_schur_mlp_destroy(ns_mlp m);
const char* nystrom_schur_mlp_last_error(ns_mlp m);

/* Opt-in kernel timing for performance measurement (callers: benchmarks).
 * enable != 0 brackets every launch of the main kernel families with HIP
 * events on the launching stream (adds a few microseconds per launch);
 * calling it also resets the accumulated totals.  Process-wide.  While a
 * timed family runs inside the block-CG or PCG iterations, those iterations
 * use plain launches instead of replayed graphs (launches recorded into a
 * graph cannot be timed one by one); results are the same. */
void nystrom_schur_kernel_timing(int32_t enable);

/* As nystrom_schur_kernel_timing, for the families whose bit is set in mask
 * (bit f = the f-th family in the list below, from 0); mask 0 turns timing
 * off.  Timing fewer families perturbs the timed run less. */
void nystrom_schur_kernel_timing_families(uint32_t mask);

/* Accumulated device time (milliseconds, from the events), launch count and
 * algorithmic work (bytes the method must move, flops it must compute: the
 * unpadded dense factor once per sweep, no re-reads) of one kernel family
 * since timing was enabled.  family: "chol_update", "chol_panel",
 * "trsm_interior_f64", "trsm_interior_f32", "trsm_interface_f64",
 * "trsm_interface_f32" (forward and backward sweeps), "schur_epi", "spmm",
 * "local_schur_form", "local_schur_apply_f64", "local_schur_apply_f32",
 * "interface_inverse_f64", "interface_inverse_f32", "mlp_forward_bf16",
 * "mlp_backward_f32", "local_schur_apply_bf16", "interface_inverse_bf16", "gram" (Gram products
 * of block vectors, both wider than 16 columns), "block_update" (block updates X M of more than 16
 * columns), "small_dense" (the one-workgroup s x s kernels), "gram_narrow" and
 * "block_update_narrow" (the same with at most 16 columns on one side, e.g. Z^T r and Z c),
 * "local_schur_apply_narrow_f64" and "interface_inverse_narrow_f64" (the FP64 applies to at most 16
 * columns, e.g. the outer iteration's S_Gamma p and A_Gamma^{-1} r; the families without "narrow" then
 * hold the wider applies).
 * Waits for the recorded events.  All outputs are HOST pointers (may be NULL).
 * NS_ERR_INVALID_ARG for an unknown family. */
ns_status nystrom_schur_kernel_stats(const char* family, double* total_ms, int64_t* launches, double* bytes,
                                     double* flops);

/* Automatic settings.  The library takes the automatic choices below from a table written by the project's
 * autotuner (paper_2101_12164_amd/autotune.py: it times the candidates on the device and keeps the fastest),
 * shipped beside the shared library as tuning_<arch>.tsv and keyed by architecture, kernel, precision and
 * size class; explicit ns_options values take precedence.  get_tuning reports, for a handle, the values
 * that apply to its sizes: out[0] columns per workgroup of the multi-column triangular sweeps (k + p
 * columns), out[1] PCG iterations per graph, out[2] block-CG iterations per graph, out[3] output columns per
 * workgroup of the local Schur products for 65-80 columns (64 or 80).  HOST array of 4.  tuning_info returns
 * the number of table entries loaded for the current device and copies the table's path into `path` (HOST,
 * capacity `cap`, may be NULL). */
ns_status nystrom_schur_get_tuning(ns_handle h, int32_t* out);
int32_t nystrom_schur_tuning_info(char* path, int32_t cap);
/* Process-wide value of one automatic setting ("trsm_cols", "pcg_graph_iters", "bcg_graph_iters",
 * "ls_gemm_cols") that takes precedence over the table until removed (value 0); the autotuner times its
 * candidates with it.  Returns 0, or -1 for a NULL name. */
int32_t nystrom_schur_tuning_override(const char* kernel, int32_t value);

/* Release everything the handle owns.  Idempotent on NULL. */
void nystrom_schur_destroy(ns_handle h);

/* Message of the last failure on h (thread-local when h == NULL).  Never NULL. */
const char* nystrom_schur_last_error(ns_handle h);

#ifdef __cplusplus
}
#endif

#endif /* NYSTROM_SCHUR_H */
