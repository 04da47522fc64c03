/*
 * fastalign.h -- C ABI of the MI355X (gfx950) FastAlign hot path.
 *
 * The library computes the optimal-transport network alignment of Algorithm 1
 * (§3.1) of the FastAlign paper: Phase 1 precomputes the S-independent costs,
 * Phase 2 rebuilds the S-dependent costs from the sparse adjacencies and the
 * dense plan, Phase 3 runs log-domain Sinkhorn (Eq. (3)) and recovers the plan
 * (Eq. (4)).
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers unless the comment says "host".
 *     The caller allocates and frees every buffer; the library never allocates
 *     device memory.  Workspaces are caller-provided byte buffers whose size is
 *     returned by the matching *_workspace_size() query (256-byte alignment).
 *   - Dense n1 x n2 matrices are row-major with leading dimension n2 and 64-bit
 *     offsets.  Row index i runs over the nodes of G1, column index j over G2.
 *   - `stream` is a hipStream_t (NULL selects the null stream).  Device entry
 *     points enqueue work on it and return without waiting, except where a
 *     comment says they synchronise.
 *   - Every entry point returns an fa_status; nothing throws across the ABI.
 *     On a non-OK status fa_last_error() returns a thread-local message.  Inputs
 *     are validated before any work is enqueued; on FA_ERR_* no output has
 *     been written unless stated otherwise.
 *   - Dual vectors follow Eq. (3): a (length n2) pairs with the column marginal
 *     nu = 1/n2, b (length n1) with the row marginal mu = 1/n1.  Duals are FP64.
 */
#ifndef FASTALIGN_H
#define FASTALIGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FA_OK = 0,
  FA_WARN_NOT_CONVERGED = 1, /* finished, but the inner tolerance was not met */
  FA_ERR_ARG = -1,           /* invalid scalar argument, null pointer, bad anchors */
  FA_ERR_SHAPE = -2,         /* inconsistent sizes */
  FA_ERR_CSR = -3,           /* malformed CSR (host-side checks) */
  FA_ERR_WORKSPACE = -4,     /* workspace missing or smaller than required */
  FA_ERR_NUMERIC = -6,       /* non-finite value where a finite one is required */
  FA_ERR_HIP = -7,           /* a HIP runtime call failed */
  FA_ERR_DEVICE = -8,        /* the current device is not a gfx950 GPU */
  FA_ERR_SYNC = -9           /* a bounded wait between co-resident workgroups of the
                                single-pass Sinkhorn iteration gave up (outputs undefined) */
} fa_status;

typedef enum { FA_F32 = 0, FA_BF16 = 1, FA_F64 = 2 } fa_dtype;

/* Pattern-only CSR of an undirected graph (§2: adjacency A with 0/1 entries).
 * rowptr: int64[n+1], colidx: int32[nnz], device.  Rows must be sorted and
 * duplicate-free without self-loops, as fa_csr_build produces them. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int64_t *rowptr;
  const int32_t *colidx;
} fa_csr;

/* Hyper-parameters of Algorithm 1 (the paper gives no values; see
 * fa_default_params for this library's defaults). */
typedef struct {
  double eps;         /* Sinkhorn entropic regulariser epsilon (Eq. (1), Eq. (3)) */
  double alpha;       /* positional vs attribute weight in C_node */
  double beta;        /* restart weight of the positional encoding */
  double lambda_e;    /* weight of C_edge (Eq. (2)) */
  double lambda_n;    /* weight of C_nbr (Eq. (2)) */
  double lambda_a;    /* weight of C_anc (Eq. (2)) */
  double lambda_p;    /* weight of the proximal term -lambda_p * log S */
  double eps_anchor;  /* epsilon inside C_anc = -log(eps_anchor + OneHot(L)) */
  double delta_nbr;   /* C_nbr = -log(Abar1^T S Abar2 + delta_nbr) */
  double tol;         /* inner stop: L1 column-marginal error <= tol (0: never) */
  int32_t k_r;        /* positional-encoding iterations */
  int32_t k_node;     /* node-cost propagation iterations */
  int32_t outer_iters;/* outer (proximal) iterations */
  int32_t inner_iters;/* cap on Sinkhorn iterations per outer iteration */
  int32_t check_every;/* evaluate the stop rule every this many iterations (>=1) */
  int32_t plan_dtype; /* FA_F32 or FA_BF16: storage of S (with FA_BF16 the C1 S half of the
                         SpMM intermediate is BF16 too; A1^T S, whose log is taken, stays FP32) */
  int32_t feat_dtype; /* FA_F32 or FA_BF16: X-hat and R operands of fa_feature_sim */
  int32_t feat_l2norm;/* 1: row-L2-normalise the attributes before the product */
  int32_t warm_start; /* 0: cold duals; 1: learned row duals for the first solve */
  int32_t chunk_rows; /* rows per Phase-2 chunk (0: automatic) */
  int32_t profile;    /* 1: time every launch with HIP events (fa_stats.kernel_ms) */
  int32_t dual_start; /* start of the inner solves after the first (fa_dual_start):
                         FA_START_ZERO a = b = 0; FA_START_CARRY the previous solve's final
                         duals; FA_START_MEAN the mean of all earlier solves' final duals.
                         Each solve's fixed point is the same from any start (its duals are
                         unique up to a constant shift); only iterates before convergence
                         differ. */
  int32_t transpose_cost; /* 1: fa_align keeps C^T beside C (one more n1*n2 FP32 buffer in
                         the workspace) and runs the a-update on its rows; 0: column
                         strips of C (less memory, a slower a-update) */
  int32_t plan_in_ct; /* 1 (needs transpose_cost = 1): fa_align keeps the working plan in the
                         C^T buffer, which is free from the plan pass until the cost rebuild
                         has read the plan; the rebuild then writes C only and one transpose
                         pass regenerates C^T.  No n1*n2 plan buffer is needed (S_out may be
                         NULL; the plan is handed out as top-k lists), results are identical
                         to plan_in_ct = 0, one extra pass over C per outer iteration. */
  int32_t warm_fallback; /* 1 (with warm_start and tol > 0): when the solve started from the
                         learned duals misses tol, the same solve is rerun from a = b = 0 and
                         the run keeps whichever ends with the smaller marginal error
                         (fa_stats.fell_back = 2 when the cold solve is kept) */
  int32_t warm_probe; /* with warm_fallback and tol > 0: iterations granted to the solve from
                         the learned duals before the cold rerun takes over (0: inner_iters).
                         A learned start either
                         converges within a few dozen iterations or decays at the cold rate,
                         so a short probe bounds what a miss costs. */
  int32_t sink_fused; /* 1: inner solves use the single-pass iteration of fa_sinkhorn_fused
                         (one read of C per iteration instead of two; C^T is then needed
                         only by plan_in_ct) when the shape and the device allow it, and
                         the two-pass iteration otherwise; 0: always two passes */
} fa_params;

/* Starts of the inner solves after the first (fa_params.dual_start). */
typedef enum { FA_START_ZERO = 0, FA_START_CARRY = 1, FA_START_MEAN = 2 } fa_dual_start;

/* Run statistics returned by fa_align (host struct). */
typedef struct {
  int32_t outer_done;
  int32_t inner_total;      /* Sinkhorn iterations summed over outer iterations (both solves
                               of the first one when the cold rerun happened) */
  int32_t fell_back;        /* learned start: 0 kept, 1 non-finite prediction (the solve ran
                               cold), 2 its solve missed tol and the cold rerun ended closer */
  int32_t converged_all;    /* 1 if every inner solve met tol */
  double marg_err;          /* L1 column-marginal error of the last inner solve */
  int32_t warm_iters;       /* iterations of the solve from the learned start (-1: none) */
  int32_t cold_iters;       /* iterations of the cold rerun of that solve (-1: none) */
  double warm_err;          /* their final marginal errors (NaN: not run) */
  double cold_err;
  double phase_ms[4];       /* Phase 1, cost rebuild, Sinkhorn, plan (device time) */
  int32_t inner_iters[64];  /* per outer iteration (first 64) */
  double inner_err[64];
  /* with params.profile: summed device time and launch count per kernel class:
   * [0] column LSE partials, [1] column merge, [2] row LSE, [3] cost stage 1
   * (left SpMM), [4] cost stage 2 (right SpMM + fused assembly), [5] plan,
   * [6] node similarity (MFMA GEMM), [7] column pass over C^T, [8] transpose of C
   * (plan_in_ct), [9] top-k plan, [10] single-pass iteration (its merge counts
   * under [1]) */
  double kernel_ms[11];
  int32_t kernel_calls[11];
} fa_stats;

/* Thread-local message describing the last non-OK status. */
const char *fa_last_error(void);

/* Fill *p with this library's defaults: eps 0.05, alpha 0.5, beta 0.15,
 * lambda_e = lambda_n = lambda_a = 1, lambda_p = eps_anchor = eps,
 * delta_nbr 1e-30, tol 0, k_r 10, k_node 1, 10 outer x 50 inner iterations,
 * check_every 1, FP32 plan and features, feat_l2norm 1, cold start, zero starts
 * for later solves, transpose_cost 0, plan_in_ct 0, warm_fallback 1, warm_probe 0,
 * sink_fused 1. */
void fa_default_params(fa_params *p);

/* 0 if the current HIP device is a gfx950 GPU, else FA_ERR_DEVICE. */
int fa_device_check(void);

/* ----------------------------------------------------------------------- */
/* Host-side graph input (§2; reading: undirected, symmetrised, self-loops   */
/* dropped, duplicates merged, columns sorted).                              */
/* ----------------------------------------------------------------------- */

/* Build the CSR of an undirected graph from an edge list.
 *   edges_uv   host int64[m*2], pairs (u, v) with 0 <= u, v < n
 *   rowptr_out host int64[n+1]
 *   colidx_out host int32[cap]
 *   nnz_out    host: number of stored entries (also set when cap is too small)
 * Returns FA_ERR_ARG for an endpoint out of range or n < 0, m < 0, and
 * FA_ERR_SHAPE if cap < nnz (rowptr_out is then valid, colidx_out is not). */
int fa_csr_build(int32_t n, int64_t m, const int64_t *edges_uv, int64_t *rowptr_out,
                 int32_t *colidx_out, int64_t cap, int64_t *nnz_out);

/* ----------------------------------------------------------------------- */
/* Phase 1 building blocks (Algorithm 1, Phase 1)                            */
/* ----------------------------------------------------------------------- */

/* Row normalisation Abar = D^-1 A: inv_deg[i] = 1/deg_i, 0 for isolated nodes.
 *   inv_deg float[A->n] (out). */
int fa_row_normalize(const fa_csr *A, float *inv_deg, void *stream);

/* Positional encoding: R^(0) one-hot at the anchor nodes (column l at node
 * anchor_nodes[l]); then k steps of R <- (1-beta) Abar R + beta R^(0).
 *   anchor_nodes int32[nL], distinct, in [0, A->n)
 *   R, R_tmp     float[A->n * nL] row-major (out, scratch)
 * Anchor validity is the caller's responsibility here (fa_align checks it). */
int fa_positional(const fa_csr *A, const float *inv_deg, const int32_t *anchor_nodes,
                  int32_t nL, double beta, int32_t k, float *R, float *R_tmp, void *stream);

/* Sampled dense-dense product on the adjacency pattern (§3.3, SDDMM):
 *   out[e] = <R[row(e),:], R[col(e),:]> * inv_deg[row(e)]   if scale_by_col == 0
 *   out[e] = <R[row(e),:], R[col(e),:]> * inv_deg[col(e)]   if scale_by_col == 1
 * i.e. the stored values of C1 = (R1 R1^T) o Abar1 (scale_by_col = 0) and of
 * C2 = (R2 R2^T) o Abar2^T (scale_by_col = 1) in the CSR order of A.
 *   R float[A->n * nL], out float[A->nnz]. */
int fa_sddmm(const fa_csr *A, const float *inv_deg, const float *R, int32_t nL,
             int32_t scale_by_col, float *out, void *stream);

/* Row-wise L2 normalisation (zero rows stay zero), written as out_dtype.
 *   X float[n*d]; out float or bf16 [n*d]. */
int fa_l2_normalize(const float *X, int32_t n, int32_t d, void *out, int32_t out_dtype,
                    void *stream);

/* Node similarity (Algorithm 1, Phase 1):
 *   C_node = alpha * exp(-R1 R2^T) + (1 - alpha) * exp(-X1 X2^T)
 * as one fused matrix-core product with an exponential epilogue.
 *   X1 [n1*d], X2 [n2*d]   (dtype x_dtype: FA_F32 or FA_BF16; d may be 0)
 *   R1 [n1*nL], R2 [n2*nL] (dtype r_dtype; nL may be 0)
 *   C_node float[n1*n2] (out).  FP32 operands use FP32 MFMA, BF16 operands
 *   BF16 MFMA; accumulation is FP32 in both.  BF16 operands whose d and nL are
 *   multiples of 8 and whose four pointers are 16-byte aligned take the faster
 *   direct-to-LDS kernel (the exponentials there are the hardware exp2 of
 *   -x log2(e), relative error at most |x| 2^-24 beyond the exp2's own ulp);
 *   other shapes run a register-staged kernel with the library expf. */
int fa_feature_sim(const void *X1, const void *X2, int32_t n1, int32_t n2, int32_t d,
                   int32_t x_dtype, const void *R1, const void *R2, int32_t nL,
                   int32_t r_dtype, double alpha, float *C_node, void *stream);

/* Workspace for fa_propagate and fa_cost (the block-transposed FP32 SpMM
 * intermediates of one row chunk, 2 * ceil(chunk/64)*64 * n2 * 4 bytes).
 * chunk_rows 0 means all n1 rows.  plan_dtype is accepted for symmetry with
 * fa_params and does not change the size. */
size_t fa_cost_workspace_size(int32_t n1, int32_t n2, int32_t plan_dtype, int32_t chunk_rows);

/* Node-cost propagation, k times C <- Abar1 C Abar2^T (two SpMMs per step).
 *   C     float[n1*n2] in/out;  C_tmp float[n1*n2] scratch
 *   ws    >= fa_cost_workspace_size(n1, n2, FA_F32, chunk_rows) bytes. */
int fa_propagate(const fa_csr *A1, const float *inv_deg1, const fa_csr *A2,
                 const float *inv_deg2, float *C, float *C_tmp, int32_t k, int32_t chunk_rows,
                 void *ws, size_t ws_bytes, void *stream);

/* Phase 2 cost rebuild (Algorithm 1, Phase 2; Eq. (2); §3.5 fusion):
 *   C_new = C_node + lambda_e * C1 S C2^T - lambda_n * log(Abar1^T S Abar2 + delta)
 *           + lambda_a * C_anc - lambda_p * log S,
 *   log S_ij = (a_j + b_i - C_prev_ij) / eps   (the plan of the previous duals).
 *   w1  float[A1->nnz]: C1 values in A1's CSR order (fa_sddmm, scale_by_col 0)
 *   w2  float[A2->nnz]: C2 values in A2's CSR order (fa_sddmm, scale_by_col 1)
 *   S   [n1*n2] of dtype s_dtype (FA_F32/FA_BF16): the current plan
 *   partner int32[n1]: anchor partner in G2 of node i, or -1
 *   a double[n2], b double[n1]: duals that produced S from C_prev
 *   C_inout float[n1*n2]: C_prev in, C_new out (updated in place, row chunk by
 *   row chunk).
 *   Ct_out float[n2*n1] or NULL: if given, also receives C_new^T (row-major n2 x n1,
 *   bit-identical to C_new), for fa_sinkhorn's transposed column pass.
 *   ws >= fa_cost_workspace_size(n1, n2, s_dtype, p->chunk_rows). */
int fa_cost(const fa_csr *A1, const fa_csr *A2, const float *w1, const float *w2,
            const float *inv_deg1, const float *inv_deg2, const void *S, int32_t s_dtype,
            const float *C_node, const int32_t *partner, const double *a, const double *b,
            const fa_params *p, float *C_inout, float *Ct_out, void *ws, size_t ws_bytes,
            void *stream);

/* ----------------------------------------------------------------------- */
/* Phase 3 (Eq. (3), Eq. (4))                                                */
/* ----------------------------------------------------------------------- */

size_t fa_sinkhorn_workspace_size(int32_t n1, int32_t n2);

/* Log-domain Sinkhorn on a fixed cost C (Eq. (3)): each iteration updates a
 * (column log-sum-exp over i) and then b (row log-sum-exp over j).  The L1
 * column-marginal error sum_j |sum_i S_ij - 1/n2| of the state after an
 * iteration is evaluated (in FP64) by the next column pass; every
 * check_every iterations the loop stops when tol > 0 and err <= tol.
 *   a double[n2], b double[n1]: starting duals in, final duals out
 *   dev_iters int32[1], dev_err double[1] (device, out): iterations done and the
 *   final marginal error.  The loop never waits for the host.
 * Ct float[n2*n1] or NULL: C^T row-major.  If given, the a-update streams it
 *   row by row (the pattern of the b-update) instead of column strips of C; the
 *   results are the same up to summation order.
 * If host_iters/host_err are non-NULL the call synchronises the stream and
 * copies the two results to them. */
int fa_sinkhorn(const float *C, const float *Ct, int32_t n1, int32_t n2, double eps, double *a, double *b,
                int32_t max_iter, double tol, int32_t check_every, int32_t *dev_iters,
                double *dev_err, int32_t *host_iters, double *host_err, void *ws,
                size_t ws_bytes, void *stream);

/* fa_sinkhorn for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (bit for bit) as fa_sinkhorn, minus the
 * workspace and the host copies: its scratch (the candidate a, the per-workgroup
 * error partials, the loop's control word and, without Ct, the per-column
 * partials) lives in a static device array of FA_SINKHORN_NOALLOC_SCRATCH bytes,
 * one per GPU, held until the process ends.  The call allocates nothing
 * (no hipMalloc, no library allocation) and never synchronises; read dev_iters /
 * dev_err after the stream has passed it.  Sizes whose scratch exceeds the array
 * (fa_sinkhorn_noalloc_need(n1, n2, Ct != NULL) > FA_SINKHORN_NOALLOC_SCRATCH) are
 * refused with FA_ERR_SHAPE: with Ct that is n2 beyond ~1.8 million, without Ct
 * the per-column partials (16 * n2 bytes per row split) limit it to small n2.
 * All calls on one GPU share its array: calls that overlap in time on one GPU
 * (other streams or threads) race and must be serialised by the caller.  The
 * first call on a device looks the array's device address up (once per device). */
#define FA_SINKHORN_NOALLOC_SCRATCH (16u << 20)
size_t fa_sinkhorn_noalloc_need(int32_t n1, int32_t n2, int32_t transposed);
int fa_sinkhorn_noalloc(const float *C, const float *Ct, int32_t n1, int32_t n2, double eps, double *a,
                        double *b, int32_t max_iter, double tol, int32_t check_every, int32_t *dev_iters,
                        double *dev_err, void *stream);

/* Single-pass form of fa_sinkhorn (Eq. (3), the same iteration): C is read once
 * per iteration instead of twice, and no C^T is needed.  Iterations 0 and 1 run
 * as in fa_sinkhorn without C^T; from iteration 2 on one pass over C does the
 * b-update of the iteration and the column sums of the a-update after it.  Each
 * row is split over gc co-resident workgroups (column slices of up to 4,096
 * columns held in registers) that exchange their partial row sums before
 * adding the row's updated plan entries to their column sums; the exponent
 * (a_j + b_i - C_ij)/eps is formed in FP64 as in fa_sinkhorn and needs no running
 * maximum (after an a-update no plan entry exceeds nu_j, and after a b-update
 * no row sum of the next plan falls below mu_i * min_j nu_j).  Results equal
 * fa_sinkhorn's up to summation order (same iteration count when both stop on
 * the same check).  Arguments as fa_sinkhorn minus Ct; ws >=
 * fa_sinkhorn_fused_workspace_size(n1, n2) bytes.  Needs n2 % 4 == 0, at most 64
 * partners per row (n2 <= 262,144), a device that co-schedules the grid, and a
 * grid that fills at least 5/8 of the co-resident workgroup slots (a row's partners
 * share an XCD, so 33..39 partners leave most of them idle); otherwise every
 * iteration takes the two-pass form (fa_sinkhorn_fused_grid says which).  The partners' waits are bounded (fa_set_sync_spin_limit):
 * a wait that gives up stops the solve, dev_iters becomes -1 and dev_err NaN, and
 * with host_iters/host_err the call returns FA_ERR_SYNC. */
size_t fa_sinkhorn_fused_workspace_size(int32_t n1, int32_t n2);
int fa_sinkhorn_fused(const float *C, int32_t n1, int32_t n2, double eps, double *a, double *b, int32_t max_iter,
                      double tol, int32_t check_every, int32_t *dev_iters, double *dev_err, int32_t *host_iters,
                      double *host_err, void *ws, size_t ws_bytes, void *stream);
/* The single-pass grid on the current device: *gr row groups x *gc partners per
 * row (host outputs; gc is the fewest partners whose column slices of <= 4,096
 * fit n2).  FA_ERR_SHAPE if the single pass is not used for this shape there. */
int fa_sinkhorn_fused_grid(int32_t n1, int32_t n2, int32_t *gr, int32_t *gc);
/* Bound on the polls of one partner wait of the single pass (>= 1; default
 * 4,194,304, about four seconds).  Process-wide; returns the previous bound. */
int32_t fa_set_sync_spin_limit(int32_t polls);

/* Plan recovery S_ij = exp((a_j + b_i - C_ij)/eps) (Eq. (4)) stored as s_dtype
 * (FA_F32 or FA_BF16, round-to-nearest-even).  If argmax is non-NULL it also
 * writes argmax_j (a_j + b_i - C_ij) per row i (lowest j on ties), int32[n1].
 * If truth (int32[n1], the true partner of row i in [0, n2), anything else = none)
 * is non-NULL, rank (int32[n1], out) receives 1 + #{j : S_ij > S_i,truth_i} computed
 * on the exact FP64 exponents in the same pass (the ranking behind Hits@K and MRR,
 * §4), or 0 for rows without a partner.  truth and rank are both NULL or both set. */
int fa_plan(const float *C, int32_t n1, int32_t n2, double eps, const double *a,
            const double *b, void *S, int32_t s_dtype, int32_t *argmax, const int32_t *truth,
            int32_t *rank, void *stream);

/* Top-k plan: for every row i the k largest entries of the plan of Eq. (4),
 * S_ij = exp((a_j + b_i - C_ij)/eps), in one pass over C and without writing S
 * (the plan is sparse in practice, §3.3, and a row's short list of candidates is
 * what an alignment consumer reads).
 *   C float[n1*n2] row-major, a double[n2], b double[n1] (device, in)
 *   1 <= k <= min(64, n2); FA_ERR_ARG otherwise
 *   val float[n1*k], idx int32[n1*k] (device, out, row-major): row i's entries,
 *     ordered by the FP64 exponent (a_j + b_i - C_ij)/eps as fa_plan forms it,
 *     larger first, lower j first on equal exponents.  idx[i*k] is fa_plan's
 *     argmax and val[i*k + q] equals fa_plan's FP32 S at (i, idx[i*k + q]) bit
 *     for bit.  Entries whose exponent is NaN are skipped; a row left with fewer
 *     than k comparable entries pads with idx = -1, val = 0.
 * Asynchronous on stream; the library allocates nothing. */
int fa_plan_topk(const float *C, int32_t n1, int32_t n2, double eps, const double *a,
                 const double *b, int32_t k, float *val, int32_t *idx, void *stream);

/* ----------------------------------------------------------------------- */
/* End to end (Algorithm 1)                                                  */
/* ----------------------------------------------------------------------- */

size_t fa_align_workspace_size(int32_t n1, int32_t n2, int32_t d, int32_t nL,
                               int64_t nnz1, int64_t nnz2, const fa_params *p);

/* Align G1 and G2 (Algorithm 1): Phase 1 once, then p->outer_iters times Phase 2 + Phase 3.
 *   X1 float[n1*d], X2 float[n2*d] (d may be 0: no attributes)
 *   anchors int32[nL*2]: pairs (node in G1, node in G2); each node may appear
 *     in at most one pair (FA_ERR_ARG otherwise; checked on the device, this
 *     check synchronises once)
 *   mlp_weights float[fa_mlp_param_count()] or NULL; required if p->warm_start
 *   S_out [n1*n2] of p->plan_dtype (out): the final plan.  Also the working plan
 *     of the outer iterations unless p->plan_in_ct; with p->plan_in_ct it may be
 *     NULL (then no dense plan is written at all)
 *   a_out double[n2], b_out double[n1], argmax_out int32[n1] (out)
 *   truth int32[n1] / rank_out int32[n1]: optional (both or neither), the rank of
 *     each row's true partner in the final plan, as in fa_plan
 *   topk (0 = none, else 1..min(64, n2)), topk_val float[n1*topk], topk_idx
 *     int32[n1*topk] (out): the final plan's top-k lists, as in fa_plan_topk
 *   stats host fa_stats (out), may be NULL
 * The call synchronises the stream after the anchor check, after every outer
 * iteration and at the end.  Returns FA_ERR_NUMERIC as soon as an inner solve
 * ends with a non-finite marginal error (the outputs are then partial), and
 * FA_WARN_NOT_CONVERGED if tol > 0 and some inner solve missed it. */
int fa_align(const fa_csr *A1, const fa_csr *A2, const float *X1, const float *X2, int32_t d,
             const int32_t *anchors, int32_t nL, const fa_params *p, const float *mlp_weights,
             void *S_out, double *a_out, double *b_out, int32_t *argmax_out, const int32_t *truth,
             int32_t *rank_out, int32_t topk, float *topk_val, int32_t *topk_idx, fa_stats *stats,
             void *ws, size_t ws_bytes, void *stream);

/* Algorithm 1 one outer iteration at a time: fa_align is exactly
 *   fa_align_begin; fa_align_step for t = 0 .. T-1; fa_align_end(steps = T)
 * on the same arguments, with the final argmax/truth/rank passed to the last step.
 * A caller can time, inspect or stop between outer iterations.  Every call takes
 * the same A1, A2, d, nL, p, S_out, a_out, b_out and workspace (the workspace holds
 * the state between calls; its layout depends on p, which must not change).
 *
 * fa_align_begin: anchor check (synchronises once), Phase 1, S^0 = mu nu^T in the
 *   working plan (S_out, or the C^T buffer with p->plan_in_ct), warm-start inputs.
 *   acc (host, nullable): phase_ms[0] accumulates the call's device time and, with
 *   p->profile, kernel_ms / kernel_calls its launches (the similarity GEMM).
 * fa_align_step: outer iteration t (cost rebuild, inner solve from the start the
 *   params select, plan).  Steps run in order, t = 0, 1, 2, ..., after
 *   fa_align_begin: each reads the state the previous ones left in the workspace
 *   (the plan, the duals, the sums behind FA_START_MEAN); calls out of order are
 *   not detected and give another (still finite-size, in-bounds) computation.  argmax_out/truth/rank_out (nullable; truth and rank_out
 *   together) are written from this step's plan, as fa_align does on its last step.
 *   Synchronises at the end; returns FA_ERR_NUMERIC if the solve's marginal error
 *   is not finite.  acc (host, nullable): with p->profile its phase_ms,
 *   kernel_ms and kernel_calls accumulate this step's device times.
 * fa_align_end: after `steps` steps (0: writes the S^0 plan and argmax into S_out
 *   like fa_align with outer_iters = 0); with p->plan_in_ct a non-NULL S_out
 *   receives the final dense plan; top-k lists as in fa_align; stats (nullable)
 *   receives every field except phase_ms, kernel_ms and kernel_calls.  Returns
 *   FA_WARN_NOT_CONVERGED like fa_align. */
int fa_align_begin(const fa_csr *A1, const fa_csr *A2, const float *X1, const float *X2, int32_t d,
                   const int32_t *anchors, int32_t nL, const fa_params *p, void *S_out, double *a_out,
                   double *b_out, fa_stats *acc, void *ws, size_t ws_bytes, void *stream);
int fa_align_step(const fa_csr *A1, const fa_csr *A2, int32_t d, int32_t nL, const fa_params *p,
                  const float *mlp_weights, int32_t t, void *S_out, double *a_out, double *b_out,
                  int32_t *argmax_out, const int32_t *truth, int32_t *rank_out, fa_stats *acc, void *ws,
                  size_t ws_bytes, void *stream);
int fa_align_end(const fa_csr *A1, const fa_csr *A2, int32_t d, int32_t nL, const fa_params *p, int32_t steps,
                 void *S_out, const double *a_out, const double *b_out, int32_t *argmax_out,
                 const int32_t *truth, int32_t *rank_out, int32_t topk, float *topk_val, int32_t *topk_idx,
                 fa_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ----------------------------------------------------------------------- */
/* Learned warm start: per-node inputs and a 3-layer MLP                     */
/* ----------------------------------------------------------------------- */

/* Width of the per-node input vector produced by fa_node_features. */
int32_t fa_node_feature_dim(void);

/* Per-node inputs of the warm-start network for one graph of an aligned pair:
 * log(1+deg), the 16-dim projection of the L2-normalised attributes by the
 * fixed matrix `proj` (float[d*16], may be NULL when d == 0), hop distance to
 * the nearest anchor (capped at 8, divided by 8), the random-walk anchor mass
 * Abar^h 1_anchor for h = 1, 2, 3, an is-anchor flag, log(n)/16 and a bias 1.
 *   A, inv_deg: this graph; anchor_nodes int32[nL] on this side
 *   X float[n*d]; out float[n * fa_node_feature_dim()] (row-major)
 *   ws >= fa_node_features_workspace_size(n) bytes. */
size_t fa_node_features_workspace_size(int32_t n);
int fa_node_features(const fa_csr *A, const float *inv_deg, const float *X, int32_t d,
                     const float *proj, const int32_t *anchor_nodes, int32_t nL, float *out,
                     void *ws, size_t ws_bytes, void *stream);

/* Parameter layout of the MLP  in -> 256 -> 256 -> 1 with SiLU activations:
 * W1[in*256], b1[256], W2[256*256], b2[256], W3[256], b3[1] (row-major, x @ W). */
int32_t fa_mlp_param_count(void);

/* Floats of the activation buffer the MLP entry points need for N rows. */
size_t fa_mlp_act_floats(int32_t N);

/* Forward pass: y[N] = scale * (h2 . W3 + b3) + offset with h1 = SiLU(x W1 + b1),
 * h2 = SiLU(h1 W2 + b2).  act float[fa_mlp_act_floats(N)] receives the
 * pre-activations and activations of both hidden layers for fa_mlp_backward. */
int fa_mlp_forward(const float *params, const float *x, int32_t N, float *y, float *act,
                   void *stream);

/* Backward pass of the mean squared error L = mean((y - t)^2) given the act of
 * the matching fa_mlp_forward call (act is consumed: overwritten with
 * intermediate gradients): grad float[fa_mlp_param_count()] (out, overwritten;
 * the scale and offset entries are not trained and get 0) and loss double[1]
 * (device, out). */
int fa_mlp_backward(const float *params, const float *x, const float *t, int32_t N,
                    const float *act, float *grad, double *loss, void *stream);

/* One Adam step (lr, beta1, beta2, eps_adam, step >= 1) on params with moment
 * buffers m, v (float[count], zero-initialised by the caller). */
int fa_adam_step(float *params, const float *grad, float *m, float *v, int32_t count,
                 double lr, double beta1, double beta2, double eps_adam, int32_t step,
                 void *stream);

/* ---------------------------------------------------------------- measurement */

/* Achievable read rate of the device (a reference for the streaming passes, not
 * part of Algorithm 1): reads x[0..n) once with 16-byte non-temporal loads and
 * writes one partial sum per thread.
 *   x        device float[n], n a multiple of 4, 16-byte aligned (in)
 *   partial  device float[nblocks * 256] (out, overwritten)
 *   nblocks  workgroups of 256 threads, 1..65536
 * Time it with events on `stream`; bytes read = 4 n.  Errors: FA_ERR_ARG. */
int fa_stream_read(const float *x, size_t n, float *partial, int32_t nblocks, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FASTALIGN_H */
