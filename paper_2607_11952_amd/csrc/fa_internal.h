// Launchers shared between translation units (not part of the ABI).
#pragma once

#include "fa_common.h"

namespace fa {

int launch_inv_deg(const fa_csr *A, float *inv, hipStream_t s);
int launch_colinv_weights(const fa_csr *A, const float *inv, float *w, hipStream_t s);
int launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
int launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);
int launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
int launch_anchor_index(const int32_t *anchors, int32_t nL, int side, int32_t n, int32_t *anchor_of,
                        int32_t *bad, hipStream_t s);
int launch_anchor_side(const int32_t *anchors, int32_t nL, int side, int32_t *nodes, hipStream_t s);
int launch_partner(const int32_t *anchors, const int32_t *anchor_of1, int32_t n1, int32_t *partner,
                   hipStream_t s);
int launch_f32_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s);
// [rows x cols] -> BF16 rows of stride ld >= cols, zero-padded (16-byte rows for the MFMA GEMM).
int launch_f32_to_bf16_rows(const float *x, int64_t rows, int32_t cols, int32_t ld, uint16_t *y, hipStream_t s);
int launch_positional(const fa_csr *A, const float *inv_deg, const int32_t *anchor_nodes, int32_t nL,
                      double beta, int32_t k, float *R, float *R_tmp, hipStream_t s);
int launch_sddmm(const fa_csr *A, const float *inv_deg, const float *R, int32_t nL, int32_t by_col,
                 float *out, hipStream_t s);
int launch_l2norm(const float *X, int32_t n, int32_t d, void *out, int32_t dt, hipStream_t s);

int launch_feature_sim(const void *X1, const void *X2, int32_t n1, int32_t n2, int32_t d, int32_t xdt,
                       const void *R1, const void *R2, int32_t nL, int32_t rdt, double alpha,
                       float *C, hipStream_t s);

// Rows per block of the block-transposed SpMM intermediate.
constexpr int kZtRows = 64;
size_t zt_bytes(int32_t chunk_rows, int32_t n2);

// Phase 2 cost rebuild over one row chunk at a time (Zt scratch of chunk_rows rows).
struct CostArgs {
  const fa_csr *A1, *A2;
  const float *w1, *inv1, *w2, *inv2;  // C1/C2 values; inverse degrees
  const void *S;
  int32_t s_dtype;
  const float *C_node;
  const int32_t *partner;
  const double *a, *b;
  double lambda_e, lambda_n, lambda_a, lambda_p, eps, eps_anchor, delta;
  float *C;
  float *Ct;  // nullable: also write C^T (n2 x n1) for the transposed column pass
};
int run_cost(const CostArgs &c, int32_t chunk_rows, void *zt, hipStream_t s, KTimer *tm = nullptr);
int run_propagate(const fa_csr *A1, const float *inv1, const fa_csr *A2, const float *inv2, float *C,
                  float *C_tmp, int32_t k, int32_t chunk_rows, void *zt, hipStream_t s);

// Sinkhorn workspace and loop.
struct SinkWs {
  double *pm;     // column partial maxima [nsplit * n2]
  double *ps;     // column partial sums   [nsplit * n2]
  double *a_next; // candidate a            [n2]
  double *errp;   // per-block L1 error partials
  int32_t *ctl;   // [0] done flag, [1] iterations done, [2] which buffer holds a, [4] abandoned wait
  double *err;    // [1] final marginal error
  uint64_t *part; // single-pass form (nullptr: two passes per iteration): tagged row partials [n1 * fuse_stride(gc)]
  double *pcol;   //   column sums per row group [gr * n2]
  int nsplit, nerrblk;
};
// fused: also carve the single-pass exchange (the loop then uses it when the
// shape and the device allow).
size_t sinkhorn_ws_bytes(int32_t n1, int32_t n2, bool fused);
int carve_sinkhorn(Carver &cv, int32_t n1, int32_t n2, SinkWs &w, bool fused);
// 1 if the last solve on this workspace abandoned a partner wait (reads the device; synchronises s).
int sinkhorn_fault(const SinkWs &w, hipStream_t s, int32_t *fault);
// Ct (nullable): C^T, row-major n2 x n1; when given the column pass streams it row by row.
int run_sinkhorn(const float *C, const float *Ct, int32_t n1, int32_t n2, double eps, double *a, double *b,
                 int32_t max_iter, double tol, int32_t check_every, int32_t *dev_iters, double *dev_err,
                 SinkWs &w, hipStream_t s, KTimer *tm = nullptr);
int run_plan(const float *C, int32_t n1, int32_t n2, double eps, const double *a, const double *b, void *S,
             int32_t sdt, int32_t *argmax, const int32_t *truth, int32_t *rank, hipStream_t s,
             KTimer *tm = nullptr);

// The plan without a dense buffer of its own: per-row top-k (k <= kTopkMax) and
// the transpose that regenerates C^T when the working plan lives in its buffer.
constexpr int kTopkMax = 64;
int run_plan_topk(const float *C, int32_t n1, int32_t n2, double eps, const double *a, const double *b, int32_t k,
                  float *val, int32_t *idx, hipStream_t s, KTimer *tm = nullptr);
int run_transpose(const float *C, int32_t n1, int32_t n2, float *Ct, hipStream_t s, KTimer *tm = nullptr);

// Warm start.
int run_node_features(const fa_csr *A, const float *inv_deg, const float *X, int32_t d, const float *proj,
                      const int32_t *anchor_nodes, int32_t nL, float *out, void *ws, size_t ws_bytes,
                      hipStream_t s);
int run_mlp_forward(const float *params, const float *x, int32_t N, float *y, float *act, hipStream_t s);
size_t mlp_act_floats(int32_t N);
size_t node_features_ws_bytes(int32_t n);
int32_t node_feature_dim();
int warm_start_duals(const float *mlp, const float *feat, int32_t n1, float *act, double eps, int32_t *bad, double *b,
                     hipStream_t s);

}  // namespace fa
