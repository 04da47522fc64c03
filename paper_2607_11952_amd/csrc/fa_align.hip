// Algorithm 1 end to end on one GPU, in one call (fa_align) or one outer iteration
// at a time (fa_align_begin, fa_align_step, fa_align_end; fa_align is exactly that
// sequence).  All buffers come from the caller's workspace; all work is enqueued on
// the caller's stream.  The host synchronises after validating the anchors on the
// device, at the end of every outer iteration (to check the solve's marginal error
// and time the phases) and at the end to return the statistics.
#include <math.h>
#include <string.h>

#include <type_traits>

#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

struct AlignLayout {
  int32_t chunk_rows;
};

static AlignLayout align_layout(int32_t n1, int32_t n2, const fa_params *p) {
  AlignLayout L;
  int32_t cr = p->chunk_rows;
  if (cr <= 0) {
    // Keep the SpMM intermediate (two sets of chunk_rows x n2) near 16 GiB.
    const double row_bytes = 2.0 * n2 * sizeof(float);
    const double cap = 16.0 * (1ull << 30);
    cr = static_cast<int32_t>(fmin(static_cast<double>(n1), floor(cap / fmax(row_bytes, 1.0))));
    cr = cr / kZtRows * kZtRows;
    if (cr < kZtRows) cr = kZtRows;
  }
  if (cr > n1) cr = n1;
  if (cr < 1) cr = 1;
  L.chunk_rows = cr;
  return L;
}

struct AlignBufs {
  float *inv1, *inv2;
  int32_t *anchor_of1, *anchor_of2, *partner, *nodes1, *nodes2, *bad;
  float *R1, *R1t, *R2, *R2t;
  uint16_t *Rb1, *Rb2;
  void *Xh1, *Xh2;
  float *w1, *w2;
  float *C_node, *C, *Ct;  // Ct: C^T (n2 x n1) when p->transpose_cost
  void *zt;
  SinkWs sink;
  int32_t *st_iters;
  double *st_err;
  float *feat, *act;  // warm start: per-node inputs (n1 rows) and MLP activations
  void *nf_ws;
  double *a_keep, *b_keep;  // warm start: the learned start's solve while the cold one runs
  double *a_sum, *b_sum;    // FA_START_MEAN: running sums of the solves' duals
};

// Row stride of the BF16 encodings: whole 16-byte pieces, so that the similarity
// GEMM stages them with vector loads; the zero pad adds nothing to R1 R2^T.
static int32_t bf16_stride(int32_t nL) { return (nL + 7) / 8 * 8; }

template <typename Cv>
static void carve_align(Cv &cv, int32_t n1, int32_t n2, int32_t d, int32_t nL, int64_t nnz1, int64_t nnz2,
                        const fa_params *p, const AlignLayout &L, AlignBufs *B) {
  const size_t N = static_cast<size_t>(n1) * n2;
  const bool bf = p->feat_dtype == FA_BF16;
  auto T = [&](auto *ptr, size_t count) {
    using E = std::remove_pointer_t<decltype(ptr)>;
    if constexpr (std::is_same_v<Cv, Sizer>) {
      cv.template take<E>(count);
      return static_cast<E *>(nullptr);
    } else {
      return cv.template take<E>(count);
    }
  };
  AlignBufs b{};
  b.inv1 = T((float *)0, n1);
  b.inv2 = T((float *)0, n2);
  b.anchor_of1 = T((int32_t *)0, n1);
  b.anchor_of2 = T((int32_t *)0, n2);
  b.partner = T((int32_t *)0, n1);
  b.nodes1 = T((int32_t *)0, nL + 1);
  b.nodes2 = T((int32_t *)0, nL + 1);
  b.bad = T((int32_t *)0, 4);
  if (bf) {
    b.Xh1 = T((uint16_t *)0, static_cast<size_t>(n1) * d);
    b.Xh2 = T((uint16_t *)0, static_cast<size_t>(n2) * d);
  } else {
    b.Xh1 = T((float *)0, static_cast<size_t>(n1) * d);
    b.Xh2 = T((float *)0, static_cast<size_t>(n2) * d);
  }
  b.w1 = T((float *)0, nnz1 + 1);
  b.w2 = T((float *)0, nnz2 + 1);
  b.C_node = T((float *)0, N);
  b.C = T((float *)0, N);
  if (p->transpose_cost) b.Ct = T((float *)0, N);
  // Phase-1 encodings R1, R2 and their ping-pong scratch are dead once the SDDMMs and
  // the similarity GEMM have run, before C is first written (propagation scratch or
  // the initial fill), so they live inside C when they fit; the BF16 copies then reuse
  // the scratch halves, dead once the encodings are built.  Otherwise they get buffers
  // of their own.
  const size_t r1 = align_up(static_cast<size_t>(n1) * nL * sizeof(float), 256);
  const size_t r2 = align_up(static_cast<size_t>(n2) * nL * sizeof(float), 256);
  const size_t s1 = static_cast<size_t>(n1) * bf16_stride(nL) * sizeof(uint16_t);
  const size_t s2 = static_cast<size_t>(n2) * bf16_stride(nL) * sizeof(uint16_t);
  const bool in_c = 2 * (r1 + r2) <= N * sizeof(float) && (!bf || (s1 <= r1 && s2 <= r2));
  if (in_c) {
    if constexpr (!std::is_same_v<Cv, Sizer>) {
      char *c = reinterpret_cast<char *>(b.C);
      b.R1 = reinterpret_cast<float *>(c);
      b.R1t = reinterpret_cast<float *>(c + r1);
      b.R2 = reinterpret_cast<float *>(c + 2 * r1);
      b.R2t = reinterpret_cast<float *>(c + 2 * r1 + r2);
      if (bf) {
        b.Rb1 = reinterpret_cast<uint16_t *>(b.R1t);
        b.Rb2 = reinterpret_cast<uint16_t *>(b.R2t);
      }
    }
  } else {
    b.R1 = T((float *)0, static_cast<size_t>(n1) * nL);
    b.R1t = T((float *)0, static_cast<size_t>(n1) * nL);
    b.R2 = T((float *)0, static_cast<size_t>(n2) * nL);
    b.R2t = T((float *)0, static_cast<size_t>(n2) * nL);
    if (bf) {
      b.Rb1 = T((uint16_t *)0, static_cast<size_t>(n1) * bf16_stride(nL));
      b.Rb2 = T((uint16_t *)0, static_cast<size_t>(n2) * bf16_stride(nL));
    }
  }
  b.zt = T((char *)0, zt_bytes(L.chunk_rows, n2));
  b.sink.pm = nullptr;
  b.st_iters = T((int32_t *)0, 64);
  b.st_err = T((double *)0, 64);
  if (p->warm_start) {
    b.feat = T((float *)0, static_cast<size_t>(n1) * node_feature_dim());
    b.act = T((float *)0, mlp_act_floats(n1) + 2 * static_cast<size_t>(ceil_div(n1, 256)) + 8);
    b.nf_ws = T((char *)0, node_features_ws_bytes(n1));
    b.a_keep = T((double *)0, n2);
    b.b_keep = T((double *)0, n1);
  }
  if (p->dual_start == FA_START_MEAN) {
    b.a_sum = T((double *)0, n2);
    b.b_sum = T((double *)0, n1);
  }
  if (B) *B = b;
}

// Start of inner solve t >= 1 from the running mean of the earlier solves' duals:
// x <- sum / t.
__global__ void k_dual_mean(const double *__restrict__ sum, int32_t n, double inv_t, double *__restrict__ x) {
  FA_GRID_STRIDE(i, n) x[i] = sum[i] * inv_t;
}
// sum <- sum + x (or sum <- x when first).
__global__ void k_dual_accum(double *__restrict__ sum, const double *__restrict__ x, int32_t n, int32_t first) {
  FA_GRID_STRIDE(i, n) sum[i] = first ? x[i] : sum[i] + x[i];
}

// Host-visible record of the learned start, kept in the workspace between steps.
struct AlignRec {
  int32_t fell_back, warm_iters, cold_iters, pad;
  double warm_err, cold_err;
};

struct AlignCtx {
  const fa_csr *A1, *A2;
  int32_t n1, n2, d, nL;
  const fa_params *p;
  AlignLayout L;
  AlignBufs B;
  AlignRec *rec;  // device
  hipStream_t s;
};

}  // namespace fa

using namespace fa;

static int validate(const fa_csr *A1, const fa_csr *A2, int32_t d, int32_t nL, const fa_params *p) {
  FA_TRY(check_csr(A1, "fa_align A1"));
  FA_TRY(check_csr(A2, "fa_align A2"));
  FA_REQUIRE(p, FA_ERR_ARG, "fa_align: null params");
  FA_REQUIRE(A1->n > 0 && A2->n > 0, FA_ERR_SHAPE, "fa_align: both graphs need nodes (n1 = %d, n2 = %d)", A1->n, A2->n);
  FA_REQUIRE(d >= 0 && nL >= 0, FA_ERR_ARG, "fa_align: d = %d, nL = %d", d, nL);
  FA_REQUIRE(p->eps > 0 && p->eps_anchor > 0 && p->delta_nbr >= 0 && p->tol >= 0, FA_ERR_ARG,
             "fa_align: need eps > 0, eps_anchor > 0, delta_nbr >= 0, tol >= 0");
  FA_REQUIRE(isfinite(p->alpha) && isfinite(p->beta) && isfinite(p->lambda_e) && isfinite(p->lambda_n) &&
                 isfinite(p->lambda_a) && isfinite(p->lambda_p),
             FA_ERR_ARG, "fa_align: non-finite parameter");
  FA_REQUIRE(p->k_r >= 0 && p->k_node >= 0 && p->outer_iters >= 0 && p->inner_iters >= 0 && p->check_every >= 1,
             FA_ERR_ARG, "fa_align: negative iteration count or check_every < 1");
  FA_REQUIRE(p->plan_dtype == FA_F32 || p->plan_dtype == FA_BF16, FA_ERR_ARG, "fa_align: plan_dtype %d",
             p->plan_dtype);
  FA_REQUIRE(p->feat_dtype == FA_F32 || p->feat_dtype == FA_BF16, FA_ERR_ARG, "fa_align: feat_dtype %d",
             p->feat_dtype);
  FA_REQUIRE(p->dual_start == FA_START_ZERO || p->dual_start == FA_START_CARRY || p->dual_start == FA_START_MEAN,
             FA_ERR_ARG, "fa_align: dual_start %d", p->dual_start);
  FA_REQUIRE(p->warm_probe >= 0, FA_ERR_ARG, "fa_align: warm_probe %d < 0", p->warm_probe);
  FA_REQUIRE(!p->plan_in_ct || p->transpose_cost, FA_ERR_ARG, "fa_align: plan_in_ct needs transpose_cost = 1");
  return FA_OK;
}

extern "C" size_t fa_align_workspace_size(int32_t n1, int32_t n2, int32_t d, int32_t nL, int64_t nnz1, int64_t nnz2,
                                          const fa_params *p) {
  if (!p || n1 <= 0 || n2 <= 0 || d < 0 || nL < 0 || nnz1 < 0 || nnz2 < 0) return 0;
  AlignLayout L = align_layout(n1, n2, p);
  Sizer z;
  carve_align(z, n1, n2, d, nL, nnz1, nnz2, p, L, nullptr);
  z.take<AlignRec>(1);
  z.off = align_up(z.off, 256) + sinkhorn_ws_bytes(n1, n2, p->sink_fused != 0);
  return z.off + 256;
}

// Validate the arguments every stepwise call shares and carve the workspace.
static int open_ctx(AlignCtx &x, const fa_csr *A1, const fa_csr *A2, int32_t d, int32_t nL, const fa_params *p,
                    void *ws, size_t ws_bytes, void *stream) {
  FA_TRY(validate(A1, A2, d, nL, p));
  x.A1 = A1;
  x.A2 = A2;
  x.n1 = A1->n;
  x.n2 = A2->n;
  x.d = d;
  x.nL = nL;
  x.p = p;
  const size_t need = fa_align_workspace_size(x.n1, x.n2, d, nL, A1->nnz, A2->nnz, p);
  FA_REQUIRE(ws && ws_bytes >= need, FA_ERR_WORKSPACE, "fa_align: workspace %zu < %zu bytes", ws_bytes, need);
  x.s = static_cast<hipStream_t>(stream);
  x.L = align_layout(x.n1, x.n2, p);
  Carver cv(ws, ws_bytes);
  carve_align(cv, x.n1, x.n2, d, nL, A1->nnz, A2->nnz, p, x.L, &x.B);
  x.rec = cv.take<AlignRec>(1);
  FA_TRY(carve_sinkhorn(cv, x.n1, x.n2, x.B.sink, p->sink_fused != 0));
  FA_REQUIRE(cv.ok, FA_ERR_WORKSPACE, "fa_align: workspace carve failed");
  return FA_OK;
}

// The plan the outer iterations read and write: the caller's S_out, or the C^T
// buffer (FP32 n2 x n1, at least as large as an n1 x n2 plan of either type)
// between the plan pass and the next cost rebuild.
static void *working_plan(const AlignCtx &x, void *S_out) {
  return x.p->plan_in_ct ? static_cast<void *>(x.B.Ct) : S_out;
}

// Anchor check (synchronises once), Phase 1, S^0 = mu nu^T and the warm-start inputs.
static int align_begin(AlignCtx &x, const float *X1, const float *X2, const int32_t *anchors, void *S_out, double *a,
                       double *b, KTimer *tm) {
  const fa_params *p = x.p;
  AlignBufs &B = x.B;
  const int32_t n1 = x.n1, n2 = x.n2, d = x.d, nL = x.nL;
  hipStream_t s = x.s;
  FA_REQUIRE(d == 0 || (X1 && X2), FA_ERR_ARG, "fa_align: null attributes with d = %d", d);
  FA_REQUIRE(nL == 0 || anchors, FA_ERR_ARG, "fa_align: null anchors");
  FA_REQUIRE((S_out || p->plan_in_ct) && a && b, FA_ERR_ARG, "fa_align: null output");
  FA_HIP(hipMemsetAsync(B.bad, 0, sizeof(int32_t) * 4, s));
  FA_TRY(launch_anchor_index(anchors, nL, 0, n1, B.anchor_of1, B.bad, s));
  FA_TRY(launch_anchor_index(anchors, nL, 1, n2, B.anchor_of2, B.bad + 1, s));
  int32_t bad[2] = {0, 0};
  FA_HIP(hipMemcpyAsync(bad, B.bad, sizeof bad, hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  FA_REQUIRE(bad[0] == 0 && bad[1] == 0, FA_ERR_ARG,
             "fa_align: anchors out of range or repeated (%d bad on G1, %d on G2)", bad[0], bad[1]);
  FA_TRY(launch_anchor_side(anchors, nL, 0, B.nodes1, s));
  FA_TRY(launch_anchor_side(anchors, nL, 1, B.nodes2, s));
  FA_TRY(launch_partner(anchors, B.anchor_of1, n1, B.partner, s));

  FA_TRY(launch_inv_deg(x.A1, B.inv1, s));
  FA_TRY(launch_inv_deg(x.A2, B.inv2, s));
  FA_TRY(launch_positional(x.A1, B.inv1, B.nodes1, nL, p->beta, p->k_r, B.R1, B.R1t, s));
  FA_TRY(launch_positional(x.A2, B.inv2, B.nodes2, nL, p->beta, p->k_r, B.R2, B.R2t, s));
  FA_TRY(launch_sddmm(x.A1, B.inv1, B.R1, nL, 0, B.w1, s));
  FA_TRY(launch_sddmm(x.A2, B.inv2, B.R2, nL, 1, B.w2, s));
  const int32_t fdt = p->feat_dtype;
  if (d > 0) {
    if (p->feat_l2norm) {
      FA_TRY(launch_l2norm(X1, n1, d, B.Xh1, fdt, s));
      FA_TRY(launch_l2norm(X2, n2, d, B.Xh2, fdt, s));
    } else if (fdt == FA_BF16) {
      FA_TRY(launch_f32_to_bf16(X1, static_cast<int64_t>(n1) * d, static_cast<uint16_t *>(B.Xh1), s));
      FA_TRY(launch_f32_to_bf16(X2, static_cast<int64_t>(n2) * d, static_cast<uint16_t *>(B.Xh2), s));
    } else {
      FA_HIP(hipMemcpyAsync(B.Xh1, X1, sizeof(float) * n1 * d, hipMemcpyDeviceToDevice, s));
      FA_HIP(hipMemcpyAsync(B.Xh2, X2, sizeof(float) * n2 * d, hipMemcpyDeviceToDevice, s));
    }
  }
  const void *R1op = B.R1, *R2op = B.R2;
  int32_t nLop = nL;
  if (fdt == FA_BF16) {
    nLop = bf16_stride(nL);
    FA_TRY(launch_f32_to_bf16_rows(B.R1, n1, nL, nLop, B.Rb1, s));
    FA_TRY(launch_f32_to_bf16_rows(B.R2, n2, nL, nLop, B.Rb2, s));
    R1op = B.Rb1;
    R2op = B.Rb2;
  }
  FA_TIMED(tm, KK_FEATSIM, s,
           FA_TRY(launch_feature_sim(B.Xh1, B.Xh2, n1, n2, d, fdt, R1op, R2op, nLop, fdt, p->alpha, B.C_node, s)));
  FA_TRY(run_propagate(x.A1, B.inv1, x.A2, B.inv2, B.C_node, B.C, p->k_node, x.L.chunk_rows, B.zt, s));

  // S^0 = mu nu^T, written as the plan of C = eps*log(n1 n2) with a = b = 0.
  const size_t N = static_cast<size_t>(n1) * n2;
  FA_TRY(launch_fill_f64(a, n2, 0.0, s));
  FA_TRY(launch_fill_f64(b, n1, 0.0, s));
  FA_TRY(launch_fill_f32(B.C, static_cast<int64_t>(N), static_cast<float>(p->eps * log(static_cast<double>(n1) * n2)), s));
  FA_TRY(run_plan(B.C, n1, n2, p->eps, a, b, working_plan(x, S_out), p->plan_dtype, nullptr, nullptr, nullptr, s));
  if (p->warm_start)
    FA_TRY(run_node_features(x.A1, B.inv1, X1, d, nullptr, B.nodes1, nL, B.feat, B.nf_ws, node_features_ws_bytes(n1),
                             s));
  FA_TRY(launch_fill_i32(B.st_iters, 64, 0, s));
  FA_TRY(launch_fill_f64(B.st_err, 64, 0.0, s));
  AlignRec r{0, -1, -1, 0, NAN, NAN};
  FA_HIP(hipMemcpyAsync(x.rec, &r, sizeof r, hipMemcpyHostToDevice, s));
  FA_HIP(hipStreamSynchronize(s));  // r lives on this stack frame
  return FA_OK;
}

// FA_ERR_SYNC if the last inner solve gave up a partner wait of the single pass
// (synchronises; only the single-pass form can give up).
static int sink_ok(const AlignCtx &x, int32_t t) {
  if (!x.p->sink_fused) return FA_OK;
  int32_t fault = 0;
  FA_TRY(sinkhorn_fault(x.B.sink, x.s, &fault));
  FA_REQUIRE(!fault, FA_ERR_SYNC, "fa_align: a partner wait of the single-pass Sinkhorn gave up at outer iteration %d",
             t);
  return FA_OK;
}

template <typename T>
static int read_dev(T *host, const T *dev, hipStream_t s) {
  FA_HIP(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  return FA_OK;
}

// Outer iteration t: cost rebuild (Phase 2), the inner solve from the configured
// start (Phase 3), the plan.  Synchronises at the end and fails with
// FA_ERR_NUMERIC if the solve's marginal error is not finite.  phase_ms (nullable)
// accumulates the device time of the three parts.
static int align_step(AlignCtx &x, int32_t t, const float *mlp, void *S_out, double *a, double *b, int32_t *argmax,
                      const int32_t *truth, int32_t *rank, KTimer *tm, double *phase_ms) {
  const fa_params *p = x.p;
  AlignBufs &B = x.B;
  const int32_t n1 = x.n1, n2 = x.n2;
  hipStream_t s = x.s;
  FA_REQUIRE(t >= 0, FA_ERR_ARG, "fa_align_step: t = %d", t);
  FA_REQUIRE(a && b && (S_out || p->plan_in_ct), FA_ERR_ARG, "fa_align_step: null output");
  FA_REQUIRE((truth == nullptr) == (rank == nullptr), FA_ERR_ARG, "fa_align_step: truth and rank go together");
  FA_REQUIRE(!p->warm_start || mlp, FA_ERR_ARG, "fa_align: warm_start needs mlp_weights");
  void *S_work = working_plan(x, S_out);
  hipEvent_t ev[4];
  int nev = 0;
  struct EvGuard {
    hipEvent_t *e;
    int &n;
    ~EvGuard() {
      for (int q = 0; q < n; ++q) (void)hipEventDestroy(e[q]);
    }
  } guard{ev, nev};
  for (; nev < 4; ++nev) FA_HIP(hipEventCreate(&ev[nev]));

  FA_HIP(hipEventRecord(ev[0], s));
  CostArgs c{x.A1, x.A2, B.w1, B.inv1, B.w2, B.inv2, S_work, p->plan_dtype, B.C_node, B.partner, a, b,
             p->lambda_e, p->lambda_n, p->lambda_a, p->lambda_p, p->eps, p->eps_anchor, p->delta_nbr, B.C,
             p->transpose_cost && !p->plan_in_ct ? B.Ct : nullptr};
  FA_TRY(run_cost(c, x.L.chunk_rows, B.zt, s, tm));
  if (p->plan_in_ct) FA_TRY(run_transpose(B.C, n1, n2, B.Ct, s, tm));  // overwrites the plan just read
  FA_HIP(hipEventRecord(ev[1], s));

  const bool warm = p->warm_start && t == 0;
  if (warm) {
    FA_TRY(warm_start_duals(mlp, B.feat, n1, B.act, p->eps, B.bad + 2, b, s));
    FA_TRY(launch_fill_f64(a, n2, 0.0, s));
  } else if (t == 0 || p->dual_start == FA_START_ZERO) {
    FA_TRY(launch_fill_f64(a, n2, 0.0, s));
    FA_TRY(launch_fill_f64(b, n1, 0.0, s));
  } else if (p->dual_start == FA_START_MEAN) {
    FA_LAUNCH(k_dual_mean, stride_grid(n2), dim3(256), 0, s, B.a_sum, n2, 1.0 / t, a);
    FA_LAUNCH(k_dual_mean, stride_grid(n1), dim3(256), 0, s, B.b_sum, n1, 1.0 / t, b);
  }  // FA_START_CARRY: the previous solve's duals are the start
  const int slot = t < 64 ? t : 63;
  int32_t *it_slot = B.st_iters + slot;
  double *er_slot = B.st_err + slot;
  const float *Ct = p->transpose_cost ? B.Ct : nullptr;
  // the learned start's solve gets warm_probe iterations when a cold rerun backs it up
  const bool probe = warm && p->warm_fallback && p->tol > 0 && p->warm_probe > 0 && p->warm_probe < p->inner_iters;
  const int32_t budget = probe ? p->warm_probe : p->inner_iters;
  FA_TRY(run_sinkhorn(B.C, Ct, n1, n2, p->eps, a, b, budget, p->tol, p->check_every, it_slot, er_slot, B.sink, s, tm));
  FA_TRY(sink_ok(x, t));
  if (warm) {
    // The cold start stays the reference: a learned start whose solve misses tol is
    // rerun from zero duals and the run keeps whichever solve ends closer to the
    // marginals.
    AlignRec r{0, -1, -1, 0, NAN, NAN};
    int32_t nonfinite = 0, both = 0;  // host sources of the copies below: alive until the sync
    double keep_err = 0.0;
    FA_TRY(read_dev(&nonfinite, B.bad + 2, s));
    FA_TRY(read_dev(&r.warm_iters, it_slot, s));
    FA_TRY(read_dev(&r.warm_err, er_slot, s));
    if (nonfinite) r.fell_back = 1;  // the start was already zero
    if (!nonfinite && p->warm_fallback && p->tol > 0 && !(r.warm_err <= p->tol)) {
      FA_HIP(hipMemcpyAsync(B.a_keep, a, sizeof(double) * n2, hipMemcpyDeviceToDevice, s));
      FA_HIP(hipMemcpyAsync(B.b_keep, b, sizeof(double) * n1, hipMemcpyDeviceToDevice, s));
      FA_TRY(launch_fill_f64(a, n2, 0.0, s));
      FA_TRY(launch_fill_f64(b, n1, 0.0, s));
      FA_TRY(run_sinkhorn(B.C, Ct, n1, n2, p->eps, a, b, p->inner_iters, p->tol, p->check_every, it_slot, er_slot,
                          B.sink, s, tm));
      FA_TRY(sink_ok(x, t));
      FA_TRY(read_dev(&r.cold_iters, it_slot, s));
      FA_TRY(read_dev(&r.cold_err, er_slot, s));
      keep_err = r.cold_err;
      if (r.warm_err <= r.cold_err) {  // the learned start's solve is at least as close: keep it
        FA_HIP(hipMemcpyAsync(a, B.a_keep, sizeof(double) * n2, hipMemcpyDeviceToDevice, s));
        FA_HIP(hipMemcpyAsync(b, B.b_keep, sizeof(double) * n1, hipMemcpyDeviceToDevice, s));
        keep_err = r.warm_err;
      } else {
        r.fell_back = 2;
      }
      both = r.warm_iters + r.cold_iters;  // both solves ran
      FA_HIP(hipMemcpyAsync(it_slot, &both, sizeof both, hipMemcpyHostToDevice, s));
      FA_HIP(hipMemcpyAsync(er_slot, &keep_err, sizeof keep_err, hipMemcpyHostToDevice, s));
    }
    FA_HIP(hipMemcpyAsync(x.rec, &r, sizeof r, hipMemcpyHostToDevice, s));
    FA_HIP(hipStreamSynchronize(s));  // the copies above read this stack frame
  }
  if (p->dual_start == FA_START_MEAN) {
    FA_LAUNCH(k_dual_accum, stride_grid(n2), dim3(256), 0, s, B.a_sum, a, n2, t == 0);
    FA_LAUNCH(k_dual_accum, stride_grid(n1), dim3(256), 0, s, B.b_sum, b, n1, t == 0);
  }
  FA_HIP(hipEventRecord(ev[2], s));
  FA_TRY(run_plan(B.C, n1, n2, p->eps, a, b, S_work, p->plan_dtype, argmax, truth, rank, s, tm));
  FA_HIP(hipEventRecord(ev[3], s));
  FA_HIP(hipEventSynchronize(ev[3]));
  if (phase_ms) {
    float ms = 0.f;
    FA_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    phase_ms[1] += ms;
    FA_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
    phase_ms[2] += ms;
    FA_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
    phase_ms[3] += ms;
  }
  double err = 0.0;
  FA_TRY(read_dev(&err, er_slot, s));
  FA_REQUIRE(isfinite(err), FA_ERR_NUMERIC, "fa_align: non-finite marginal error at outer iteration %d", t);
  return FA_OK;
}

// After the last step: the plan of S^0 when no step ran, the dense plan when the
// working plan lived in C^T, the top-k lists and the statistics.  Returns
// FA_WARN_NOT_CONVERGED if tol > 0 and some recorded solve missed it.
static int align_end(AlignCtx &x, int32_t steps, void *S_out, const double *a, const double *b, int32_t *argmax,
                     const int32_t *truth, int32_t *rank, int32_t topk, float *topk_val, int32_t *topk_idx,
                     fa_stats *stats, KTimer *tm) {
  const fa_params *p = x.p;
  AlignBufs &B = x.B;
  const int32_t n1 = x.n1, n2 = x.n2;
  hipStream_t s = x.s;
  FA_REQUIRE(steps >= 0, FA_ERR_ARG, "fa_align_end: steps = %d", steps);
  FA_REQUIRE((truth == nullptr) == (rank == nullptr), FA_ERR_ARG, "fa_align: truth and rank_out go together");
  FA_REQUIRE(topk == 0 || (topk >= 1 && topk <= kTopkMax && topk <= n2 && topk_val && topk_idx), FA_ERR_ARG,
             "fa_align: topk = %d needs 1 <= topk <= min(%d, n2) and both top-k outputs", topk, kTopkMax);
  if (steps == 0) {
    FA_REQUIRE(S_out || p->plan_in_ct, FA_ERR_ARG, "fa_align: null output");
    FA_TRY(run_plan(B.C, n1, n2, p->eps, a, b, S_out ? S_out : working_plan(x, S_out), p->plan_dtype, argmax, truth,
                    rank, s));
  } else if (p->plan_in_ct && S_out) {
    FA_TRY(run_plan(B.C, n1, n2, p->eps, a, b, S_out, p->plan_dtype, nullptr, nullptr, nullptr, s, tm));
  }
  if (topk > 0) FA_TRY(run_plan_topk(B.C, n1, n2, p->eps, a, b, topk, topk_val, topk_idx, s, tm));
  int32_t iters[64] = {0};
  double errs[64] = {0};
  AlignRec r{0, -1, -1, 0, NAN, NAN};
  const int nrec = steps < 64 ? steps : 64;
  FA_HIP(hipMemcpyAsync(&r, x.rec, sizeof r, hipMemcpyDeviceToHost, s));
  if (nrec > 0) {
    FA_HIP(hipMemcpyAsync(iters, B.st_iters, sizeof(int32_t) * nrec, hipMemcpyDeviceToHost, s));
    FA_HIP(hipMemcpyAsync(errs, B.st_err, sizeof(double) * nrec, hipMemcpyDeviceToHost, s));
  }
  FA_HIP(hipStreamSynchronize(s));
  bool all_conv = true;
  int32_t total = 0;
  for (int t = 0; t < nrec; ++t) {
    total += iters[t];
    if (!(errs[t] <= p->tol)) all_conv = false;
  }
  if (stats) {
    stats->outer_done = steps;
    stats->inner_total = total;
    stats->fell_back = r.fell_back;
    stats->converged_all = all_conv ? 1 : 0;
    stats->marg_err = nrec > 0 ? errs[nrec - 1] : 0.0;
    stats->warm_iters = r.warm_iters;
    stats->cold_iters = r.cold_iters;
    stats->warm_err = r.warm_err;
    stats->cold_err = r.cold_err;
    for (int t = 0; t < 64; ++t) {
      stats->inner_iters[t] = t < nrec ? iters[t] : 0;
      stats->inner_err[t] = t < nrec ? errs[t] : 0.0;
    }
  }
  if (p->tol > 0 && !all_conv) return FA_WARN_NOT_CONVERGED;
  return FA_OK;
}

static void stats_timing(fa_stats *st, const KTimer *tm, const double *phase_ms, bool add) {
  if (!st) return;
  for (int q = 0; q < 4; ++q) st->phase_ms[q] = (add ? st->phase_ms[q] : 0.0) + phase_ms[q];
  for (int k = 0; k < KK_COUNT; ++k) {
    st->kernel_ms[k] = (add ? st->kernel_ms[k] : 0.0) + (tm ? tm->ms[k] : 0.0);
    st->kernel_calls[k] = (add ? st->kernel_calls[k] : 0) + (tm ? tm->calls[k] : 0);
  }
}

extern "C" int fa_align(const fa_csr *A1, const fa_csr *A2, const float *X1, const float *X2, int32_t d,
                        const int32_t *anchors, int32_t nL, const fa_params *p, const float *mlp_weights, void *S_out,
                        double *a_out, double *b_out, int32_t *argmax_out, const int32_t *truth,
                        int32_t *rank_out, int32_t topk, float *topk_val, int32_t *topk_idx, fa_stats *stats,
                        void *ws, size_t ws_bytes, void *stream) {
  AlignCtx x;
  FA_TRY(open_ctx(x, A1, A2, d, nL, p, ws, ws_bytes, stream));
  FA_REQUIRE((truth == nullptr) == (rank_out == nullptr), FA_ERR_ARG, "fa_align: truth and rank_out go together");
  FA_REQUIRE(argmax_out, FA_ERR_ARG, "fa_align: null output");
  FA_REQUIRE(topk == 0 || (topk >= 1 && topk <= kTopkMax && topk <= x.n2 && topk_val && topk_idx), FA_ERR_ARG,
             "fa_align: topk = %d needs 1 <= topk <= min(%d, n2) and both top-k outputs", topk, kTopkMax);
  FA_REQUIRE(!p->warm_start || mlp_weights, FA_ERR_ARG, "fa_align: warm_start needs mlp_weights");
  KTimer *tm = nullptr;
  struct TmGuard {
    KTimer *&t;
    ~TmGuard() { delete t; }
  } tmguard{tm};
  if (p->profile) {
    tm = new KTimer();
    FA_REQUIRE(tm->init(), FA_ERR_HIP, "fa_align: could not create timing events");
  }
  double phase_ms[4] = {0, 0, 0, 0};
  hipEvent_t e0, e1;
  FA_HIP(hipEventCreate(&e0));
  struct EvGuard {
    hipEvent_t a, b;
    bool hb;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      if (hb) (void)hipEventDestroy(b);
    }
  } evg{e0, e0, false};
  FA_HIP(hipEventCreate(&e1));
  evg.b = e1;
  evg.hb = true;
  FA_HIP(hipEventRecord(e0, x.s));
  FA_TRY(align_begin(x, X1, X2, anchors, S_out, a_out, b_out, tm));
  FA_HIP(hipEventRecord(e1, x.s));
  FA_HIP(hipEventSynchronize(e1));
  float f = 0.f;
  FA_HIP(hipEventElapsedTime(&f, e0, e1));
  phase_ms[0] = f;
  const int32_t T = p->outer_iters;
  for (int32_t t = 0; t < T; ++t) {
    const bool last = t == T - 1;
    FA_TRY(align_step(x, t, mlp_weights, S_out, a_out, b_out, last ? argmax_out : nullptr, last ? truth : nullptr,
                      last ? rank_out : nullptr, tm, phase_ms));
    if (tm) tm->collect();
  }
  const int st = align_end(x, T, S_out, a_out, b_out, T == 0 ? argmax_out : nullptr, T == 0 ? truth : nullptr,
                           T == 0 ? rank_out : nullptr, topk, topk_val, topk_idx, stats, tm);
  FA_TRY(st);
  if (tm) tm->collect();  // launches after the last outer iteration (top-k; all of them if T = 0)
  stats_timing(stats, tm, phase_ms, false);
  return st;
}

extern "C" int fa_align_begin(const fa_csr *A1, const fa_csr *A2, const float *X1, const float *X2, int32_t d,
                              const int32_t *anchors, int32_t nL, const fa_params *p, void *S_out, double *a_out,
                              double *b_out, fa_stats *acc, void *ws, size_t ws_bytes, void *stream) {
  AlignCtx x;
  FA_TRY(open_ctx(x, A1, A2, d, nL, p, ws, ws_bytes, stream));
  KTimer *tm = nullptr;
  struct TmGuard {
    KTimer *&t;
    ~TmGuard() { delete t; }
  } tmguard{tm};
  if (p->profile && acc) {
    tm = new KTimer();
    FA_REQUIRE(tm->init(), FA_ERR_HIP, "fa_align_begin: could not create timing events");
  }
  hipEvent_t e0, e1;
  FA_HIP(hipEventCreate(&e0));
  struct EvGuard {
    hipEvent_t a, b;
    bool hb;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      if (hb) (void)hipEventDestroy(b);
    }
  } evg{e0, e0, false};
  FA_HIP(hipEventCreate(&e1));
  evg.b = e1;
  evg.hb = true;
  FA_HIP(hipEventRecord(e0, x.s));
  FA_TRY(align_begin(x, X1, X2, anchors, S_out, a_out, b_out, tm));
  FA_HIP(hipEventRecord(e1, x.s));
  FA_HIP(hipEventSynchronize(e1));
  if (acc) {
    float f = 0.f;
    FA_HIP(hipEventElapsedTime(&f, e0, e1));
    const double phase_ms[4] = {f, 0.0, 0.0, 0.0};
    if (tm) tm->collect();
    stats_timing(acc, tm, phase_ms, true);
  }
  return FA_OK;
}

extern "C" int fa_align_step(const fa_csr *A1, const fa_csr *A2, int32_t d, int32_t nL, const fa_params *p,
                             const float *mlp_weights, int32_t t, void *S_out, double *a_out, double *b_out,
                             int32_t *argmax_out, const int32_t *truth, int32_t *rank_out, fa_stats *acc, void *ws,
                             size_t ws_bytes, void *stream) {
  AlignCtx x;
  FA_TRY(open_ctx(x, A1, A2, d, nL, p, ws, ws_bytes, stream));
  KTimer *tm = nullptr;
  struct TmGuard {
    KTimer *&t;
    ~TmGuard() { delete t; }
  } tmguard{tm};
  if (p->profile && acc) {
    tm = new KTimer();
    FA_REQUIRE(tm->init(), FA_ERR_HIP, "fa_align_step: could not create timing events");
  }
  double phase_ms[4] = {0, 0, 0, 0};
  FA_TRY(align_step(x, t, mlp_weights, S_out, a_out, b_out, argmax_out, truth, rank_out, tm, phase_ms));
  if (tm) tm->collect();
  if (acc) stats_timing(acc, tm, phase_ms, true);
  return FA_OK;
}

extern "C" int fa_align_end(const fa_csr *A1, const fa_csr *A2, int32_t d, int32_t nL, const fa_params *p,
                            int32_t steps, void *S_out, const double *a, const double *b, int32_t *argmax_out,
                            const int32_t *truth, int32_t *rank_out, int32_t topk, float *topk_val,
                            int32_t *topk_idx, fa_stats *stats, void *ws, size_t ws_bytes, void *stream) {
  AlignCtx x;
  FA_TRY(open_ctx(x, A1, A2, d, nL, p, ws, ws_bytes, stream));
  FA_REQUIRE(a && b, FA_ERR_ARG, "fa_align_end: null duals");
  return align_end(x, steps, S_out, a, b, argmax_out, truth, rank_out, topk, topk_val, topk_idx, stats, nullptr);
}
