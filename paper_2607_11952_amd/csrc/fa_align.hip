// Algorithm 1 end to end on one GPU.  All buffers come from the caller's
// workspace; all work is enqueued on the caller's stream.  The host synchronises
// twice: once after validating the anchors on the device, once at the end to
// return the statistics.
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
  }
  if (B) *B = b;
}

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
  FA_REQUIRE(!p->plan_in_ct || p->transpose_cost, FA_ERR_ARG, "fa_align: plan_in_ct needs transpose_cost = 1");
  return FA_OK;
}

extern "C" size_t fa_align_workspace_size(int32_t n1, int32_t n2, int32_t d, int32_t nL, int64_t nnz1, int64_t nnz2,
                                          const fa_params *p) {
  if (!p || n1 <= 0 || n2 <= 0 || d < 0 || nL < 0 || nnz1 < 0 || nnz2 < 0) return 0;
  AlignLayout L = align_layout(n1, n2, p);
  Sizer z;
  carve_align(z, n1, n2, d, nL, nnz1, nnz2, p, L, nullptr);
  z.off = align_up(z.off, 256) + sinkhorn_ws_bytes(n1, n2);
  return z.off + 256;
}

extern "C" int fa_align(const fa_csr *A1, const fa_csr *A2, const float *X1, const float *X2, int32_t d,
                        const int32_t *anchors, int32_t nL, const fa_params *p, const float *mlp_weights, void *S_out,
                        double *a_out, double *b_out, int32_t *argmax_out, const int32_t *truth,
                        int32_t *rank_out, int32_t topk, float *topk_val, int32_t *topk_idx, fa_stats *stats,
                        void *ws, size_t ws_bytes, void *stream) {
  FA_TRY(validate(A1, A2, d, nL, p));
  FA_REQUIRE((truth == nullptr) == (rank_out == nullptr), FA_ERR_ARG, "fa_align: truth and rank_out go together");
  const int32_t n1 = A1->n, n2 = A2->n;
  FA_REQUIRE((S_out || p->plan_in_ct) && a_out && b_out && argmax_out, FA_ERR_ARG, "fa_align: null output");
  FA_REQUIRE(topk == 0 || (topk >= 1 && topk <= kTopkMax && topk <= n2 && topk_val && topk_idx), FA_ERR_ARG,
             "fa_align: topk = %d needs 1 <= topk <= min(%d, n2) and both top-k outputs", topk, kTopkMax);
  FA_REQUIRE(d == 0 || (X1 && X2), FA_ERR_ARG, "fa_align: null attributes with d = %d", d);
  FA_REQUIRE(nL == 0 || anchors, FA_ERR_ARG, "fa_align: null anchors");
  FA_REQUIRE(!p->warm_start || mlp_weights, FA_ERR_ARG, "fa_align: warm_start needs mlp_weights");
  const size_t need = fa_align_workspace_size(n1, n2, d, nL, A1->nnz, A2->nnz, p);
  FA_REQUIRE(ws && ws_bytes >= need, FA_ERR_WORKSPACE, "fa_align: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  AlignLayout L = align_layout(n1, n2, p);
  Carver cv(ws, ws_bytes);
  AlignBufs B;
  carve_align(cv, n1, n2, d, nL, A1->nnz, A2->nnz, p, L, &B);
  FA_TRY(carve_sinkhorn(cv, n1, n2, B.sink));
  FA_REQUIRE(cv.ok, FA_ERR_WORKSPACE, "fa_align: workspace carve failed");
  // The working plan: the caller's S_out, or the C^T buffer (FP32 n2 x n1, at least
  // as large as an n1 x n2 plan of either type) between the plan pass and the next
  // cost rebuild.
  const bool plan_in_ct = p->plan_in_ct != 0;
  void *S_work = plan_in_ct ? static_cast<void *>(B.Ct) : S_out;
  void *S_final = S_out ? S_out : S_work;
  const int T = p->outer_iters;
  KTimer *tm = nullptr;
  struct TmGuard {
    KTimer *&t;
    ~TmGuard() { delete t; }
  } tmguard{tm};
  if (p->profile) {
    tm = new KTimer();
    FA_REQUIRE(tm->init(), FA_ERR_HIP, "fa_align: could not create timing events");
  }

  hipEvent_t ev[4];
  for (int q = 0; q < 4; ++q) FA_HIP(hipEventCreate(&ev[q]));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int q = 0; q < 4; ++q) (void)hipEventDestroy(e[q]);
    }
  } guard{ev};
  double ms_cost = 0, ms_sink = 0, ms_plan = 0, ms_p1 = 0;
  (void)ms_cost;

  // ---------------- anchors (validated on the device)
  FA_HIP(hipEventRecord(ev[0], s));
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

  // ---------------- Phase 1
  FA_TRY(launch_inv_deg(A1, B.inv1, s));
  FA_TRY(launch_inv_deg(A2, B.inv2, s));
  FA_TRY(launch_positional(A1, B.inv1, B.nodes1, nL, p->beta, p->k_r, B.R1, B.R1t, s));
  FA_TRY(launch_positional(A2, B.inv2, B.nodes2, nL, p->beta, p->k_r, B.R2, B.R2t, s));
  FA_TRY(launch_sddmm(A1, B.inv1, B.R1, nL, 0, B.w1, s));
  FA_TRY(launch_sddmm(A2, B.inv2, B.R2, nL, 1, B.w2, s));
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
  FA_TRY(run_propagate(A1, B.inv1, A2, B.inv2, B.C_node, B.C, p->k_node, L.chunk_rows, B.zt, s));

  // ---------------- initial plan S0 = mu nu^T, written as the plan of C = eps*log(n1 n2), a = b = 0
  const size_t N = static_cast<size_t>(n1) * n2;
  FA_TRY(launch_fill_f64(a_out, n2, 0.0, s));
  FA_TRY(launch_fill_f64(b_out, n1, 0.0, s));
  FA_TRY(launch_fill_f32(B.C, static_cast<int64_t>(N), static_cast<float>(p->eps * log(static_cast<double>(n1) * n2)), s));
  FA_TRY(run_plan(B.C, n1, n2, p->eps, a_out, b_out, S_work, p->plan_dtype, nullptr, nullptr, nullptr, s));
  if (p->warm_start) {
    FA_TRY(run_node_features(A1, B.inv1, X1, d, nullptr, B.nodes1, nL, B.feat, B.nf_ws, node_features_ws_bytes(n1),
                             s));
  }
  FA_HIP(hipEventRecord(ev[1], s));
  FA_HIP(hipEventSynchronize(ev[1]));
  float f = 0.f;
  FA_HIP(hipEventElapsedTime(&f, ev[0], ev[1]));
  ms_p1 = f;

  CostArgs c{A1, A2, B.w1, B.inv1, B.w2, B.inv2, S_work, p->plan_dtype, B.C_node, B.partner, a_out, b_out,
             p->lambda_e, p->lambda_n, p->lambda_a, p->lambda_p, p->eps, p->eps_anchor, p->delta_nbr, B.C,
             p->transpose_cost && !plan_in_ct ? B.Ct : nullptr};
  // Events: ev[0] start of cost, ev[1] end of cost, ev[2] end of Sinkhorn, ev[3] end of plan.
  double t_cost = 0, t_sink = 0, t_plan = 0;
  for (int t = 0; t < T; ++t) {
    FA_HIP(hipEventRecord(ev[0], s));
    FA_TRY(run_cost(c, L.chunk_rows, B.zt, s, tm));
    if (plan_in_ct) FA_TRY(run_transpose(B.C, n1, n2, B.Ct, s, tm));  // overwrites the plan just read
    FA_HIP(hipEventRecord(ev[1], s));
    if (p->warm_start && t == 0) {
      FA_TRY(warm_start_duals(mlp_weights, B.feat, n1, B.act, p->eps, B.bad + 2, b_out, s));
      FA_TRY(launch_fill_f64(a_out, n2, 0.0, s));
    } else if (t == 0 || !p->carry_duals) {
      FA_TRY(launch_fill_f64(a_out, n2, 0.0, s));
      FA_TRY(launch_fill_f64(b_out, n1, 0.0, s));
    }  // else: the previous solve's duals are the start
    int32_t *it_slot = B.st_iters + (t < 64 ? t : 63);
    double *er_slot = B.st_err + (t < 64 ? t : 63);
    FA_TRY(run_sinkhorn(B.C, p->transpose_cost ? B.Ct : nullptr, n1, n2, p->eps, a_out, b_out, p->inner_iters,
                        p->tol, p->check_every, it_slot, er_slot, B.sink, s, tm));
    FA_HIP(hipEventRecord(ev[2], s));
    FA_TRY(run_plan(B.C, n1, n2, p->eps, a_out, b_out, t == T - 1 ? S_final : S_work, p->plan_dtype,
                    t == T - 1 ? argmax_out : nullptr,
                    t == T - 1 ? truth : nullptr, t == T - 1 ? rank_out : nullptr, s,
                    tm));
    FA_HIP(hipEventRecord(ev[3], s));
    // Per-outer timing costs one event wait per outer iteration (the loop is
    // dominated by multi-millisecond passes at the sizes where timing matters).
    FA_HIP(hipEventSynchronize(ev[3]));
    float x = 0.f;
    FA_HIP(hipEventElapsedTime(&x, ev[0], ev[1]));
    t_cost += x;
    FA_HIP(hipEventElapsedTime(&x, ev[1], ev[2]));
    t_sink += x;
    FA_HIP(hipEventElapsedTime(&x, ev[2], ev[3]));
    t_plan += x;
    if (tm) tm->collect();
  }
  if (T == 0) FA_TRY(run_plan(B.C, n1, n2, p->eps, a_out, b_out, S_final, p->plan_dtype, argmax_out, truth, rank_out, s));
  if (topk > 0) FA_TRY(run_plan_topk(B.C, n1, n2, p->eps, a_out, b_out, topk, topk_val, topk_idx, s, tm));
  ms_cost = t_cost;
  ms_sink = t_sink;
  ms_plan = t_plan;

  int32_t iters[64] = {0};
  double errs[64] = {0};
  int32_t fell = 0;
  if (p->warm_start && T > 0) FA_HIP(hipMemcpyAsync(&fell, B.bad + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  const int nrec = T < 64 ? T : 64;
  if (nrec > 0) {
    FA_HIP(hipMemcpyAsync(iters, B.st_iters, sizeof(int32_t) * nrec, hipMemcpyDeviceToHost, s));
    FA_HIP(hipMemcpyAsync(errs, B.st_err, sizeof(double) * nrec, hipMemcpyDeviceToHost, s));
  }
  FA_HIP(hipStreamSynchronize(s));
  if (tm) tm->collect();  // launches after the last outer iteration (top-k; all of them if T = 0)
  bool all_conv = true;
  int32_t total = 0;
  for (int t = 0; t < nrec; ++t) {
    total += iters[t];
    if (!(errs[t] <= p->tol)) all_conv = false;
    if (!isfinite(errs[t])) {
      set_error("fa_align: non-finite marginal error at outer iteration %d", t);
      return FA_ERR_NUMERIC;
    }
  }
  if (stats) {
    memset(stats, 0, sizeof *stats);
    stats->outer_done = T;
    stats->inner_total = total;
    stats->fell_back = fell != 0 ? 1 : 0;
    stats->converged_all = all_conv ? 1 : 0;
    stats->marg_err = nrec > 0 ? errs[nrec - 1] : 0.0;
    stats->phase_ms[0] = ms_p1;
    stats->phase_ms[1] = ms_cost;
    stats->phase_ms[2] = ms_sink;
    stats->phase_ms[3] = ms_plan;
    for (int t = 0; t < nrec; ++t) {
      stats->inner_iters[t] = iters[t];
      stats->inner_err[t] = errs[t];
    }
    if (tm)
      for (int k = 0; k < KK_COUNT; ++k) {
        stats->kernel_ms[k] = tm->ms[k];
        stats->kernel_calls[k] = tm->calls[k];
      }
  }
  if (p->tol > 0 && !all_conv) return FA_WARN_NOT_CONVERGED;
  return FA_OK;
}
