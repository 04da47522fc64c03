// Phase 2 of Algorithm 1: the S-dependent cost terms as two SpMMs per triple
// product (§3.3), fused with the cost assembly of Eq. (2) (§3.5).
//
//   Z_e = C1 S,  Z_n = Abar1^T S             stage 1: each output row gathers whole
//                                            row segments of S (left SpMM)
//   E   = Z_e C2^T,  P = Z_n Abar2           stage 2: each output column j gathers
//                                            columns l in N2(j) of Z (right SpMM)
//   C  <- C_node + le*E - ln*log(P + delta) + la*C_anc - lp*(a_j + b_i - C_prev)/eps
//
// Both stages read contiguous multi-hundred-byte segments: stage 1 writes Z in a
// block-transposed layout Zt[block][l][r] (64 rows r of a row block stored
// contiguously per column l), so stage 2's gather of column l of a row block is
// one 256-byte (FP32) or 128-byte (BF16) segment.  Neighbour lists are uniform
// per wavefront (one output row or column per wave), so indices and weights come
// through the scalar cache and no lane diverges on the power-law degrees.
#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

size_t zt_bytes(int32_t chunk_rows, int32_t n2, int32_t zdt) {
  const size_t nblk = (static_cast<size_t>(chunk_rows) + kZtRows - 1) / kZtRows;
  const size_t el = zdt == FA_BF16 ? 2 : 4;
  return 2 * align_up(nblk * kZtRows * static_cast<size_t>(n2) * el, 256);
}

template <typename T>
__device__ inline void store16(T *dst, const float *v);
template <>
__device__ inline void store16<float>(float *dst, const float *v) {
  float4 *d = reinterpret_cast<float4 *>(dst);
#pragma unroll
  for (int q = 0; q < 4; ++q) d[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}
template <>
__device__ inline void store16<uint16_t>(uint16_t *dst, const float *v) {
  uint4 *d = reinterpret_cast<uint4 *>(dst);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      w[t] = static_cast<uint32_t>(f32_to_bf16(v[8 * q + 2 * t])) |
             (static_cast<uint32_t>(f32_to_bf16(v[8 * q + 2 * t + 1])) << 16);
    d[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// Stage 1 (left SpMM into the block-transposed layout).
//   grid.x = row block within the chunk, grid.y = 128-column tile; 4 waves, wave
//   w owns rows 16w..16w+15 of the block, lane owns columns c0+lane, c0+64+lane.
//   Set a: Za[i,:] = rsa[i] * sum_e wa[e] S[col[e],:]          (wa/rsa may be null = 1)
//   Set b: Zb[i,:] = sum_e csb[col[e]] S[col[e],:]            (only when TWO)
template <typename TS, typename TZ, bool TWO>
__global__ __launch_bounds__(256) void k_stage1(const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col,
                                                const float *__restrict__ wa, const float *__restrict__ rsa,
                                                const float *__restrict__ csb,
                                                const TS *__restrict__ S, int32_t n2, int32_t row0,
                                                int32_t nrows, TZ *__restrict__ Za, TZ *__restrict__ Zb) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = blockIdx.x;
  const int c0 = blockIdx.y * 128;
  const int ca = c0 + lane, cb = c0 + 64 + lane;
  const bool va = ca < n2, vb = cb < n2;
  float za[16][2], zb[16][2];
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    const int rloc = blk * kZtRows + w * 16 + rr;
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
    if (rloc < nrows) {
      const int i = row0 + rloc;
      const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
      int64_t e = e0;
      for (; e + 4 <= e1; e += 4) {
        float s0[4], s1[4], fa_[4], fb_[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const TS *row = S + static_cast<int64_t>(col[e + u]) * n2;
          s0[u] = va ? load_as_f32<TS>(row, ca) : 0.f;
          s1[u] = vb ? load_as_f32<TS>(row, cb) : 0.f;
          fa_[u] = wa ? wa[e + u] : 1.f;
          if (TWO) fb_[u] = csb[col[e + u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a0 += fa_[u] * s0[u];
          a1 += fa_[u] * s1[u];
          if (TWO) {
            b0 += fb_[u] * s0[u];
            b1 += fb_[u] * s1[u];
          }
        }
      }
      for (; e < e1; ++e) {
        const TS *row = S + static_cast<int64_t>(col[e]) * n2;
        const float s0 = va ? load_as_f32<TS>(row, ca) : 0.f;
        const float s1 = vb ? load_as_f32<TS>(row, cb) : 0.f;
        const float f = wa ? wa[e] : 1.f;
        a0 += f * s0;
        a1 += f * s1;
        if (TWO) {
          const float g = csb[col[e]];
          b0 += g * s0;
          b1 += g * s1;
        }
      }
      if (rsa) {
        const float r = rsa[i];
        a0 *= r;
        a1 *= r;
      }
    }
    za[rr][0] = a0;
    za[rr][1] = a1;
    zb[rr][0] = b0;
    zb[rr][1] = b1;
  }
  // Each lane writes 16 consecutive rows of its two columns.
  const int64_t base = static_cast<int64_t>(blk) * n2;
  float v[16];
  if (va) {
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) v[rr] = za[rr][0];
    store16<TZ>(Za + (base + ca) * kZtRows + w * 16, v);
    if (TWO) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) v[rr] = zb[rr][0];
      store16<TZ>(Zb + (base + ca) * kZtRows + w * 16, v);
    }
  }
  if (vb) {
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) v[rr] = za[rr][1];
    store16<TZ>(Za + (base + cb) * kZtRows + w * 16, v);
    if (TWO) {
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) v[rr] = zb[rr][1];
      store16<TZ>(Zb + (base + cb) * kZtRows + w * 16, v);
    }
  }
}

struct CostCoef {
  double le, ln, la, kp;     // lambda_e, lambda_n, lambda_a, lambda_p/eps
  double anc_on, anc_off;    // -log(1 + eps_a), -log(eps_a)
  double delta;
};

// Natural log of a positive float with an absolute error of a few 1e-8: the
// binary exponent enters exactly, only the mantissa in [0.5, 1) goes through logf.
__device__ inline double log_accurate(float x) {
  int e;
  const float m = frexpf(x, &e);
  return static_cast<double>(logf(m)) + static_cast<double>(e) * kLn2;
}

// Stage 2 (right SpMM from the block-transposed layout) with a fused epilogue.
//   grid.x = 64-column output tile, grid.y = row block; wave w owns output
//   columns j0+16w..j0+16w+15, lane = row of the block.
//   COST:  C[i,j] <- C_node + le*E - ln*log(P+delta) + la*C_anc + kp*(C_prev - a_j - b_i)
//          with E = sum_e w2a[e] Za[:,col e], P = sum_e cs2b[col e] Zb[:,col e]
//          (E, P accumulated in FP64; the tile of results is kept in FP64 until the
//          epilogue rounds the assembled cost once)
//   PLAIN: out[i,j] = rs[j] * sum_e Za[:,col e]
template <typename TZ, bool COST>
__global__ __launch_bounds__(256) void k_stage2(const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col,
                                                const float *__restrict__ w2a, const float *__restrict__ cs2b,
                                                const float *__restrict__ rs, const TZ *__restrict__ Za,
                                                const TZ *__restrict__ Zb, int32_t n2, int32_t row0,
                                                int32_t nrows, const float *__restrict__ C_node,
                                                const int32_t *__restrict__ partner,
                                                const double *__restrict__ a, const double *__restrict__ b,
                                                CostCoef cf, float *__restrict__ out) {
  __shared__ double tile[kZtRows][65];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j0 = blockIdx.x * 64;
  const int blk = blockIdx.y;
  const TZ *za = Za + static_cast<int64_t>(blk) * n2 * kZtRows + lane;
  const TZ *zb = COST ? Zb + static_cast<int64_t>(blk) * n2 * kZtRows + lane : nullptr;
  for (int jj = 0; jj < 16; ++jj) {
    const int j = j0 + w * 16 + jj;
    double g = 0.0;
    if (j < n2) {
      const int64_t e0 = rowptr[j], e1 = rowptr[j + 1];
      double E = 0.0, P = 0.0;
      int64_t e = e0;
      for (; e + 4 <= e1; e += 4) {
        float x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t l = col[e + u];
          x[u] = load_as_f32<TZ>(za, l * kZtRows);
          if (COST) y[u] = cs2b[l] * load_as_f32<TZ>(zb, l * kZtRows);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (COST) {
            E = fma(static_cast<double>(w2a[e + u]), static_cast<double>(x[u]), E);
            P += static_cast<double>(y[u]);
          } else {
            E += static_cast<double>(x[u]);
          }
        }
      }
      for (; e < e1; ++e) {
        const int64_t l = col[e];
        const float x = load_as_f32<TZ>(za, l * kZtRows);
        if (COST) {
          E = fma(static_cast<double>(w2a[e]), static_cast<double>(x), E);
          P += static_cast<double>(cs2b[l] * load_as_f32<TZ>(zb, l * kZtRows));
        } else {
          E += static_cast<double>(x);
        }
      }
      if (COST)
        g = cf.le * E - cf.ln * log_accurate(static_cast<float>(P + cf.delta));
      else
        g = static_cast<double>(rs[j]) * E;
    }
    tile[lane][w * 16 + jj] = g;
  }
  __syncthreads();
  const int j = j0 + lane;
  if (j >= n2) return;
  const double aj = COST ? a[j] : 0.0;
  for (int rr = 0; rr < 16; ++rr) {
    const int r = w * 16 + rr;
    const int rloc = blk * kZtRows + r;
    if (rloc >= nrows) break;
    const int i = row0 + rloc;
    const int64_t idx = static_cast<int64_t>(i) * n2 + j;
    const double g = tile[r][lane];
    if (COST) {
      const double anc = partner[i] == j ? cf.anc_on : cf.anc_off;
      const double v = static_cast<double>(C_node[idx]) + g + cf.la * anc +
                       cf.kp * (static_cast<double>(out[idx]) - aj - b[i]);
      out[idx] = static_cast<float>(v);
    } else {
      out[idx] = static_cast<float>(g);
    }
  }
}

template <typename TS, typename TZ>
static int cost_chunks(const CostArgs &c, int32_t chunk_rows, void *zt, hipStream_t s, KTimer *tm) {
  const int32_t n1 = c.A1->n, n2 = c.A2->n;
  const size_t nblk_max = (static_cast<size_t>(chunk_rows) + kZtRows - 1) / kZtRows;
  TZ *Za = static_cast<TZ *>(zt);
  TZ *Zb = reinterpret_cast<TZ *>(static_cast<char *>(zt) +
                                  align_up(nblk_max * kZtRows * static_cast<size_t>(n2) * sizeof(TZ), 256));
  CostCoef cf;
  cf.le = c.lambda_e;
  cf.ln = c.lambda_n;
  cf.la = c.lambda_a;
  cf.kp = c.lambda_p / c.eps;
  cf.anc_on = -log(1.0 + c.eps_anchor);
  cf.anc_off = -log(c.eps_anchor);
  cf.delta = c.delta;
  for (int32_t r0 = 0; r0 < n1; r0 += chunk_rows) {
    const int32_t nr = n1 - r0 < chunk_rows ? n1 - r0 : chunk_rows;
    const int nblk = ceil_div(nr, kZtRows);
    FA_TIMED(tm, KK_STAGE1, s,
             FA_LAUNCH((k_stage1<TS, TZ, true>), dim3(nblk, ceil_div(n2, 128)), dim3(256), 0, s, c.A1->rowptr,
                       c.A1->colidx, c.w1, nullptr, c.inv1, static_cast<const TS *>(c.S), n2, r0, nr, Za, Zb));
    FA_TIMED(tm, KK_STAGE2, s,
             FA_LAUNCH((k_stage2<TZ, true>), dim3(ceil_div(n2, 64), nblk), dim3(256), 0, s, c.A2->rowptr,
                       c.A2->colidx, c.w2, c.inv2, nullptr, Za, Zb, n2, r0, nr, c.C_node, c.partner, c.a, c.b, cf,
                       c.C));
  }
  return FA_OK;
}

int run_cost(const CostArgs &c, int32_t chunk_rows, int32_t zdt, void *zt, hipStream_t s, KTimer *tm) {
  if (c.A1->n == 0 || c.A2->n == 0) return FA_OK;
  if (c.s_dtype == FA_BF16) {
    if (zdt == FA_BF16) return cost_chunks<uint16_t, uint16_t>(c, chunk_rows, zt, s, tm);
    return cost_chunks<uint16_t, float>(c, chunk_rows, zt, s, tm);
  }
  if (zdt == FA_BF16) return cost_chunks<float, uint16_t>(c, chunk_rows, zt, s, tm);
  return cost_chunks<float, float>(c, chunk_rows, zt, s, tm);
}

// k times C <- Abar1 C Abar2^T.  Stage 1 reads every row of C, so each step
// writes into C_tmp and the two buffers swap; the result ends in C.
int run_propagate(const fa_csr *A1, const float *inv1, const fa_csr *A2, const float *inv2, float *C,
                  float *C_tmp, int32_t k, int32_t chunk_rows, void *zt, hipStream_t s) {
  const int32_t n1 = A1->n, n2 = A2->n;
  if (n1 == 0 || n2 == 0 || k == 0) return FA_OK;
  float *src = C, *dst = C_tmp;
  float *Z = static_cast<float *>(zt);
  CostCoef cf{};
  for (int it = 0; it < k; ++it) {
    for (int32_t r0 = 0; r0 < n1; r0 += chunk_rows) {
      const int32_t nr = n1 - r0 < chunk_rows ? n1 - r0 : chunk_rows;
      const int nblk = ceil_div(nr, kZtRows);
      FA_LAUNCH((k_stage1<float, float, false>), dim3(nblk, ceil_div(n2, 128)), dim3(256), 0, s, A1->rowptr,
                A1->colidx, nullptr, inv1, nullptr, src, n2, r0, nr, Z, nullptr);
      FA_LAUNCH((k_stage2<float, false>), dim3(ceil_div(n2, 64), nblk), dim3(256), 0, s, A2->rowptr,
                A2->colidx, nullptr, nullptr, inv2, Z, nullptr, n2, r0, nr, nullptr, nullptr, nullptr,
                nullptr, cf, dst);
    }
    float *t = src;
    src = dst;
    dst = t;
  }
  if (src != C) FA_HIP(hipMemcpyAsync(C, src, sizeof(float) * n1 * n2, hipMemcpyDeviceToDevice, s));
  return FA_OK;
}

}  // namespace fa

using namespace fa;

static int resolve_chunk(int32_t n1, int32_t chunk_rows) {
  if (chunk_rows <= 0 || chunk_rows > n1) chunk_rows = n1;
  return chunk_rows < 1 ? 1 : chunk_rows;
}

extern "C" size_t fa_cost_workspace_size(int32_t n1, int32_t n2, int32_t plan_dtype, int32_t chunk_rows) {
  if (n1 <= 0 || n2 <= 0) return 0;
  return zt_bytes(resolve_chunk(n1, chunk_rows), n2, plan_dtype == FA_BF16 ? FA_BF16 : FA_F32);
}

extern "C" int fa_propagate(const fa_csr *A1, const float *inv_deg1, const fa_csr *A2, const float *inv_deg2,
                            float *C, float *C_tmp, int32_t k, int32_t chunk_rows, void *ws, size_t ws_bytes,
                            void *stream) {
  FA_TRY(check_csr(A1, "fa_propagate A1"));
  FA_TRY(check_csr(A2, "fa_propagate A2"));
  FA_REQUIRE(k >= 0, FA_ERR_ARG, "fa_propagate: k < 0");
  const int32_t n1 = A1->n, n2 = A2->n;
  if (n1 == 0 || n2 == 0 || k == 0) return FA_OK;
  FA_REQUIRE(C && C_tmp && inv_deg1 && inv_deg2, FA_ERR_ARG, "fa_propagate: null pointer");
  const int32_t cr = resolve_chunk(n1, chunk_rows);
  FA_REQUIRE(ws && ws_bytes >= zt_bytes(cr, n2, FA_F32), FA_ERR_WORKSPACE,
             "fa_propagate: workspace %zu < %zu bytes", ws_bytes, zt_bytes(cr, n2, FA_F32));
  return run_propagate(A1, inv_deg1, A2, inv_deg2, C, C_tmp, k, cr, ws, static_cast<hipStream_t>(stream));
}

extern "C" int fa_cost(const fa_csr *A1, const fa_csr *A2, const float *w1, const float *w2, const float *inv_deg1,
                       const float *inv_deg2, const void *S, int32_t s_dtype, const float *C_node,
                       const int32_t *partner, const double *a, const double *b, const fa_params *p,
                       float *C_inout, void *ws, size_t ws_bytes, void *stream) {
  FA_TRY(check_csr(A1, "fa_cost A1"));
  FA_TRY(check_csr(A2, "fa_cost A2"));
  FA_REQUIRE(p, FA_ERR_ARG, "fa_cost: null params");
  FA_REQUIRE(s_dtype == FA_F32 || s_dtype == FA_BF16, FA_ERR_ARG, "fa_cost: s_dtype %d", s_dtype);
  FA_REQUIRE(p->eps > 0 && p->eps_anchor > 0 && p->delta_nbr >= 0, FA_ERR_ARG, "fa_cost: eps, eps_anchor must be > 0");
  const int32_t n1 = A1->n, n2 = A2->n;
  if (n1 == 0 || n2 == 0) return FA_OK;
  FA_REQUIRE(S && C_node && partner && a && b && C_inout && inv_deg1 && inv_deg2, FA_ERR_ARG, "fa_cost: null pointer");
  FA_REQUIRE((A1->nnz == 0 || w1) && (A2->nnz == 0 || w2), FA_ERR_ARG, "fa_cost: null C1/C2 values");
  const int32_t cr = resolve_chunk(n1, p->chunk_rows);
  const size_t need = zt_bytes(cr, n2, s_dtype);
  FA_REQUIRE(ws && ws_bytes >= need, FA_ERR_WORKSPACE, "fa_cost: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  CostArgs c{A1, A2, w1, inv_deg1, w2, inv_deg2, S, s_dtype, C_node, partner, a, b,
             p->lambda_e, p->lambda_n, p->lambda_a, p->lambda_p, p->eps, p->eps_anchor, p->delta_nbr, C_inout};
  return run_cost(c, cr, s_dtype, ws, s);
}
