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
// block-transposed layout Zt[block][l][set][r] (64 rows r of a row block stored
// contiguously per column l, the two value sets side by side), so stage 2's
// gather of column l of a row block is one 512-byte piece.  The N-set is FP32 in
// both precision forms (log P needs it near P = 0); the BF16 form stores the
// E-set in BF16 (a 384-byte piece), which cuts stage 2's gather traffic, the
// fabric behind L2 that bounds it, by a quarter at a relative error of 2^-8 per
// entry of Z_e (stage 2 accumulates in FP64).  Neighbour lists are uniform per
// wavefront (one output row or column per wave), fetched 64 at a time with one
// coalesced load and broadcast lane by lane, so no lane diverges on the power-law
// degrees.  With a C^T buffer, stage 2 also writes the transposed cost for the
// Sinkhorn column pass.
#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

size_t zt_bytes(int32_t chunk_rows, int32_t n2) {
  const size_t nblk = (static_cast<size_t>(chunk_rows) + kZtRows - 1) / kZtRows;
  return 2 * align_up(nblk * kZtRows * static_cast<size_t>(n2) * sizeof(float), 256);
}

// Vector loads of VW consecutive elements (aligned: the row length is a multiple
// of VW whenever VW > 1) converted to FP32.
template <typename T, int VW>
struct VLoad;
template <>
struct VLoad<float, 1> {
  static __device__ inline void run(const float *p, float *o) { o[0] = p[0]; }
};
template <>
struct VLoad<float, 2> {
  static __device__ inline void run(const float *p, float *o) {
    const float2 t = *reinterpret_cast<const float2 *>(p);
    o[0] = t.x;
    o[1] = t.y;
  }
};
template <>
struct VLoad<uint16_t, 1> {
  static __device__ inline void run(const uint16_t *p, float *o) { o[0] = bf16_to_f32(p[0]); }
};
template <>
struct VLoad<uint16_t, 2> {
  static __device__ inline void run(const uint16_t *p, float *o) {
    const uint32_t t = *reinterpret_cast<const uint32_t *>(p);
    o[0] = __uint_as_float(t << 16);
    o[1] = __uint_as_float(t & 0xffff0000u);
  }
};

__device__ inline int bcast_i(int v, int u) { return __builtin_amdgcn_readlane(v, u); }
__device__ inline float bcast_f(float v, int u) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), u)); }

// Record of one (row block, column) in Zt, in floats: the 64 rows of each value
// set.  Both sets FP32: [E-set | N-set], 512 bytes.  With ZEB (the BF16 form) the
// E-set is stored in BF16 after the FP32 N-set: [N-set 256 B | E-set 128 B].
// One set (propagation): 64 floats.
template <bool TWO, bool ZEB>
__host__ __device__ constexpr int zt_record() {
  return TWO ? (ZEB ? 96 : 128) : 64;
}
// Offset in floats of a set's rows inside the record (set 0 = E-set, set 1 = N-set).
template <bool TWO, bool ZEB>
__device__ constexpr int zt_offset(int set) {
  return !TWO ? 0 : (ZEB ? (set == 0 ? 64 : 0) : set * 64);
}
__device__ inline uint32_t pack_bf16(float x, float y) {
  return static_cast<uint32_t>(f32_to_bf16(x)) | (static_cast<uint32_t>(f32_to_bf16(y)) << 16);
}

// Gathers kept in flight per wave: stage 1 (row segments of S), stage 2 (Zt
// column segments, per value set).  Both divide the 64-entry neighbour chunks.
constexpr int kUnroll1 = 8;
constexpr int kUnroll2 = 8;

// Stage 1 (left SpMM into the block-transposed layout).
//   grid.x = row block within the chunk, grid.y = column tile of 64*VW columns;
//   64/RW waves, wave w owns rows RW*w..RW*w+RW-1 of the block, lane owns VW consecutive
//   columns and reads them with one vector load per gathered row segment.  A
//   row's neighbour list is fetched 64 entries at a time with one coalesced load
//   and broadcast lane by lane (readlane), so gathers never wait on index loads.
//   Set 0: Z[i,:] = rsa[i] * sum_e wa[e] S[col[e],:]           (wa/rsa may be null = 1)
//   Set 1: Z[i,:] = sum_e csb[col[e]] S[col[e],:]             (only when TWO)
template <typename TS, bool TWO, int VW, int RW, bool ZEB>
__global__ __launch_bounds__(64 * 64 / RW) void k_stage1(const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col,
                                                const float *__restrict__ wa, const float *__restrict__ rsa,
                                                const float *__restrict__ csb,
                                                const TS *__restrict__ S, int32_t n2, int32_t row0,
                                                int32_t nrows, float *__restrict__ Z) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = blockIdx.x;
  const int c = blockIdx.y * (64 * VW) + lane * VW;
  // Lanes past the last column read column 0 instead (always in bounds) and their
  // sums are never stored, so the gathers need no per-lane branch: a branch around
  // each load would make the wave wait for it before the next one issues.
  const TS *Sc = S + (c < n2 ? c : 0);
  float za[RW][VW], zb[RW][VW];
#pragma unroll
  for (int rr = 0; rr < RW; ++rr) {
    const int rloc = blk * kZtRows + w * RW + rr;
    float a[VW], b[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) a[v] = b[v] = 0.f;
    if (rloc < nrows) {
      const int i = row0 + rloc;
      const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
      for (int64_t base = e0; base < e1; base += 64) {
        const int cnt = static_cast<int>(min<int64_t>(64, e1 - base));
        int my_k = 0;
        float my_a = 0.f, my_b = 0.f;
        if (lane < cnt) {
          my_k = col[base + lane];
          my_a = wa ? wa[base + lane] : 1.f;
          if (TWO) my_b = csb[my_k];
        }
        // Whole groups of kUnroll1 even past cnt: lanes >= cnt hold index 0 and zero
        // weights, so the extra gathers re-read one hot row and add nothing, and a
        // row of degree d costs ceil(d / kUnroll1) round trips instead of a serial tail.
        for (int u = 0; u < cnt; u += kUnroll1) {
          float sv[kUnroll1][VW];
#pragma unroll
          for (int q = 0; q < kUnroll1; ++q) {
            const int k = bcast_i(my_k, u + q);
            VLoad<TS, VW>::run(Sc + static_cast<int64_t>(k) * n2, sv[q]);
          }
#pragma unroll
          for (int q = 0; q < kUnroll1; ++q) {
            const float fa = bcast_f(my_a, u + q);
            const float fb = TWO ? bcast_f(my_b, u + q) : 0.f;
#pragma unroll
            for (int v = 0; v < VW; ++v) {
              a[v] += fa * sv[q][v];
              if (TWO) b[v] += fb * sv[q][v];
            }
          }
        }
      }
      if (rsa) {
        const float r = rsa[i];
#pragma unroll
        for (int v = 0; v < VW; ++v) a[v] *= r;
      }
    }
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      za[rr][v] = a[v];
      zb[rr][v] = b[v];
    }
  }
  // Write the 64-row block transposed through LDS so that every 64-row column
  // segment leaves as whole 128-byte lines.  The buffer holds NL columns; with
  // VW = 4 the lanes take two turns (lanes 0-31, then 32-63), which keeps the
  // buffer at 34 KB and four workgroups per CU resident.
  constexpr int NL = VW >= 2 ? 128 : 64;            // columns staged per turn
  constexpr int LP = NL / VW;                       // lanes per turn
  constexpr int LS = kZtRows + 4;                   // padded column stride keeps float4 alignment
  __shared__ float lds[NL * LS];
  const int ct = blockIdx.y * (64 * VW);
  constexpr int REC = zt_record<TWO, ZEB>();  // floats per (block, column) record
  const int64_t base = static_cast<int64_t>(blk) * n2;
#pragma unroll
  for (int set = 0; set < (TWO ? 2 : 1); ++set) {
#pragma unroll
    for (int turn = 0; turn < 64 / LP; ++turn) {
      __syncthreads();
      if (lane / LP == turn) {
        const int lc = (lane % LP) * VW;
#pragma unroll
        for (int v = 0; v < VW; ++v)
#pragma unroll
          for (int rr = 0; rr < RW; ++rr) lds[(lc + v) * LS + w * RW + rr] = set ? zb[rr][v] : za[rr][v];
      }
      __syncthreads();
      const int c0 = ct + turn * NL;
      if (ZEB && set == 0) {
        // the E-set in BF16: eight rows per 16-byte piece, after the FP32 N-set
        for (int q = threadIdx.x; q < NL * (kZtRows / 8); q += blockDim.x) {
          const int cl = q / (kZtRows / 8), part = q % (kZtRows / 8);
          if (c0 + cl < n2) {
            const float4 lo = *reinterpret_cast<const float4 *>(&lds[cl * LS + part * 8]);
            const float4 hi = *reinterpret_cast<const float4 *>(&lds[cl * LS + part * 8 + 4]);
            const uint4 pk = make_uint4(pack_bf16(lo.x, lo.y), pack_bf16(lo.z, lo.w), pack_bf16(hi.x, hi.y),
                                        pack_bf16(hi.z, hi.w));
            *reinterpret_cast<uint4 *>(Z + (base + c0 + cl) * REC + zt_offset<TWO, ZEB>(0) + part * 4) = pk;
          }
        }
      } else {
        for (int q = threadIdx.x; q < NL * (kZtRows / 4); q += blockDim.x) {
          const int cl = q / (kZtRows / 4), part = q % (kZtRows / 4);
          if (c0 + cl < n2) {
            const float4 val = *reinterpret_cast<const float4 *>(&lds[cl * LS + part * 4]);
            *reinterpret_cast<float4 *>(Z + (base + c0 + cl) * REC + zt_offset<TWO, ZEB>(set) + part * 4) = val;
          }
        }
      }
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
//   grid.x = 64-column output tile, grid.y = row block; 8 waves, wave w owns
//   output columns j0+8w..j0+8w+7, lane = row of the block.
//   COST:  C[i,j] <- C_node + le*E - ln*log(P+delta) + la*C_anc + kp*(C_prev - a_j - b_i)
//          with E = sum_e w2a[e] Z[set 0][:,col e], P = sum_e cs2b[col e] Z[set 1][:,col e]
//          (E, P accumulated in FP64; the tile of results is kept in FP64 until the
//          epilogue rounds the assembled cost once)
//   PLAIN: out[i,j] = rs[j] * sum_e Z[:,col e]
template <bool COST, bool ZEB>
__global__ __launch_bounds__(512) void k_stage2(const int64_t *__restrict__ rowptr,
                                                const int32_t *__restrict__ col,
                                                const float *__restrict__ w2a, const float *__restrict__ cs2b,
                                                const float *__restrict__ rs, const float *__restrict__ Z,
                                                int32_t n2, int32_t row0,
                                                int32_t nrows, const float *__restrict__ C_node,
                                                const int32_t *__restrict__ partner,
                                                const double *__restrict__ a, const double *__restrict__ b,
                                                CostCoef cf, float *__restrict__ out, float *__restrict__ outT,
                                                int32_t n1t) {
  __shared__ double tile[kZtRows][65];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j0 = blockIdx.x * 64;
  const int blk = blockIdx.y;
  // both value sets of column l of the block sit in one record (384 or 512 bytes)
  constexpr int REC = zt_record<COST, ZEB>();
  const float *zr = Z + static_cast<int64_t>(blk) * n2 * REC;
  for (int jj = 0; jj < 8; ++jj) {
    const int j = j0 + w * 8 + jj;
    double E = 0.0, P = 0.0;
    if (j < n2) {
      const int64_t e0 = rowptr[j], e1 = rowptr[j + 1];
      for (int64_t base = e0; base < e1; base += 64) {
        const int cnt = static_cast<int>(min<int64_t>(64, e1 - base));
        int my_l = 0;
        float my_w = 0.f, my_c = 0.f;
        if (lane < cnt) {
          my_l = col[base + lane];
          my_w = COST ? w2a[base + lane] : 1.f;
          if (COST) my_c = cs2b[my_l];
        }
        // Whole groups of kUnroll2 (lanes >= cnt hold column 0 and zero weights):
        // 2 kUnroll2 gathers in flight per wave and no serial tail.
        for (int u = 0; u < cnt; u += kUnroll2) {
          float x[kUnroll2], y[kUnroll2];
#pragma unroll
          for (int t = 0; t < kUnroll2; ++t) {
            const float *rec = zr + static_cast<int64_t>(bcast_i(my_l, u + t)) * REC;
            if (ZEB)
              x[t] = bf16_to_f32(reinterpret_cast<const uint16_t *>(rec + zt_offset<COST, ZEB>(0))[lane]);
            else
              x[t] = rec[zt_offset<COST, ZEB>(0) + lane];
            if (COST) y[t] = rec[zt_offset<COST, ZEB>(1) + lane];
          }
#pragma unroll
          for (int t = 0; t < kUnroll2; ++t) {
            E = fma(static_cast<double>(bcast_f(my_w, u + t)), static_cast<double>(x[t]), E);
            if (COST) P = fma(static_cast<double>(bcast_f(my_c, u + t)), static_cast<double>(y[t]), P);
          }
        }
      }
    }
    double g = 0.0;
    if (j < n2) {
      if (COST)
        g = cf.le * E - cf.ln * log_accurate(static_cast<float>(P + cf.delta));
      else
        g = static_cast<double>(rs[j]) * E;
    }
    tile[lane][w * 8 + jj] = g;
  }
  __syncthreads();
  const int j = j0 + lane;
  float vt[8];
  if (j < n2) {
    const double aj = COST ? a[j] : 0.0;
    for (int rr = 0; rr < 8; ++rr) {
      const int r = w * 8 + rr;
      const int rloc = blk * kZtRows + r;
      if (rloc >= nrows) break;
      const int i = row0 + rloc;
      const int64_t idx = static_cast<int64_t>(i) * n2 + j;
      const double g = tile[r][lane];
      if (COST) {
        const double anc = partner[i] == j ? cf.anc_on : cf.anc_off;
        const double v = static_cast<double>(ld_stream(C_node + idx)) + g + cf.la * anc +
                         cf.kp * (static_cast<double>(ld_stream(out + idx)) - aj - b[i]);
        vt[rr] = static_cast<float>(v);
        st_stream(out + idx, vt[rr]);
      } else {
        st_stream(out + idx, static_cast<float>(g));
      }
    }
  }
  if (!COST || outT == nullptr) return;
  // C^T: the assembled tile goes through LDS (reusing the FP64 tile's storage once
  // every thread has read its entries) so that column j0+c of the tile leaves as 64
  // consecutive floats of row j0+c of C^T.
  __syncthreads();
  float(*tt)[65] = reinterpret_cast<float(*)[65]>(&tile[0][0]);
  if (j < n2)
    for (int rr = 0; rr < 8 && blk * kZtRows + w * 8 + rr < nrows; ++rr) tt[w * 8 + rr][lane] = vt[rr];
  __syncthreads();
  const int i0 = row0 + blk * kZtRows;
  for (int cc = 0; cc < 8; ++cc) {
    const int c = w * 8 + cc;
    if (j0 + c < n2 && blk * kZtRows + lane < nrows)
      st_stream(outT + static_cast<int64_t>(j0 + c) * n1t + i0 + lane, tt[lane][c]);
  }
}

template <typename TS>
static int cost_chunks(const CostArgs &c, int32_t chunk_rows, void *zt, hipStream_t s, KTimer *tm) {
  const int32_t n1 = c.A1->n, n2 = c.A2->n;
  float *Z = static_cast<float *>(zt);
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
    // two columns per lane (8-byte FP32 or 4-byte BF16 loads), eight rows per wave:
    // 32 accumulators and eight gathers in flight per wave at full occupancy
    constexpr int VW = 2, RW = 8;
    constexpr bool ZEB = sizeof(TS) == 2;  // the BF16 form keeps the E-set of the intermediate in BF16
    if (n2 % VW == 0)
      FA_TIMED(tm, KK_STAGE1, s,
               FA_LAUNCH((k_stage1<TS, true, VW, RW, ZEB>), dim3(nblk, ceil_div(n2, 64 * VW)), dim3(64 * 64 / RW), 0, s,
                         c.A1->rowptr, c.A1->colidx, c.w1, nullptr, c.inv1, static_cast<const TS *>(c.S), n2, r0, nr,
                         Z));
    else
      FA_TIMED(tm, KK_STAGE1, s,
               FA_LAUNCH((k_stage1<TS, true, 1, 8, ZEB>), dim3(nblk, ceil_div(n2, 64)), dim3(512), 0, s, c.A1->rowptr,
                         c.A1->colidx, c.w1, nullptr, c.inv1, static_cast<const TS *>(c.S), n2, r0, nr, Z));
    FA_TIMED(tm, KK_STAGE2, s,
             FA_LAUNCH((k_stage2<true, ZEB>), dim3(ceil_div(n2, 64), nblk), dim3(512), 0, s, c.A2->rowptr,
                       c.A2->colidx, c.w2, c.inv2, nullptr, Z, n2, r0, nr, c.C_node, c.partner, c.a, c.b, cf,
                       c.C, c.Ct, n1));
  }
  return FA_OK;
}

int run_cost(const CostArgs &c, int32_t chunk_rows, void *zt, hipStream_t s, KTimer *tm) {
  if (c.A1->n == 0 || c.A2->n == 0) return FA_OK;
  if (c.s_dtype == FA_BF16) return cost_chunks<uint16_t>(c, chunk_rows, zt, s, tm);
  return cost_chunks<float>(c, chunk_rows, zt, s, tm);
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
      if (n2 % 2 == 0)
        FA_LAUNCH((k_stage1<float, false, 2, 8, false>), dim3(nblk, ceil_div(n2, 128)), dim3(512), 0, s, A1->rowptr,
                  A1->colidx, nullptr, inv1, nullptr, src, n2, r0, nr, Z);
      else
        FA_LAUNCH((k_stage1<float, false, 1, 8, false>), dim3(nblk, ceil_div(n2, 64)), dim3(512), 0, s, A1->rowptr,
                  A1->colidx, nullptr, inv1, nullptr, src, n2, r0, nr, Z);
      FA_LAUNCH((k_stage2<false, false>), dim3(ceil_div(n2, 64), nblk), dim3(512), 0, s, A2->rowptr,
                A2->colidx, nullptr, nullptr, inv2, Z, n2, r0, nr, nullptr, nullptr, nullptr,
                nullptr, cf, dst, nullptr, n1);
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
  (void)plan_dtype;  // the intermediate is FP32 in both forms
  return zt_bytes(resolve_chunk(n1, chunk_rows), n2);
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
  FA_REQUIRE(ws && ws_bytes >= zt_bytes(cr, n2), FA_ERR_WORKSPACE,
             "fa_propagate: workspace %zu < %zu bytes", ws_bytes, zt_bytes(cr, n2));
  return run_propagate(A1, inv_deg1, A2, inv_deg2, C, C_tmp, k, cr, ws, static_cast<hipStream_t>(stream));
}

extern "C" int fa_cost(const fa_csr *A1, const fa_csr *A2, const float *w1, const float *w2, const float *inv_deg1,
                       const float *inv_deg2, const void *S, int32_t s_dtype, const float *C_node,
                       const int32_t *partner, const double *a, const double *b, const fa_params *p,
                       float *C_inout, float *Ct_out, void *ws, size_t ws_bytes, void *stream) {
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
  const size_t need = zt_bytes(cr, n2);
  FA_REQUIRE(ws && ws_bytes >= need, FA_ERR_WORKSPACE, "fa_cost: workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  CostArgs c{A1, A2, w1, inv_deg1, w2, inv_deg2, S, s_dtype, C_node, partner, a, b,
             p->lambda_e, p->lambda_n, p->lambda_a, p->lambda_p, p->eps, p->eps_anchor, p->delta_nbr, C_inout,
             Ct_out};
  return run_cost(c, cr, ws, s);
}
