// Phase 1 of Algorithm 1: row normalisation, positional encoding (SpMM with a
// restart epilogue), the SDDMM intra-network matrices and attribute normalisation.
#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

// inv_deg[i] = 1/deg_i, 0 for an isolated node.
__global__ void k_inv_deg(const int64_t *__restrict__ rowptr, int32_t n, float *__restrict__ inv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t d = rowptr[i + 1] - rowptr[i];
  inv[i] = d > 0 ? 1.0f / static_cast<float>(d) : 0.0f;
}

// w[e] = inv_deg[col[e]]: the stored values of Abar^T in the CSR order of A
// (A is symmetric, so Abar^T has A's pattern with entry (i,k) = 1/deg_k).
__global__ void k_colinv_weights(const int32_t *__restrict__ col, int64_t nnz,
                                 const float *__restrict__ inv, float *__restrict__ w) {
  FA_GRID_STRIDE(e, nnz) w[e] = inv[col[e]];
}

// out[i, c] = scale * inv_deg[i] * sum_{k in N(i)} X[k, c]
// One workgroup per (row, 1024-column slab); the row's neighbour list is uniform
// across the workgroup so its indices come through the scalar cache.
__global__ __launch_bounds__(256) void k_spmm_rows(const int64_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col,
                                                   const float *__restrict__ inv_deg,
                                                   const float *__restrict__ X, int32_t width,
                                                   float scale, float *__restrict__ out) {
  const int i = blockIdx.x;
  const int c0 = blockIdx.y * 1024;
  const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  int64_t e = e0;
  for (; e + 2 <= e1; e += 2) {
    const float *xa = X + static_cast<int64_t>(col[e]) * width;
    const float *xb = X + static_cast<int64_t>(col[e + 1]) * width;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int c = c0 + q * 256 + threadIdx.x;
      if (c < width) acc[q] += xa[c] + xb[c];
    }
  }
  for (; e < e1; ++e) {
    const float *xa = X + static_cast<int64_t>(col[e]) * width;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int c = c0 + q * 256 + threadIdx.x;
      if (c < width) acc[q] += xa[c];
    }
  }
  const float s = scale * (inv_deg ? inv_deg[i] : 1.0f);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int c = c0 + q * 256 + threadIdx.x;
    if (c < width) out[static_cast<int64_t>(i) * width + c] = s * acc[q];
  }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  FA_GRID_STRIDE(i, n) p[i] = v;
}
__global__ void k_fill_f32(float *p, int64_t n, float v) {
  FA_GRID_STRIDE(i, n) p[i] = v;
}
__global__ void k_fill_f64(double *p, int64_t n, double v) {
  FA_GRID_STRIDE(i, n) p[i] = v;
}

// R[node_l, l] += v for every anchor l (R^(0) is one-hot at the anchor nodes).
__global__ void k_add_onehot(const int32_t *__restrict__ nodes, int32_t nL, float v, float *__restrict__ R) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nL) R[static_cast<int64_t>(nodes[l]) * nL + l] += v;
}

// anchor_of[node_l] = l; counts collisions and out-of-range nodes in *bad.
__global__ void k_anchor_index(const int32_t *__restrict__ anchors, int32_t nL, int side, int32_t n,
                               int32_t *__restrict__ anchor_of, int32_t *__restrict__ bad) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nL) return;
  int u = anchors[2 * l + side];
  if (u < 0 || u >= n) {
    atomicAdd(bad, 1);
    return;
  }
  if (atomicCAS(&anchor_of[u], -1, l) != -1) atomicAdd(bad, 1);
}

// nodes[l] = anchors[2l + side]
__global__ void k_anchor_side(const int32_t *__restrict__ anchors, int32_t nL, int side,
                              int32_t *__restrict__ nodes) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nL) nodes[l] = anchors[2 * l + side];
}

// partner[i] = G2 node of the anchor whose G1 node is i, else -1.
__global__ void k_partner(const int32_t *__restrict__ anchors, const int32_t *__restrict__ anchor_of1,
                          int32_t n1, int32_t *__restrict__ partner) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1) return;
  int l = anchor_of1[i];
  partner[i] = l >= 0 ? anchors[2 * l + 1] : -1;
}

// SDDMM: one workgroup per row, the row's R vector staged in LDS, one wave per
// neighbour at a time, deterministic wave reduction.
template <bool STAGE>
__global__ __launch_bounds__(256) void k_sddmm(const int64_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col,
                                               const float *__restrict__ inv_deg,
                                               const float *__restrict__ R, int32_t nL,
                                               int32_t scale_by_col, float *__restrict__ out) {
  extern __shared__ float ri[];
  const int i = blockIdx.x;
  const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
  if (e0 == e1) return;
  const float *Ri = R + static_cast<int64_t>(i) * nL;
  // STAGE: row i of R in LDS (nL <= 16384); otherwise every wave reads it from
  // global memory, where the workgroup's repeated reads hit the caches
  const float *src = STAGE ? ri : Ri;
  if (STAGE) {
    for (int c = threadIdx.x; c < nL; c += 256) ri[c] = Ri[c];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t e = e0 + w; e < e1; e += 4) {
    const int k = col[e];
    const float *Rk = R + static_cast<int64_t>(k) * nL;
    float acc = 0.f;
    for (int c = lane; c < nL; c += 64) acc += src[c] * Rk[c];
    acc = wave_sum(acc);
    if (lane == 0) out[e] = acc * inv_deg[scale_by_col ? k : i];
  }
}

// Row L2 normalisation: one wave per row.
template <typename TO>
__global__ __launch_bounds__(256) void k_l2norm(const float *__restrict__ X, int32_t n, int32_t d,
                                                TO *__restrict__ out) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const float *x = X + static_cast<int64_t>(row) * d;
  float ss = 0.f;
  for (int c = lane; c < d; c += 64) ss += x[c] * x[c];
  ss = wave_sum(ss);
  const float inv = ss > 0.f ? 1.0f / sqrtf(ss) : 0.0f;
  for (int c = lane; c < d; c += 64) store_from_f32<TO>(out, static_cast<int64_t>(row) * d + c, x[c] * inv);
}

__global__ void k_f32_to_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y) {
  FA_GRID_STRIDE(i, n) y[i] = f32_to_bf16(x[i]);
}

// Row-major [rows x cols] FP32 -> BF16 with row stride ld >= cols, pad columns zero.
__global__ void k_f32_to_bf16_rows(const float *__restrict__ x, int64_t rows, int32_t cols, int32_t ld,
                                   uint16_t *__restrict__ y) {
  FA_GRID_STRIDE(i, rows * ld) {
    const int64_t r = i / ld;
    const int32_t c = static_cast<int32_t>(i - r * ld);
    y[i] = c < cols ? f32_to_bf16(x[r * cols + c]) : static_cast<uint16_t>(0);
  }
}

// ------------------------------------------------------------- launchers

int launch_inv_deg(const fa_csr *A, float *inv, hipStream_t s) {
  if (A->n == 0) return FA_OK;
  FA_LAUNCH(k_inv_deg, dim3(ceil_div(A->n, 256)), dim3(256), 0, s, A->rowptr, A->n, inv);
  return FA_OK;
}

int launch_colinv_weights(const fa_csr *A, const float *inv, float *w, hipStream_t s) {
  if (A->nnz == 0) return FA_OK;
  FA_LAUNCH(k_colinv_weights, stride_grid(A->nnz), dim3(256), 0, s, A->colidx, A->nnz, inv, w);
  return FA_OK;
}

int launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n == 0) return FA_OK;
  FA_LAUNCH(k_fill_i32, stride_grid(n), dim3(256), 0, s, p, n, v);
  return FA_OK;
}
int launch_fill_f32(float *p, int64_t n, float v, hipStream_t s) {
  if (n == 0) return FA_OK;
  FA_LAUNCH(k_fill_f32, stride_grid(n), dim3(256), 0, s, p, n, v);
  return FA_OK;
}
int launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
  if (n == 0) return FA_OK;
  FA_LAUNCH(k_fill_f64, stride_grid(n), dim3(256), 0, s, p, n, v);
  return FA_OK;
}

int launch_anchor_index(const int32_t *anchors, int32_t nL, int side, int32_t n, int32_t *anchor_of,
                        int32_t *bad, hipStream_t s) {
  FA_TRY(launch_fill_i32(anchor_of, n, -1, s));
  if (nL == 0) return FA_OK;
  FA_LAUNCH(k_anchor_index, dim3(ceil_div(nL, 256)), dim3(256), 0, s, anchors, nL, side, n, anchor_of, bad);
  return FA_OK;
}

int launch_anchor_side(const int32_t *anchors, int32_t nL, int side, int32_t *nodes, hipStream_t s) {
  if (nL == 0) return FA_OK;
  FA_LAUNCH(k_anchor_side, dim3(ceil_div(nL, 256)), dim3(256), 0, s, anchors, nL, side, nodes);
  return FA_OK;
}

int launch_partner(const int32_t *anchors, const int32_t *anchor_of1, int32_t n1, int32_t *partner,
                   hipStream_t s) {
  if (n1 == 0) return FA_OK;
  FA_LAUNCH(k_partner, dim3(ceil_div(n1, 256)), dim3(256), 0, s, anchors, anchor_of1, n1, partner);
  return FA_OK;
}

int launch_f32_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s) {
  if (n == 0) return FA_OK;
  FA_LAUNCH(k_f32_to_bf16, stride_grid(n), dim3(256), 0, s, x, n, y);
  return FA_OK;
}

int launch_f32_to_bf16_rows(const float *x, int64_t rows, int32_t cols, int32_t ld, uint16_t *y, hipStream_t s) {
  if (rows == 0 || ld == 0) return FA_OK;
  FA_LAUNCH(k_f32_to_bf16_rows, stride_grid(rows * ld), dim3(256), 0, s, x, rows, cols, ld, y);
  return FA_OK;
}

// R <- (1-beta) Abar R + beta R^(0), k times, ping-ponging between R and R_tmp;
// the result always ends in R.
int launch_positional(const fa_csr *A, const float *inv_deg, const int32_t *anchor_nodes, int32_t nL,
                      double beta, int32_t k, float *R, float *R_tmp, hipStream_t s) {
  const int64_t n = A->n;
  FA_TRY(launch_fill_f32(R, n * nL, 0.f, s));
  if (nL == 0 || n == 0) return FA_OK;
  FA_LAUNCH(k_add_onehot, dim3(ceil_div(nL, 256)), dim3(256), 0, s, anchor_nodes, nL, 1.0f, R);
  float *src = R, *dst = R_tmp;
  dim3 grid(static_cast<unsigned>(n), ceil_div(nL, 1024));
  for (int it = 0; it < k; ++it) {
    FA_LAUNCH(k_spmm_rows, grid, dim3(256), 0, s, A->rowptr, A->colidx, inv_deg, src, nL,
              static_cast<float>(1.0 - beta), dst);
    FA_LAUNCH(k_add_onehot, dim3(ceil_div(nL, 256)), dim3(256), 0, s, anchor_nodes, nL,
              static_cast<float>(beta), dst);
    float *t = src;
    src = dst;
    dst = t;
  }
  if (src != R) FA_HIP(hipMemcpyAsync(R, src, sizeof(float) * n * nL, hipMemcpyDeviceToDevice, s));
  return FA_OK;
}

int launch_sddmm(const fa_csr *A, const float *inv_deg, const float *R, int32_t nL, int32_t by_col,
                 float *out, hipStream_t s) {
  if (A->n == 0 || A->nnz == 0) return FA_OK;
  if (nL == 0) return launch_fill_f32(out, A->nnz, 0.f, s);
  if (static_cast<size_t>(nL) * 4 <= 64 * 1024)
    FA_LAUNCH(k_sddmm<true>, dim3(A->n), dim3(256), sizeof(float) * nL, s, A->rowptr, A->colidx, inv_deg, R,
              nL, by_col, out);
  else
    FA_LAUNCH(k_sddmm<false>, dim3(A->n), dim3(256), 0, s, A->rowptr, A->colidx, inv_deg, R, nL, by_col, out);
  return FA_OK;
}

int launch_l2norm(const float *X, int32_t n, int32_t d, void *out, int32_t dt, hipStream_t s) {
  if (n == 0 || d == 0) return FA_OK;
  if (dt == FA_BF16)
    FA_LAUNCH(k_l2norm<uint16_t>, dim3(ceil_div(n, 4)), dim3(256), 0, s, X, n, d, static_cast<uint16_t *>(out));
  else
    FA_LAUNCH(k_l2norm<float>, dim3(ceil_div(n, 4)), dim3(256), 0, s, X, n, d, static_cast<float *>(out));
  return FA_OK;
}

}  // namespace fa

// ------------------------------------------------------------- ABI

using namespace fa;

extern "C" int fa_row_normalize(const fa_csr *A, float *inv_deg, void *stream) {
  FA_TRY(check_csr(A, "fa_row_normalize"));
  FA_REQUIRE(A->n == 0 || inv_deg, FA_ERR_ARG, "fa_row_normalize: null inv_deg");
  return launch_inv_deg(A, inv_deg, static_cast<hipStream_t>(stream));
}

extern "C" int fa_positional(const fa_csr *A, const float *inv_deg, const int32_t *anchor_nodes, int32_t nL,
                             double beta, int32_t k, float *R, float *R_tmp, void *stream) {
  FA_TRY(check_csr(A, "fa_positional"));
  FA_REQUIRE(nL >= 0 && k >= 0, FA_ERR_ARG, "fa_positional: nL = %d, k = %d", nL, k);
  FA_REQUIRE(nL == 0 || (R && R_tmp && anchor_nodes && inv_deg), FA_ERR_ARG, "fa_positional: null pointer");
  return launch_positional(A, inv_deg, anchor_nodes, nL, beta, k, R, R_tmp,
                           static_cast<hipStream_t>(stream));
}

extern "C" int fa_sddmm(const fa_csr *A, const float *inv_deg, const float *R, int32_t nL, int32_t scale_by_col,
                        float *out, void *stream) {
  FA_TRY(check_csr(A, "fa_sddmm"));
  FA_REQUIRE(nL >= 0, FA_ERR_ARG, "fa_sddmm: nL < 0");
  FA_REQUIRE(A->nnz == 0 || (out && inv_deg && (nL == 0 || R)), FA_ERR_ARG, "fa_sddmm: null pointer");
  return launch_sddmm(A, inv_deg, R, nL, scale_by_col, out, static_cast<hipStream_t>(stream));
}

extern "C" int fa_l2_normalize(const float *X, int32_t n, int32_t d, void *out, int32_t out_dtype, void *stream) {
  FA_REQUIRE(n >= 0 && d >= 0, FA_ERR_ARG, "fa_l2_normalize: negative size");
  FA_REQUIRE(out_dtype == FA_F32 || out_dtype == FA_BF16, FA_ERR_ARG, "fa_l2_normalize: dtype %d", out_dtype);
  FA_REQUIRE(n * (int64_t)d == 0 || (X && out), FA_ERR_ARG, "fa_l2_normalize: null pointer");
  return launch_l2norm(X, n, d, out, out_dtype, static_cast<hipStream_t>(stream));
}
