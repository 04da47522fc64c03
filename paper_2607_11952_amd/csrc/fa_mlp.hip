// Learned warm start: per-node inputs and a 3-layer MLP (in -> 256 -> 256 -> 1,
// SiLU) with forward, backward (mean squared error) and Adam kernels.
//
// The network predicts the row duals b_i / eps of the first outer solve from
// per-node inputs of G1; fa_align uses the prediction as the starting b of that
// solve (the a-update comes first in each Sinkhorn iteration, so b is the only
// start that matters).  The dense layers are small FP32 contractions
// (N x 24 x 256, N x 256 x 256) done by one LDS-tiled kernel; the whole network
// is a few hundred microseconds at N = 120k.
#include <math.h>

#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

constexpr int kFeat = 24;     // per-node input width
constexpr int kHid = 256;     // hidden width
constexpr int kProj = 16;     // attribute projection width
constexpr int kHops = 8;      // BFS cap

// Parameter blob: W1[kFeat*kHid] b1[kHid] W2[kHid*kHid] b2[kHid] W3[kHid] b3[1] scale[1] offset[1]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid;
constexpr int kOffScale = kOffB3 + 1;
constexpr int kOffOffset = kOffScale + 1;
constexpr int kParams = kOffOffset + 1;

int32_t node_feature_dim() { return kFeat; }

size_t node_features_ws_bytes(int32_t n) {
  Sizer z;
  z.take<int32_t>(n);        // BFS distance
  z.take<float>(n);          // walk mass h
  z.take<float>(n);          // walk mass h+1
  z.take<float>(3 * static_cast<size_t>(n));  // masses h = 1..3
  z.take<float>(static_cast<size_t>(n) * kProj);  // normalised projection
  z.take<float>(kProj * 1024);  // projection matrix (d <= 1024)
  return z.off;
}

// ---------------------------------------------------------------- node inputs

__global__ void k_bfs_init(int32_t *dist, int32_t n, const int32_t *nodes, int32_t nL) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dist[i] = -1;
}
__global__ void k_bfs_seed(int32_t *dist, const int32_t *nodes, int32_t nL) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nL) dist[nodes[l]] = 0;
}
// Pull step: an unvisited node joins level h if a neighbour is at level h-1.
__global__ void k_bfs_level(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t n, int h,
                            int32_t *__restrict__ dist) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || dist[i] >= 0) return;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
    if (dist[col[e]] == h - 1) {
      dist[i] = h;
      return;
    }
}
__global__ void k_indicator(float *r, int32_t n, const int32_t *nodes, int32_t nL) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = 0.f;
}
__global__ void k_indicator_set(float *r, const int32_t *nodes, int32_t nL) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nL) r[nodes[l]] = 1.f;
}
// y = Abar x (one thread per row)
__global__ void k_spmv_avg(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const float *__restrict__ inv, const float *__restrict__ x, int32_t n, float *__restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += x[col[e]];
  y[i] = acc * inv[i];
}

// Fixed Gaussian projection N(0, 1/16) from a counter-based generator
// (SplitMix64 of the element index, then Box-Muller).
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_gauss_proj(float *P, int32_t count, uint64_t seed) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const uint64_t r1 = splitmix64(seed ^ (2ull * q)), r2 = splitmix64(seed ^ (2ull * q + 1));
  const double u1 = (static_cast<double>(r1 >> 11) + 1.0) * (1.0 / 9007199254740992.0);
  const double u2 = static_cast<double>(r2 >> 11) * (1.0 / 9007199254740992.0);
  P[q] = static_cast<float>(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2) * 0.25);
}

// out[i] = [log1p(deg), log1p(sum_{k in N(i)} 1/deg_k), proj(x_hat)[16], dist/8, m1, m2, m3, is_anchor, log(n)/16]
__global__ __launch_bounds__(256) void k_assemble(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                  const float *__restrict__ inv, const float *__restrict__ X, int32_t d,
                                                  const float *__restrict__ P, const int32_t *__restrict__ dist,
                                                  const float *__restrict__ m1, const float *__restrict__ m2,
                                                  const float *__restrict__ m3, int32_t n, float *__restrict__ out) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  // projection of the L2-normalised attribute row (lanes split the 16 outputs x d)
  float ss = 0.f;
  for (int c = lane; c < d; c += 64) ss += X[static_cast<int64_t>(i) * d + c] * X[static_cast<int64_t>(i) * d + c];
  ss = wave_sum(ss);
  const float inrm = ss > 0.f ? 1.0f / sqrtf(ss) : 0.f;
  float proj = 0.f;
  const int q = lane & 15, part = lane >> 4;  // 4 lanes per output
  for (int c = part; c < d; c += 4) proj += X[static_cast<int64_t>(i) * d + c] * P[c * kProj + q];
  proj += __shfl_xor(proj, 16, 64);
  proj += __shfl_xor(proj, 32, 64);
  float *o = out + static_cast<int64_t>(i) * kFeat;
  if (lane < 16) o[2 + lane] = proj * inrm;
  if (lane == 0) {
    const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
    float sinv = 0.f;
    for (int64_t e = e0; e < e1; ++e) sinv += inv[col[e]];
    const int dd = dist[i];
    o[0] = log1pf(static_cast<float>(e1 - e0));
    o[1] = log1pf(sinv);
    o[18] = (dd < 0 ? static_cast<float>(kHops) : static_cast<float>(dd)) / kHops;
    o[19] = m1[i];
    o[20] = m2[i];
    o[21] = m3[i];
    o[22] = dd == 0 ? 1.f : 0.f;
    o[23] = logf(static_cast<float>(n)) / 16.f;
  }
}

int run_node_features(const fa_csr *A, const float *inv_deg, const float *X, int32_t d, const float *proj,
                      const int32_t *nodes, int32_t nL, float *out, void *ws, size_t ws_bytes, hipStream_t s) {
  const int32_t n = A->n;
  if (n == 0) return FA_OK;
  FA_REQUIRE(d <= 1024, FA_ERR_SHAPE, "node features: d = %d above 1024", d);
  Carver cv(ws, ws_bytes);
  int32_t *dist = cv.take<int32_t>(n);
  float *r0 = cv.take<float>(n);
  float *r1 = cv.take<float>(n);
  float *mm = cv.take<float>(3 * static_cast<size_t>(n));
  (void)cv.take<float>(static_cast<size_t>(n) * kProj);
  float *P = cv.take<float>(kProj * 1024);
  FA_REQUIRE(cv.ok, FA_ERR_WORKSPACE, "node features: workspace too small");
  const dim3 g(ceil_div(n, 256)), gl(ceil_div(nL > 0 ? nL : 1, 256));
  FA_LAUNCH(k_bfs_init, g, dim3(256), 0, s, dist, n, nodes, nL);
  if (nL > 0) FA_LAUNCH(k_bfs_seed, gl, dim3(256), 0, s, dist, nodes, nL);
  for (int h = 1; h <= kHops; ++h) FA_LAUNCH(k_bfs_level, g, dim3(256), 0, s, A->rowptr, A->colidx, n, h, dist);
  FA_LAUNCH(k_indicator, g, dim3(256), 0, s, r0, n, nodes, nL);
  if (nL > 0) FA_LAUNCH(k_indicator_set, gl, dim3(256), 0, s, r0, nodes, nL);
  float *src = r0;
  for (int h = 0; h < 3; ++h) {
    float *dst = mm + static_cast<size_t>(h) * n;
    FA_LAUNCH(k_spmv_avg, g, dim3(256), 0, s, A->rowptr, A->colidx, inv_deg, src, n, dst);
    src = dst;
  }
  (void)r1;
  const float *Pp = proj;
  if (!Pp) {
    if (d > 0) FA_LAUNCH(k_gauss_proj, dim3(ceil_div(d * kProj, 256)), dim3(256), 0, s, P, d * kProj, 0x5eedf00dull);
    Pp = P;
  }
  FA_LAUNCH(k_assemble, dim3(ceil_div(n, 4)), dim3(256), 0, s, A->rowptr, A->colidx, inv_deg, X, d, Pp, dist, mm,
            mm + n, mm + 2 * static_cast<size_t>(n), n, out);
  return FA_OK;
}

// ---------------------------------------------------------------- dense layers

__device__ inline float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }

// C[M x N] = op(A) op(B) (+ bias[col]); op(A) is M x K, op(B) is K x N.
// TA: A stored K x M (use A^T); TB: B stored N x K (use B^T).  64x64 tile,
// 256 threads each computing 4x4 outputs, K staged through LDS 16 at a time.
// EPI 0: plain; 1: add bias; 2: add bias and also write silu into H.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_dense(int M, int N, int K, const float *__restrict__ A, int lda,
                                               const float *__restrict__ B, int ldb, const float *__restrict__ bias,
                                               float *__restrict__ Cm, int ldc, float *__restrict__ H) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int t = threadIdx.x; t < 16 * 64; t += 256) {
      const int kk = t / 64, mm = t % 64;
      const int gm = m0 + mm, gk = k0 + kk;
      float va = 0.f;
      if (gm < M && gk < K) va = TA ? A[static_cast<int64_t>(gk) * lda + gm] : A[static_cast<int64_t>(gm) * lda + gk];
      As[kk][mm] = va;
      const int gn = n0 + mm;
      float vb = 0.f;
      if (gn < N && gk < K) vb = TB ? B[static_cast<int64_t>(gn) * ldb + gk] : B[static_cast<int64_t>(gk) * ldb + gn];
      Bs[kk][mm] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = As[kk][ty * 4 + q];
        bv[q] = Bs[kk][tx * 4 + q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += av[p] * bv[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gm = m0 + ty * 4 + p, gn = n0 + tx * 4 + q;
      if (gm < M && gn < N) {
        float v = acc[p][q];
        if (EPI >= 1) v += bias[gn];
        Cm[static_cast<int64_t>(gm) * ldc + gn] = v;
        if (EPI == 2) H[static_cast<int64_t>(gm) * ldc + gn] = v * sigmoidf_(v);
      }
    }
}

// y[i] = scale * (h2[i,:] . W3 + b3) + offset   (one wave per row)
__global__ __launch_bounds__(256) void k_head(const float *__restrict__ h2, const float *__restrict__ prm, int32_t N,
                                              float *__restrict__ y) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  float acc = 0.f;
  for (int c = lane; c < kHid; c += 64) acc += h2[static_cast<int64_t>(i) * kHid + c] * prm[kOffW3 + c];
  acc = wave_sum(acc);
  if (lane == 0) y[i] = prm[kOffScale] * (acc + prm[kOffB3]) + prm[kOffOffset];
}

int run_mlp_forward(const float *prm, const float *x, int32_t N, float *y, float *act, hipStream_t s) {
  if (N == 0) return FA_OK;
  // act: z1 | h1 | z2 | h2, each N x 256
  const size_t NH = static_cast<size_t>(N) * kHid;
  float *z1 = act, *h1 = act + NH, *z2 = act + 2 * NH, *h2 = act + 3 * NH;
  const dim3 g(kHid / 64, ceil_div(N, 64));
  FA_LAUNCH((k_dense<false, false, 2>), g, dim3(256), 0, s, N, kHid, kFeat, x, kFeat, prm + kOffW1, kHid,
            prm + kOffB1, z1, kHid, h1);
  FA_LAUNCH((k_dense<false, false, 2>), g, dim3(256), 0, s, N, kHid, kHid, h1, kHid, prm + kOffW2, kHid,
            prm + kOffB2, z2, kHid, h2);
  FA_LAUNCH(k_head, dim3(ceil_div(N, 4)), dim3(256), 0, s, h2, prm, N, y);
  return FA_OK;
}

// dy[i] = 2 (y_i - t_i) / N * scale ; loss partials (FP64) per block
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t, int32_t N,
                                             float scale, float *__restrict__ dy, double *__restrict__ part) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (i < N) {
    const float r = y[i] - t[i];
    dy[i] = 2.0f * r / static_cast<float>(N) * scale;
    e2 = static_cast<double>(r) * r;
  }
  __shared__ double red[4];
  e2 = wave_sum(e2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ void k_sum_parts(const double *part, int n, double denom, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int q = 0; q < n; ++q) s += part[q];
  *out = s / denom;
}

// dz[i,c] = (sum of dh sources) * silu'(z): mode 0: dh = dy[i] * W3[c]; mode 1: dh given
__global__ void k_silu_back(const float *__restrict__ z, const float *__restrict__ dh, const float *__restrict__ dy,
                            const float *__restrict__ w3, int64_t total, float *__restrict__ dz) {
  int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= total) return;
  const int64_t i = q / kHid;
  const int c = static_cast<int>(q % kHid);
  const float g = dh ? dh[q] : dy[i] * w3[c];
  const float sg = sigmoidf_(z[q]);
  dz[q] = g * sg * (1.0f + z[q] * (1.0f - sg));
}

// out[c] = sum_i M[i, c] (+ optional second column vector), fixed order per column
__global__ void k_colsum(const float *__restrict__ M, int32_t N, int32_t W, float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= W) return;
  double s = 0.0;
  for (int i = 0; i < N; ++i) s += M[static_cast<int64_t>(i) * W + c];
  out[c] = static_cast<float>(s);
}

// gW3[c] = sum_i h2[i,c] dy[i]; gb3 = sum_i dy[i]   (one thread per c, one extra for b3)
__global__ void k_head_grad(const float *__restrict__ h2, const float *__restrict__ dy, int32_t N,
                            float *__restrict__ g) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > kHid) return;
  double s = 0.0;
  if (c < kHid)
    for (int i = 0; i < N; ++i) s += static_cast<double>(h2[static_cast<int64_t>(i) * kHid + c]) * dy[i];
  else
    for (int i = 0; i < N; ++i) s += dy[i];
  g[c < kHid ? kOffW3 + c : kOffB3] = static_cast<float>(s);
}

__global__ void k_zero(float *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

__global__ void k_scale_dy(float *dy, int32_t N, const float *__restrict__ prm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dy[i] *= prm[kOffScale];
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int32_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Warm-start duals for the first outer solve: b_i = eps * MLP(features_i); if any
// prediction is non-finite (e.g. corrupt weights) the whole start falls back to zero.
__global__ void k_pred_check(const float *__restrict__ pred, int32_t n, int32_t *__restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(pred[i])) atomicOr(bad, 1);
}
__global__ void k_pred_to_b(const float *__restrict__ pred, int32_t n, double eps, const int32_t *__restrict__ bad,
                            double *__restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = *bad ? 0.0 : eps * static_cast<double>(pred[i]);
}

size_t mlp_act_floats(int32_t N) { return static_cast<size_t>(N) * (4 * kHid + 2); }

int warm_start_duals(const float *mlp, const float *feat, int32_t n1, float *act, double eps, int32_t *bad, double *b,
                     hipStream_t s) {
  if (n1 == 0) return FA_OK;
  float *pred = act + static_cast<size_t>(n1) * 4 * kHid;
  FA_TRY(run_mlp_forward(mlp, feat, n1, pred, act, s));
  FA_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
  FA_LAUNCH(k_pred_check, dim3(ceil_div(n1, 256)), dim3(256), 0, s, pred, n1, bad);
  FA_LAUNCH(k_pred_to_b, dim3(ceil_div(n1, 256)), dim3(256), 0, s, pred, n1, eps, bad, b);
  return FA_OK;
}

int run_mlp_backward(const float *prm, const float *x, const float *t, int32_t N, float *act, float *grad,
                     double *loss, hipStream_t s) {
  const size_t NH = static_cast<size_t>(N) * kHid;
  float *z1 = act, *h1 = act + NH, *z2 = act + 2 * NH, *h2 = act + 3 * NH;
  float *y = act + 4 * NH, *dy = y + N;
  const int nblk = ceil_div(N, 256);
  double *part = reinterpret_cast<double *>(dy + N);  // 4*N*256 + 2*N floats precede it: 8-byte aligned
  FA_LAUNCH(k_head, dim3(ceil_div(N, 4)), dim3(256), 0, s, h2, prm, N, y);
  FA_LAUNCH(k_mse, dim3(nblk), dim3(256), 0, s, y, t, N, 1.0f, dy, part);
  FA_LAUNCH(k_sum_parts, dim3(1), dim3(64), 0, s, part, nblk, static_cast<double>(N), loss);
  // gradient w.r.t. the pre-scale head output: dL/du = dL/dy * scale
  FA_LAUNCH(k_scale_dy, dim3(nblk), dim3(256), 0, s, dy, N, prm);
  FA_LAUNCH(k_zero, dim3(ceil_div(kParams, 256)), dim3(256), 0, s, grad, kParams);
  FA_LAUNCH(k_head_grad, dim3(ceil_div(kHid + 1, 256)), dim3(256), 0, s, h2, dy, N, grad);
  const int64_t tot = static_cast<int64_t>(NH);
  FA_LAUNCH(k_silu_back, dim3(ceil_div(tot, 256)), dim3(256), 0, s, z2, nullptr, dy, prm + kOffW3, tot, z2);
  // dW2 = h1^T dz2, db2 = colsum dz2
  FA_LAUNCH((k_dense<true, false, 0>), dim3(kHid / 64, kHid / 64), dim3(256), 0, s, kHid, kHid, N, h1, kHid, z2, kHid,
            nullptr, grad + kOffW2, kHid, nullptr);
  FA_LAUNCH(k_colsum, dim3(1), dim3(kHid), 0, s, z2, N, kHid, grad + kOffB2);
  // dh1 = dz2 W2^T (into the h2 slot), dz1 = dh1 * silu'(z1) (into z1)
  FA_LAUNCH((k_dense<false, true, 0>), dim3(kHid / 64, ceil_div(N, 64)), dim3(256), 0, s, N, kHid, kHid, z2, kHid,
            prm + kOffW2, kHid, nullptr, h2, kHid, nullptr);
  FA_LAUNCH(k_silu_back, dim3(ceil_div(tot, 256)), dim3(256), 0, s, z1, h2, nullptr, nullptr, tot, z1);
  // dW1 = x^T dz1, db1 = colsum dz1
  FA_LAUNCH((k_dense<true, false, 0>), dim3(kHid / 64, ceil_div(kFeat, 64)), dim3(256), 0, s, kFeat, kHid, N, x, kFeat,
            z1, kHid, nullptr, grad + kOffW1, kHid, nullptr);
  FA_LAUNCH(k_colsum, dim3(1), dim3(kHid), 0, s, z1, N, kHid, grad + kOffB1);
  return FA_OK;
}

}  // namespace fa

using namespace fa;

extern "C" int32_t fa_node_feature_dim(void) { return kFeat; }
extern "C" int32_t fa_mlp_param_count(void) { return kParams; }
extern "C" size_t fa_node_features_workspace_size(int32_t n) { return n > 0 ? node_features_ws_bytes(n) : 256; }

extern "C" int fa_node_features(const fa_csr *A, const float *inv_deg, const float *X, int32_t d, const float *proj,
                                const int32_t *anchor_nodes, int32_t nL, float *out, void *ws, size_t ws_bytes,
                                void *stream) {
  FA_TRY(check_csr(A, "fa_node_features"));
  FA_REQUIRE(d >= 0 && nL >= 0, FA_ERR_ARG, "fa_node_features: negative size");
  if (A->n == 0) return FA_OK;
  FA_REQUIRE(inv_deg && out && (d == 0 || X) && (nL == 0 || anchor_nodes), FA_ERR_ARG,
             "fa_node_features: null pointer");
  FA_REQUIRE(ws && ws_bytes >= node_features_ws_bytes(A->n), FA_ERR_WORKSPACE, "fa_node_features: workspace too small");
  return run_node_features(A, inv_deg, X, d, proj, anchor_nodes, nL, out, ws, ws_bytes,
                           static_cast<hipStream_t>(stream));
}

extern "C" size_t fa_mlp_act_floats(int32_t N) { return N > 0 ? mlp_act_floats(N) + 2 * ceil_div(N, 256) + 8 : 0; }

extern "C" int fa_mlp_forward(const float *params, const float *x, int32_t N, float *y, float *act, void *stream) {
  FA_REQUIRE(N >= 0, FA_ERR_ARG, "fa_mlp_forward: N < 0");
  if (N == 0) return FA_OK;
  FA_REQUIRE(params && x && y && act, FA_ERR_ARG, "fa_mlp_forward: null pointer");
  return run_mlp_forward(params, x, N, y, act, static_cast<hipStream_t>(stream));
}

extern "C" int fa_mlp_backward(const float *prm, const float *x, const float *t, int32_t N, const float *act,
                               float *grad, double *loss, void *stream) {
  FA_REQUIRE(N > 0, FA_ERR_ARG, "fa_mlp_backward: N must be positive");
  FA_REQUIRE(prm && x && t && act && grad && loss, FA_ERR_ARG, "fa_mlp_backward: null pointer");
  return run_mlp_backward(prm, x, t, N, const_cast<float *>(act), grad, loss, static_cast<hipStream_t>(stream));
}

extern "C" int fa_adam_step(float *params, const float *grad, float *m, float *v, int32_t count, double lr, double beta1,
                            double beta2, double eps_adam, int32_t step, void *stream) {
  FA_REQUIRE(count >= 0 && step >= 1 && lr >= 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps_adam > 0,
             FA_ERR_ARG, "fa_adam_step: bad hyper-parameters");
  if (count == 0) return FA_OK;
  FA_REQUIRE(params && grad && m && v, FA_ERR_ARG, "fa_adam_step: null pointer");
  const float c1 = static_cast<float>(1.0 - pow(beta1, step)), c2 = static_cast<float>(1.0 - pow(beta2, step));
  FA_LAUNCH(k_adam, dim3(ceil_div(count, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), params, grad, m, v,
            count, static_cast<float>(lr), static_cast<float>(beta1), static_cast<float>(beta2),
            static_cast<float>(eps_adam), c1, c2);
  return FA_OK;
}
