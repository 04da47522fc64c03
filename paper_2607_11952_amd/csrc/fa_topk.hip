// The plan without a dense buffer of its own.
//
// Top-k plan.  S is concentrated on a few entries per row once the outer
// iterations sharpen it (the paper notes that the plan is often sparse: §3.3,
// memory reduction), and what a caller consumes at scale is each row's short
// list of candidates.
// k_plan_topk streams C once and keeps, per row i, the k largest entries of
// S_ij = exp((a_j + b_i - C_ij)/eps) (Eq. (4)) with their column indices: no
// n1 x n2 output.  Entries are ordered by the FP64 exponent formed exactly as
// the plan pass forms it (larger first, lower j first on equal exponents), so
// the first entry is the plan pass's argmax and every value is, bit for bit,
// the FP32 plan entry the plan pass stores.
//
// Transpose.  When the working plan shares the C^T buffer (the plan is dead
// once the cost rebuild has read it, C^T is dead until the rebuild has written
// the new C), the rebuild writes C only and k_transpose then regenerates C^T
// for the column pass.
#include <limits.h>

#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

// Total order of the top-k lists: larger exponent first, lower column on ties.
__device__ inline bool ranks_before(double y1, int j1, double y2, int j2) {
  return y1 > y2 || (y1 == y2 && j1 < j2);
}

// One wavefront's sorted list (lane l holds its l-th entry; lanes past k hold
// entries shifted out of the list, which are never read) absorbs every pending
// candidate of every lane that still ranks before the list's k-th entry.
// Candidates go in one at a time, the first pending one of the lowest lane
// first; each insertion shifts the entries behind it one lane up.
template <int V>
__device__ inline void absorb(double &ey, int &ej, double &ty, int &tj, const double *y, const int *jj, bool *pend,
                              int k) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    double cy = 0.0;
    int cj = 0, pv = -1;
#pragma unroll
    for (int v = V - 1; v >= 0; --v)
      if (pend[v]) {
        cy = y[v];
        cj = jj[v];
        pv = v;
      }
    const uint64_t m = __ballot(pv >= 0);
    if (m == 0) break;
    const int src = __ffsll(static_cast<unsigned long long>(m)) - 1;
    const double xy = __shfl(cy, src, 64);
    const int xj = __shfl(cj, src, 64);
    const double py = __shfl_up(ey, 1, 64);
    const int pj = __shfl_up(ej, 1, 64);
    if (!ranks_before(ey, ej, xy, xj)) {
      if (lane == 0 || ranks_before(py, pj, xy, xj)) {
        ey = xy;
        ej = xj;
      } else {
        ey = py;
        ej = pj;
      }
    }
    ty = __shfl(ey, k - 1, 64);
    tj = __shfl(ej, k - 1, 64);
    for (int v = 0; v < V; ++v)
      pend[v] = pend[v] && !(lane == src && v == pv) && ranks_before(y[v], jj[v], ty, tj);
  }
}

// R = 4 rows per workgroup.  Each wavefront keeps one list per row over its
// share of the columns (the columns of a step are spread over the workgroup as
// in the plan pass); wavefront r then merges the four lists of row r.
template <int V>
__global__ __launch_bounds__(256) void k_plan_topk(const float *__restrict__ C, int32_t n1, int32_t n2,
                                                   const double *__restrict__ a, const double *__restrict__ b,
                                                   double k2, int32_t k, float *__restrict__ val,
                                                   int32_t *__restrict__ idx) {
  constexpr int R = 4;
  const int i0 = blockIdx.x * R;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double bk[R], ey[R], ty[R];
  int ej[R], tj[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    bk[r] = (i0 + r < n1) ? b[i0 + r] * k2 : 0.0;
    ey[r] = -INFINITY;
    ej[r] = INT_MAX;
    ty[r] = -INFINITY;
    tj[r] = INT_MAX;
  }
  // Wave-uniform trip count: every lane takes part in the list updates.
  for (int base = 0; base < n2; base += 256 * V) {
    const int j = base + threadIdx.x * V;
    const bool in = j < n2;
    const int jc = in ? j : 0;
    double aj[V];
#pragma unroll
    for (int v = 0; v < V; ++v) aj[v] = a[jc + v];
    float cr[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) Vec<V>::load(C + static_cast<int64_t>(min(i0 + r, n1 - 1)) * n2 + jc, cr[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (i0 + r >= n1) continue;  // uniform over the workgroup
      double y[V];
      int jj[V];
      bool pend[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        y[v] = fma(-static_cast<double>(cr[r][v]), k2, fma(aj[v], k2, bk[r]));
        jj[v] = j + v;
        pend[v] = in && ranks_before(y[v], jj[v], ty[r], tj[r]);
      }
      absorb<V>(ey[r], ej[r], ty[r], tj[r], y, jj, pend, k);
    }
  }
  __shared__ double sy[R][4][64];
  __shared__ int sj[R][4][64];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    sy[r][w][lane] = ey[r];
    sj[r][w][lane] = ej[r];
  }
  __syncthreads();
  const int r = w;
  const int i = i0 + r;
  if (i >= n1) return;  // whole wavefront
  double my = sy[r][0][lane], mty = __shfl(my, k - 1, 64);
  int mj = sj[r][0][lane], mtj = __shfl(mj, k - 1, 64);
  for (int q = 1; q < 4; ++q) {
    double y[1] = {sy[r][q][lane]};
    int jj[1] = {sj[r][q][lane]};
    bool pend[1] = {lane < k && ranks_before(y[0], jj[0], mty, mtj)};
    absorb<1>(my, mj, mty, mtj, y, jj, pend, k);
  }
  if (lane < k) {
    const int64_t o = static_cast<int64_t>(i) * k + lane;
    const bool got = mj != INT_MAX;  // fewer than k comparable entries (NaN in C)
    val[o] = got ? exp2_split(my) : 0.0f;
    idx[o] = got ? mj : -1;
  }
}

// C (n1 x n2) -> C^T (n2 x n1), 64 x 64 tiles through LDS; 16-byte accesses on
// interior tiles when both row lengths are multiples of 4.
template <bool VEC>
__global__ __launch_bounds__(256) void k_transpose(const float *__restrict__ C, int32_t n1, int32_t n2,
                                                   float *__restrict__ Ct) {
  __shared__ float t[64][65];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const bool full = VEC && c0 + 64 <= n2 && r0 + 64 <= n1;
  if (full) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = ty + 16 * q;
      const f32x4 v = ld_stream4(C + static_cast<int64_t>(r0 + r) * n2 + c0 + 4 * tx);
      t[r][4 * tx] = v.x;
      t[r][4 * tx + 1] = v.y;
      t[r][4 * tx + 2] = v.z;
      t[r][4 * tx + 3] = v.w;
    }
  } else {
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int r = e >> 6, c = e & 63;
      if (r0 + r < n1 && c0 + c < n2) t[r][c] = ld_stream(C + static_cast<int64_t>(r0 + r) * n2 + c0 + c);
    }
  }
  __syncthreads();
  if (full) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = ty + 16 * q;
      f32x4 v;
      v.x = t[4 * tx][c];
      v.y = t[4 * tx + 1][c];
      v.z = t[4 * tx + 2][c];
      v.w = t[4 * tx + 3][c];
      __builtin_nontemporal_store(v, reinterpret_cast<f32x4 *>(Ct + static_cast<int64_t>(c0 + c) * n1 + r0 + 4 * tx));
    }
  } else {
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int c = e >> 6, r = e & 63;
      if (r0 + r < n1 && c0 + c < n2) st_stream(Ct + static_cast<int64_t>(c0 + c) * n1 + r0 + r, t[r][c]);
    }
  }
}

int run_plan_topk(const float *C, int32_t n1, int32_t n2, double eps, const double *a, const double *b, int32_t k,
                  float *val, int32_t *idx, hipStream_t s, KTimer *tm) {
  if (n1 == 0 || n2 == 0 || k == 0) return FA_OK;
  const int tid = tm ? tm->begin(KK_TOPK, s) : -1;
  const double k2 = kLog2e / eps;
  const dim3 g(ceil_div(n1, 4));
  if (n2 % 4 == 0)
    FA_LAUNCH((k_plan_topk<4>), g, dim3(256), 0, s, C, n1, n2, a, b, k2, k, val, idx);
  else
    FA_LAUNCH((k_plan_topk<1>), g, dim3(256), 0, s, C, n1, n2, a, b, k2, k, val, idx);
  if (tm) tm->end(tid, s);
  return FA_OK;
}

int run_transpose(const float *C, int32_t n1, int32_t n2, float *Ct, hipStream_t s, KTimer *tm) {
  if (n1 == 0 || n2 == 0) return FA_OK;
  const int tid = tm ? tm->begin(KK_TRANSPOSE, s) : -1;
  const dim3 g(ceil_div(n2, 64), ceil_div(n1, 64));
  if (n1 % 4 == 0 && n2 % 4 == 0)
    FA_LAUNCH((k_transpose<true>), g, dim3(256), 0, s, C, n1, n2, Ct);
  else
    FA_LAUNCH((k_transpose<false>), g, dim3(256), 0, s, C, n1, n2, Ct);
  if (tm) tm->end(tid, s);
  return FA_OK;
}

}  // namespace fa

using namespace fa;

extern "C" int fa_plan_topk(const float *C, int32_t n1, int32_t n2, double eps, const double *a, const double *b,
                            int32_t k, float *val, int32_t *idx, void *stream) {
  FA_REQUIRE(n1 >= 0 && n2 >= 0 && eps > 0, FA_ERR_ARG, "fa_plan_topk: bad sizes or eps");
  FA_REQUIRE(k >= 1 && k <= kTopkMax && k <= n2, FA_ERR_ARG, "fa_plan_topk: k = %d outside [1, min(%d, n2 = %d)]",
             k, kTopkMax, n2);
  if (n1 == 0) return FA_OK;
  FA_REQUIRE(C && a && b && val && idx, FA_ERR_ARG, "fa_plan_topk: null pointer");
  return run_plan_topk(C, n1, n2, eps, a, b, k, val, idx, static_cast<hipStream_t>(stream));
}
