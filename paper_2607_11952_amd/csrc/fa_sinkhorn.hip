// Phase 3 of Algorithm 1: log-domain Sinkhorn (Eq. (3)) and plan recovery (Eq. (4)).
//
// Each pass streams the FP32 cost once with fused shift / exp / sum (§3.5): the
// exponent (a_j + b_i - C_ij)/eps is assembled in FP64 (duals are FP64), shifted
// by the running maximum in FP64, and only the shifted value (at most 0, small
// where it matters) is rounded to FP32 for exp2; sums accumulate in FP64.
// Shifting by the current duals turns each update into an increment,
//   a_j <- a_j + eps * (log nu_j - LSE_i((a_j + b_i - C_ij)/eps)),
//   b_i <- b_i + eps * (log mu_i - LSE_j((a_j + b_i - C_ij)/eps)),
// which is Eq. (3) rewritten, so FP32 only ever sees well-scaled exponents.
//
// Two forms of the column pass (a-update).  With a transposed copy C^T (written by
// the cost rebuild) it streams rows of C^T exactly like the row pass streams rows
// of C: R columns per workgroup, each workgroup leaves its share of the marginal
// error and a one-workgroup kernel forms the total and the stop decision.
// Without it, workgroups own a column strip and a row range of C and leave a
// (max, sum) partial per column, and a merge kernel folds the partials in a fixed
// order.  Either way the pass also yields the column sums of the current plan,
// i.e. the L1 marginal error of the previous iteration, for free, and every
// reduction runs in a fixed order (deterministic, no float atomics).  The row pass
// (b-update) gives each workgroup eight rows and reduces across the workgroup with
// wavefront shuffles.
//
// Single-pass form (fa_sinkhorn_fused, and fa_align with sink_fused): from the
// third iteration on, one pass over C does the b-update of an iteration and the
// column sums of the a-update that follows, so C is read once per iteration
// instead of twice.  A row's b needs the whole row, and the row's plan entries
// after that update feed every column sum; a row is split across gc partner
// workgroups (column slices, kept in registers), which exchange their partial row
// sums through tagged 64-bit slots (a bounded wait on co-resident workgroups,
// launched cooperatively), then fold the row's new plan entries into
// per-workgroup column sums.  No running maximum is needed:
// after an a-update every plan entry is at most nu_j, and once b comes from a
// b-update every row sum is at least mu_i * min_j nu_j, so 2^y with the exponent
// y = (a_j + b_i - C_ij) log2(e)/eps of the current duals stays in FP32 range.
//
// The loop never waits for the host: a device control word marks convergence and
// every later kernel of the loop returns at its first instruction.
#include <atomic>
#include <mutex>

#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

struct SinkCtl {
  int32_t done;
  int32_t iters;
  int32_t which;    // buffer (0: caller's a, 1: scratch) that holds the final a
  uint32_t arrive;  // last-block counter of the merge kernel
  int32_t fault;    // a partner wait of the single-pass form exceeded its bound
};

constexpr int kColTRowsPerWg = 8;  // columns (rows of C^T) per workgroup of the transposed column pass

struct SinkLayout {
  int V, ncolblk, nsplit, rows_per_split, nmerge, ncolt;
};

static SinkLayout sink_layout(int32_t n1, int32_t n2) {
  SinkLayout L;
  L.V = (n2 % 4 == 0) ? 4 : 1;
  L.ncolblk = ceil_div(n2, 256 * L.V);
  // about 5000 workgroups (three rounds of resident ones): long row ranges keep
  // each workgroup's stream sequential (measured: ~45 splits of 2,700 rows at
  // n = 120k beat 70, 105 or 139 splits), while the tail stays short
  int want = ceil_div(5120, L.ncolblk > 0 ? L.ncolblk : 1);
  int maxs = n1 / 64 > 1 ? n1 / 64 : 1;  // at least 64 rows per split: partials stay small next to C
  L.nsplit = want < 1 ? 1 : (want > maxs ? maxs : want);
  L.rows_per_split = ceil_div(n1 > 0 ? n1 : 1, L.nsplit);
  L.nmerge = ceil_div(n2, 64);
  L.ncolt = ceil_div(n2, kColTRowsPerWg);
  return L;
}

// Single-pass form: kFuseQ quads (four consecutive columns) per thread and
// 256 threads per workgroup, so a partner's slice holds up to 4096 columns;
// kFuseK rows per exchange batch; at most kFuseMaxGrid co-resident workgroups.
constexpr int kFuseQ = 4;
constexpr int kFuseK = 2;
constexpr int kFuseMaxGrid = 2048;
constexpr int32_t kFuseSpinDefault = 1 << 22;

// Partners per row: the fewest whose slices fit kFuseQ quads per thread (more
// partners would only mean fewer row groups on the same co-resident grid).
static int fuse_partners(int32_t n2) {
  const int64_t nq = n2 / 4;
  const int64_t need = (nq + 256 * kFuseQ - 1) / (256 * kFuseQ);
  return static_cast<int>(need > 0 ? need : 1);
}
// Slots per row of the exchange: gc rounded up to a multiple of 8, so a batch of
// kFuseK = 2 rows fills whole 128-byte lines and no line holds slots of two
// batches: the stores publishing one batch and the snapshot loads of the next never
// touch the same line (rows packed at gc slots ran the pass several percent slower).
__host__ __device__ constexpr int fuse_stride(int gc) { return (gc + 7) & ~7; }
// Row groups a grid can have: kFuseMaxGrid / gc, and no more than batches of rows.
static int fuse_groups_cap(int32_t n1, int32_t n2) {
  const int gc = fuse_partners(n2);
  const int64_t by_grid = gc >= kFuseMaxGrid ? 1 : kFuseMaxGrid / gc;
  const int64_t by_rows = (static_cast<int64_t>(n1) + kFuseK - 1) / kFuseK;
  const int64_t cap = by_grid < by_rows ? by_grid : by_rows;
  return static_cast<int>(cap > 0 ? cap : 1);
}

// Which scratch a solve carves: the strip partials pm/ps serve the column pass
// without C^T; SINK_FUSED adds the single-pass exchange (a tagged row partial per
// row and partner, column sums per row group).
enum SinkMode { SINK_TWO_PASS = 0, SINK_T_ONLY = 1, SINK_FUSED = 2 };

template <typename Z>
static void take_sink(Z &z, int32_t n1, int32_t n2, SinkMode mode) {
  SinkLayout L = sink_layout(n1, n2);
  if (mode != SINK_T_ONLY) {
    z.template take<double>(static_cast<size_t>(L.nsplit) * n2);
    z.template take<double>(static_cast<size_t>(L.nsplit) * n2);
  }
  z.template take<double>(n2);
  z.template take<double>((L.nmerge > L.ncolt ? L.nmerge : L.ncolt) + 1);
  z.template take<SinkCtl>(1);
  z.template take<double>(1);
  if (mode == SINK_FUSED) {
    z.template take<uint64_t>(static_cast<size_t>(n1) * fuse_stride(fuse_partners(n2)));
    z.template take<double>(static_cast<size_t>(fuse_groups_cap(n1, n2)) * n2);
  }
}

static size_t sink_scratch_bytes(int32_t n1, int32_t n2, SinkMode mode) {
  Sizer z;
  take_sink(z, n1, n2, mode);
  return z.off;
}

size_t sinkhorn_ws_bytes(int32_t n1, int32_t n2, bool fused) {
  return sink_scratch_bytes(n1, n2, fused ? SINK_FUSED : SINK_TWO_PASS);
}

static int carve_sink(Carver &cv, int32_t n1, int32_t n2, SinkWs &w, SinkMode mode) {
  SinkLayout L = sink_layout(n1, n2);
  w.pm = mode == SINK_T_ONLY ? nullptr : cv.take<double>(static_cast<size_t>(L.nsplit) * n2);
  w.ps = mode == SINK_T_ONLY ? nullptr : cv.take<double>(static_cast<size_t>(L.nsplit) * n2);
  w.a_next = cv.take<double>(n2);
  w.errp = cv.take<double>((L.nmerge > L.ncolt ? L.nmerge : L.ncolt) + 1);
  w.ctl = reinterpret_cast<int32_t *>(cv.take<SinkCtl>(1));
  w.err = cv.take<double>(1);
  w.part = nullptr;
  w.pcol = nullptr;
  if (mode == SINK_FUSED) {
    w.part = cv.take<uint64_t>(static_cast<size_t>(n1) * fuse_stride(fuse_partners(n2)));
    w.pcol = cv.take<double>(static_cast<size_t>(fuse_groups_cap(n1, n2)) * n2);
  }
  w.nsplit = L.nsplit;
  w.nerrblk = L.nmerge;
  return cv.ok ? FA_OK : FA_ERR_WORKSPACE;
}

int carve_sinkhorn(Carver &cv, int32_t n1, int32_t n2, SinkWs &w, bool fused) {
  return carve_sink(cv, n1, n2, w, fused ? SINK_FUSED : SINK_TWO_PASS);
}

// Vector store of V consecutive plan entries (one 16-byte FP32 or 8-byte BF16
// store per lane for V = 4).
template <typename T, int V>
struct VStore {
  static __device__ inline void run(T *p, const float *v) {
#pragma unroll
    for (int q = 0; q < V; ++q) store_from_f32<T>(p, q, v[q]);
  }
};
template <>
struct VStore<float, 4> {
  static __device__ inline void run(float *p, const float *v) {
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};
template <>
struct VStore<uint16_t, 4> {
  static __device__ inline void run(uint16_t *p, const float *v) {
    const uint32_t w0 = static_cast<uint32_t>(f32_to_bf16(v[0])) | (static_cast<uint32_t>(f32_to_bf16(v[1])) << 16);
    const uint32_t w1 = static_cast<uint32_t>(f32_to_bf16(v[2])) | (static_cast<uint32_t>(f32_to_bf16(v[3])) << 16);
    *reinterpret_cast<uint2 *>(p) = make_uint2(w0, w1);
  }
};

// Rows of C in flight per thread and step of the column pass.
constexpr int kColRowsPerStep = 4;

// Column pass, part 1: per (column strip, row range) partial LSE of
// y_ij = (a_j + b_i - C_ij) * log2(e)/eps over the rows of the range.
template <int V, int U>
__global__ __launch_bounds__(256) void k_lse_col_partial(const float *__restrict__ C, int32_t n1, int32_t n2,
                                                         const double *__restrict__ bufA0,
                                                         const double *__restrict__ bufA1, int32_t cur,
                                                         const double *__restrict__ b, double k2,
                                                         int32_t rows_per_split, double *__restrict__ pm,
                                                         double *__restrict__ ps,
                                                         const SinkCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const double *a = cur ? bufA1 : bufA0;
  const int j = (blockIdx.x * 256 + threadIdx.x) * V;
  const int split = blockIdx.y;
  const int r0 = split * rows_per_split;
  const int r1 = min(n1, r0 + rows_per_split);
  if (j >= n2) return;
  double ak[V], m[V], s[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    ak[v] = a[j + v] * k2;
    m[v] = -INFINITY;
    s[v] = 0.0;
  }
  for (int i = r0; i < r1; i += U) {
    // All U row loads are issued before any is used (no branch around a load, so
    // none waits for the previous one); rows past the range re-read row r1-1 and
    // are masked to -inf.
    float c[U][V];
    double bk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int iu = min(i + u, r1 - 1);
      Vec<V>::load(C + static_cast<int64_t>(iu) * n2 + j, c[u]);
      bk[u] = b[iu] * k2;
    }
    double x[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < V; ++v)
        x[u][v] = (i + u < r1) ? fma(-static_cast<double>(c[u][v]), k2, ak[v] + bk[u]) : -INFINITY;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      double mx = x[0][v];
#pragma unroll
      for (int u = 1; u < U; ++u) mx = fmax(mx, x[u][v]);
      if (mx > m[v]) {
        s[v] *= static_cast<double>(exp2f(static_cast<float>(m[v] - mx)));
        m[v] = mx;
      }
      float t = 0.f;
#pragma unroll
      for (int u = 0; u < U; ++u) t += exp2f(static_cast<float>(x[u][v] - m[v]));
      s[v] += static_cast<double>(t);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    pm[static_cast<int64_t>(split) * n2 + j + v] = m[v];
    ps[static_cast<int64_t>(split) * n2 + j + v] = s[v];
  }
}

// Block-order sum of the per-column violations e (one value per thread, zero
// where a thread owns no column) and, in the last workgroup to arrive, the
// fixed-order total and the stop rule.  Called by every thread of the workgroup.
__device__ inline void finish_error(double e, double *__restrict__ errp, SinkCtl *__restrict__ ctl, int32_t it,
                                    int32_t is_check, int32_t is_final, double tol, int32_t cur,
                                    int32_t *__restrict__ out_iters, double *__restrict__ out_err) {
  __shared__ double red[4];
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  __shared__ bool last;
  if (threadIdx.x == 0) {
    errp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    __threadfence();
    const uint32_t prev = atomicAdd(&ctl->arrive, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double t = 0.0;
  for (int q = threadIdx.x; q < static_cast<int>(gridDim.x); q += 256)
    t += __hip_atomic_load(&errp[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  t = wave_sum(t);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double err = (red[0] + red[1]) + (red[2] + red[3]);
    ctl->arrive = 0u;
    *out_err = err;
    if (is_final || (is_check && tol > 0.0 && err <= tol)) {
      ctl->done = 1;
      ctl->iters = it;
      ctl->which = cur;
      *out_iters = it;
    }
  }
}

// Block-order sum of e into errp[blockIdx.x] only (no arrival counter): for
// grids too large for one same-address atomic per workgroup to stay cheap.
__device__ inline void block_error(double e, double *__restrict__ errp) {
  __shared__ double red[4];
  e = wave_sum(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) errp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One workgroup: the fixed-order total of nblk block partials and the stop rule.
__global__ __launch_bounds__(256) void k_error_finish(const double *__restrict__ errp, int32_t nblk,
                                                      SinkCtl *__restrict__ ctl, int32_t it, int32_t is_check,
                                                      int32_t is_final, double tol, int32_t cur,
                                                      int32_t *__restrict__ out_iters, double *__restrict__ out_err) {
  if (ctl->done) return;
  double t = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 256) t += errp[q];
  __shared__ double red[4];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double err = (red[0] + red[1]) + (red[2] + red[3]);
    *out_err = err;
    if (is_final || (is_check && tol > 0.0 && err <= tol)) {
      ctl->done = 1;
      ctl->iters = it;
      ctl->which = cur;
      *out_iters = it;
    }
  }
}

// Column pass, part 2: fold the partials of each column in a fixed order, form the
// new a_j (into the other buffer) and the column's marginal violation; the last
// workgroup to finish sums the violations in block order and applies the stop rule.
// A workgroup takes 64 columns; four lanes per column fold every fourth split
// each (one pass, online max), then lane group 0 folds the four results in order.
__global__ __launch_bounds__(256) void k_lse_col_merge(int32_t n2, int32_t nsplit, const double *__restrict__ pm,
                                                       const double *__restrict__ ps, double *__restrict__ bufA0,
                                                       double *__restrict__ bufA1, int32_t cur, double eps,
                                                       double log_nu, double nu, double *__restrict__ errp,
                                                       SinkCtl *__restrict__ ctl, int32_t it, int32_t is_check,
                                                       int32_t is_final, double tol, int32_t *__restrict__ out_iters,
                                                       double *__restrict__ out_err) {
  if (ctl->done) return;
  const double *a = cur ? bufA1 : bufA0;
  double *an = cur ? bufA0 : bufA1;
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  double M = -INFINITY, S = 0.0;
  if (j < n2)
    for (int q = g; q < nsplit; q += 4)
      lse2_merge(M, S, pm[static_cast<int64_t>(q) * n2 + j], ps[static_cast<int64_t>(q) * n2 + j]);
  __shared__ double fm[4][64], fs[4][64];
  fm[g][c] = M;
  fs[g][c] = S;
  __syncthreads();
  double e = 0.0;
  if (g == 0 && j < n2) {
    for (int q = 1; q < 4; ++q) lse2_merge(M, S, fm[q][c], fs[q][c]);
    const double l2 = M + log2(S);  // log2 of the column sum
    an[j] = a[j] + eps * (log_nu - l2 * kLn2);
    e = fabs(exp2(l2) - nu);
  }
  finish_error(e, errp, ctl, it, is_check, is_final, tol, cur, out_iters, out_err);
}

// Row pass (b-update): R rows per workgroup, the a-values of a column chunk are
// loaded once and reused for the R rows.
constexpr int kRowsPerWg = 8;
template <int V, int R>
__global__ __launch_bounds__(256) void k_lse_row(const float *__restrict__ C, int32_t n1, int32_t n2,
                                                 const double *__restrict__ bufA0, const double *__restrict__ bufA1,
                                                 int32_t nxt, double *__restrict__ b, double k2, double eps,
                                                 double log_mu, const SinkCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const double *a = nxt ? bufA1 : bufA0;
  const int i0 = blockIdx.x * R;
  double bk[R], m[R], s[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    bk[r] = (i0 + r < n1) ? b[i0 + r] * k2 : 0.0;
    m[r] = -INFINITY;
    s[r] = 0.0;
  }
  for (int j = threadIdx.x * V; j < n2; j += 256 * V) {
    // the R row loads go out together; rows past n1 re-read row n1-1, their sums are dropped
    float cr[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) Vec<V>::load(C + static_cast<int64_t>(min(i0 + r, n1 - 1)) * n2 + j, cr[r]);
    double ak[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ak[v] = a[j + v] * k2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float *c = cr[r];
      double x[V];
      double mx = -INFINITY;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        x[v] = fma(-static_cast<double>(c[v]), k2, ak[v] + bk[r]);
        mx = fmax(mx, x[v]);
      }
      if (mx > m[r]) {
        s[r] *= static_cast<double>(exp2f(static_cast<float>(m[r] - mx)));
        m[r] = mx;
      }
      float t = 0.f;
#pragma unroll
      for (int v = 0; v < V; ++v) t += exp2f(static_cast<float>(x[v] - m[r]));
      s[r] += static_cast<double>(t);
    }
  }
  __shared__ double sm[R][4];
  __shared__ double ss[R][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double mr = m[r];
    double sr = s[r];
    wave_lse2(mr, sr);
    if (lane == 0) {
      sm[r][w] = mr;
      ss[r][w] = sr;
    }
  }
  __syncthreads();
  if (threadIdx.x < R) {
    const int r = threadIdx.x;
    if (i0 + r < n1) {
      double M = sm[r][0];
      double S = ss[r][0];
      for (int q = 1; q < 4; ++q) lse2_merge(M, S, sm[r][q], ss[r][q]);
      const double l2 = M + log2(S);
      b[i0 + r] = b[i0 + r] + eps * (log_mu - l2 * kLn2);
    }
  }
}

// Column pass from the transposed cost Ct = C^T (n2 rows of length n1): the row
// pass's streaming pattern (whole rows, R at a time) applied to columns, so the
// a-update reads long contiguous runs instead of 4 KB pieces of many rows.
// Computes the new a_j (into the other buffer) and the column's marginal
// violation; k_error_finish then forms the total and applies the stop rule.
template <int V, int R>
__global__ __launch_bounds__(256) void k_lse_col_t(const float *__restrict__ Ct, int32_t n1, int32_t n2,
                                                   double *__restrict__ bufA0, double *__restrict__ bufA1,
                                                   int32_t cur, const double *__restrict__ b, double k2, double eps,
                                                   double log_nu, double nu, double *__restrict__ errp,
                                                   const SinkCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const double *a = cur ? bufA1 : bufA0;
  double *an = cur ? bufA0 : bufA1;
  const int j0 = blockIdx.x * R;
  double ak[R], m[R], s[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ak[r] = (j0 + r < n2) ? a[j0 + r] * k2 : 0.0;
    m[r] = -INFINITY;
    s[r] = 0.0;
  }
  for (int i = threadIdx.x * V; i < n1; i += 256 * V) {
    // the R row loads of Ct go out together; rows past n2 re-read row n2-1, their sums are dropped
    float cr[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) Vec<V>::load(Ct + static_cast<int64_t>(min(j0 + r, n2 - 1)) * n1 + i, cr[r]);
    double bk[V];
#pragma unroll
    for (int v = 0; v < V; ++v) bk[v] = b[i + v] * k2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float *c = cr[r];
      double x[V];
      double mx = -INFINITY;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        x[v] = fma(-static_cast<double>(c[v]), k2, bk[v] + ak[r]);
        mx = fmax(mx, x[v]);
      }
      if (mx > m[r]) {
        s[r] *= static_cast<double>(exp2f(static_cast<float>(m[r] - mx)));
        m[r] = mx;
      }
      float t = 0.f;
#pragma unroll
      for (int v = 0; v < V; ++v) t += exp2f(static_cast<float>(x[v] - m[r]));
      s[r] += static_cast<double>(t);
    }
  }
  __shared__ double sm[R][4];
  __shared__ double ss[R][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double mr = m[r];
    double sr = s[r];
    wave_lse2(mr, sr);
    if (lane == 0) {
      sm[r][w] = mr;
      ss[r][w] = sr;
    }
  }
  __syncthreads();
  double e = 0.0;
  if (threadIdx.x < R) {
    const int r = threadIdx.x, j = j0 + r;
    if (j < n2) {
      double M = sm[r][0];
      double S = ss[r][0];
      for (int q = 1; q < 4; ++q) lse2_merge(M, S, sm[r][q], ss[r][q]);
      const double l2 = M + log2(S);  // log2 of the column sum of the current plan
      an[j] = a[j] + eps * (log_nu - l2 * kLn2);
      e = fabs(exp2(l2) - nu);
    }
  }
  block_error(e, errp);
}

// Final a: copy the scratch buffer into the caller's a if it holds the result.  After
// an aborted single-pass iteration the outputs say so: iterations -1, error NaN.
__global__ void k_final_a(double *__restrict__ a, const double *__restrict__ alt, int32_t n2,
                          const SinkCtl *__restrict__ ctl, int32_t *__restrict__ out_iters,
                          double *__restrict__ out_err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0 && ctl->fault) {
    *out_iters = -1;
    *out_err = NAN;
  }
  if (ctl->which != 1) return;
  if (j < n2) a[j] = alt[j];
}

__global__ void k_sink_reset(SinkCtl *ctl) {
  ctl->done = 0;
  ctl->iters = 0;
  ctl->which = 0;
  ctl->arrive = 0u;
  ctl->fault = 0;
}

// ---------------------------------------------------------------- single-pass iteration

// Exchange slots of the single pass: a partner's partial row sum (FP64, positive)
// with its low 8 mantissa bits replaced by the pass tag (1..255; 0 = cleared), so
// value and tag travel in one 64-bit word and a reader needs no ordering between
// them: it polls a row's slots with device-scope atomic loads until every tag is
// the current pass's.  Dropping 8 of 52 fraction bits changes the value by at most
// 2^-44 relative.
__device__ __forceinline__ uint64_t fuse_pack(double v, uint32_t tag) {
  return (static_cast<uint64_t>(__double_as_longlong(v)) & ~0xffull) | tag;
}
__device__ __forceinline__ double fuse_value(uint64_t x) {
  return __longlong_as_double(static_cast<long long>(x & ~0xffull));
}

// v + (v of the lane the DPP control selects), on both halves of an FP64 value; lanes
// outside row_mask add 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
  return v + __hiloint2double(hi2, lo2);
}

// Sum over aligned groups of g lanes (g a power of two <= 64), in a fixed order,
// without leaving the vector unit: quad swaps, half-row and row mirrors, then row
// broadcasts.  The group's sum ends in its last lane (every lane of the group for
// g <= 16).
__device__ __forceinline__ double group_sum(double v, int g) {
  if (g >= 2) v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  if (g >= 4) v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  if (g >= 8) v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  if (g >= 16) v = dpp_add<0x140, 0xf>(v); // row_mirror
  if (g >= 32) v = dpp_add<0x142, 0xa>(v); // row_bcast:15 into rows 1 and 3
  if (g >= 64) v = dpp_add<0x143, 0xc>(v); // row_bcast:31 into rows 2 and 3
  return v;
}

// The rows of one row group, for one partner workgroup (one column slice), as a
// pipeline over batches of K rows: load, then produce (2^y of the batch's entries,
// its partial row sums published by wave 0), then consume (every wave forms the
// batch's row sums over all partners itself, partner 0 updates b, and the batch's
// plan entries go into the column sums).  Step t loads batch t+3, produces batch
// t+2 and consumes batch t, so a batch's exchange has more than a step to complete
// before it is needed.  ak (a_j log2(e)/eps of the slice; -inf for masked quads,
// whose 2^y is then 0) and the column sums cs live in LDS, each thread owning its
// entries.  A wave that gives up a wait records the fault and stops waiting but
// runs to the end, so the workgroup's barriers stay matched.
template <int Q, int K>
struct FusePipe {
  const float *C;
  int32_t n2;
  double k2, eps, log_mu, mu;
  int32_t gc, gs, c, spin_limit, glog;  // gs slots per row; 1 << glog lanes per row in the exchange (>= gc)
  uint32_t tag;
  int64_t row0, row1;
  double *b;
  uint64_t *part;
  SinkCtl *ctl;
  const double *ak;  // LDS [Q][256][4]
  double *cs;        // LDS [Q][256][4]
  double *bold;      // LDS [4][K]: the rows' b before the update, by batch mod 4
  int jq[Q];
  bool faulted;

  __device__ __forceinline__ void load(int t, f32x4 (&x)[K][Q], double (&bx)[K]) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      int64_t i = row0 + static_cast<int64_t>(t) * K + k;
      if (i > row1 - 1) i = row1 - 1;  // rows past the group re-read its last row; they publish nothing
#pragma unroll
      for (int u = 0; u < Q; ++u) x[k][u] = ld_stream4(C + i * n2 + jq[u]);
      bx[k] = b[i];
    }
  }

  // 2^y of the batch (in place) and its partial row sums, published by wave 0.
  __device__ __forceinline__ void produce(int t, f32x4 (&x)[K][Q], const double (&bx)[K], double (&red)[K][4]) const {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double sk[K];
    double bk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      sk[k] = 0.0;
      bk[k] = bx[k] * k2;
    }
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      double a4[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) a4[v] = ak[(u * 256 + threadIdx.x) * 4 + v];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float q4 = 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // y <= log2(nu_j) <= 0 after an a-update; below 2^-126 the result flushes to 0
          const float e = __builtin_amdgcn_exp2f(static_cast<float>(fma(-static_cast<double>(x[k][u][v]), k2, a4[v] + bk[k])));
          x[k][u][v] = e;
          q4 += e;
        }
        sk[k] += static_cast<double>(q4);
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double v = group_sum(sk[k], 64);  // the wave's sum, in lane 63
      if (lane == 63) red[k][wv] = v;
    }
    __syncthreads();
    const int64_t ib = row0 + static_cast<int64_t>(t) * K;
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < K; ++k) bold[(t & 3) * K + k] = bx[k];  // read when batch t is consumed
    if (wv == 0 && lane < K && ib + lane < row1)
      __hip_atomic_store(&part[(ib + lane) * gs + c],
                         fuse_pack((red[lane][0] + red[lane][1]) + (red[lane][2] + red[lane][3]), tag),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  // This wave's snapshot of the batch's slots (lane l: row ib + (l >> glog),
  // partner l mod 2^glog; needs K << glog <= 64), loaded before the step's data
  // loads so that reading it later does not wait for those (vector loads return
  // in order).  Lanes without a slot, and rows past the group, read as ready.  The read skips
  // the CU's L1 and is served by the XCD's L2, where the stores of partners on the
  // same XCD land (the grid puts a row group's partners on one XCD); it may miss a
  // store from another XCD, but a stale slot carries an earlier pass's tag, so the
  // batch then goes to the device-coherent gather.
  __device__ __forceinline__ uint64_t snap(int64_t ib) const {
    const int lane = threadIdx.x & 63;
    const int k = lane >> glog, q = lane & ((1 << glog) - 1);
    if (k >= K || q >= gc || ib + k >= row1) return tag;
    // a uniform base plus a small per-lane offset, with no per-lane address kept
    // across the loop
    return __hip_atomic_load(part + ib * gs + (k * gs + q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  // With 33..64 partners a row takes the whole wave: one snapshot load per row.
  __device__ __forceinline__ uint64_t snap_row(int64_t i) const {
    const int lane = threadIdx.x & 63;
    if (lane >= gc || i >= row1) return tag;
    return __hip_atomic_load(part + i * gs + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }

  // Device-coherent gather (bounded wait): until every partner's slot of the
  // batch's rows carries this pass's tag, then the row sums in partner order.
  // After a wait is given up the fault is recorded and nothing more is awaited.
  __device__ __forceinline__ void gather(int64_t ib, double (&rs)[K]) {
    const int lane = threadIdx.x & 63;
    int32_t spins = 0;
    while (!faulted) {
      bool ready = true;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (ib + k < row1)
          for (int q = lane; q < gc; q += 64)
            ready &= (__hip_atomic_load(&part[(ib + k) * gs + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                      0xffull) == tag;
      if (__all(ready)) break;
      ++spins;
      if (spins > spin_limit ||
          ((spins & 15) == 0 && __hip_atomic_load(&ctl->fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        if (lane == 0) {
          __hip_atomic_store(&ctl->fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&ctl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        faulted = true;
      }
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double v = 0.0;
      if (ib + k < row1)
        for (int q = lane; q < gc; q += 64)
          v += fuse_value(__hip_atomic_load(&part[(ib + k) * gs + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      rs[k] = wave_sum(v);
    }
  }

  // Row sums of batch t from all partners (this wave's snapshot if every tag in it
  // is this pass's: a fixed butterfly within each row's gc lanes; else the gather),
  // b (partner 0, wave 0), and the batch's plan entries into cs.
  __device__ __forceinline__ void consume(int t, const f32x4 (&x)[K][Q], uint64_t x0, uint64_t x1) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t ib = row0 + static_cast<int64_t>(t) * K;
    double rs[K];
    const int g = 1 << glog;
    if (K == 2 && glog == 6 && __all((x0 & 0xffull) == tag) && __all((x1 & 0xffull) == tag)) {
      const double v0 = group_sum(lane < gc ? fuse_value(x0) : 0.0, 64);
      const double v1 = group_sum(lane < gc ? fuse_value(x1) : 0.0, 64);
      rs[0] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v0), 63),
                               __builtin_amdgcn_readlane(__double2loint(v0), 63));
      rs[K - 1] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v1), 63),
                                   __builtin_amdgcn_readlane(__double2loint(v1), 63));
    } else if ((K << glog) <= 64 && __all((x0 & 0xffull) == tag)) {
      const double v = group_sum((lane >> glog) < K && (lane & (g - 1)) < gc ? fuse_value(x0) : 0.0, g);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int last = (k + 1) * g - 1 < 64 ? (k + 1) * g - 1 : 63;
        rs[k] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), last),
                                 __builtin_amdgcn_readlane(__double2loint(v), last));
      }
    } else {
      gather(ib, rs);
    }
    // scale of 2^y to the plan after the b-update; kept in FP64 (as an FP32 factor its
    // rounding would shift every entry of the row the same way)
    double sg[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool valid = ib + k < row1;
      sg[k] = valid ? mu / rs[k] : 0.0;
      if (valid && c == 0 && wv == 0 && lane == 0) b[ib + k] = bold[(t & 3) * K + k] + eps * (log_mu - log(rs[k]));
    }
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      double *cp = cs + (u * 256 + threadIdx.x) * 4;
      double c4[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) c4[v] = cp[v];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int k = 0; k < K; ++k) c4[v] = fma(static_cast<double>(x[k][u][v]), sg[k], c4[v]);
#pragma unroll
      for (int v = 0; v < 4; ++v) cp[v] = c4[v];
    }
  }

  // One pipeline step: snapshot batch t's slots, load batch t+3 into w, produce
  // batch t+2 in y, consume batch t from x.  The compiler barriers keep the
  // snapshot ahead of the data loads, and the loads are unconditional (past the
  // group's end they re-read its last row; needs nb > 0): the same number of loads
  // on every path lets the wait for the snapshot leave them in flight.  red is
  // double-buffered by step parity: wave 0 may still read one step's partial sums
  // while faster waves write the next step's.
  __device__ __forceinline__ void step(int t, int nb, f32x4 (&x)[K][Q], double (&bx)[K], f32x4 (&y)[K][Q],
                                       double (&by)[K], f32x4 (&w)[K][Q], double (&bw)[K], double (&red)[2][K][4]) {
    uint64_t x0 = 0, x1 = 0;
    const int64_t ib = row0 + static_cast<int64_t>(t) * K;
    if ((K << glog) <= 64) {
      x0 = snap(ib);
    } else if (K == 2 && glog == 6) {
      x0 = snap_row(ib);
      x1 = snap_row(ib + 1);
    }
    asm volatile("" ::: "memory");
    load(t + 3, w, bw);
    asm volatile("" ::: "memory");
    if (t + 2 < nb) produce(t + 2, y, by, red[t & 1]);
    consume(t, x, x0, x1);
  }
};

// The single-pass iteration (b-update, then the column sums for the next
// a-update) over rows [row0, row1) of a row group and one column slice.  The
// grid is gr row groups x gc partners, all co-resident; with gr a multiple of 8
// the partners of a row group are consecutive on one XCD (workgroup w runs on XCD
// w mod 8), so their exchange stays in one L2.  Writes b (partner 0) and this
// group's column sums pcol[r][j] of the plan after the b-update.
template <int Q, int K>
__global__ __launch_bounds__(256, 2) void k_sink_fused(const float *__restrict__ C, int32_t n1, int32_t n2,
                                                       const double *__restrict__ bufA0,
                                                       const double *__restrict__ bufA1, int32_t cur,
                                                       double *__restrict__ b, double k2, double eps, double log_mu,
                                                       double mu, int32_t gc, int32_t glog, int32_t gr, uint32_t tag,
                                                       uint64_t *__restrict__ part, double *__restrict__ pcol,
                                                       SinkCtl *__restrict__ ctl, int32_t spin_limit) {
  if (ctl->done) return;
  const double *a = cur ? bufA1 : bufA0;
  const int w = blockIdx.x;
  int r, c;
  if (gr % 8 == 0) {
    const int l = w >> 3;
    r = (w & 7) * (gr >> 3) + l / gc;
    c = l % gc;
  } else {
    r = w / gc;
    c = w % gc;
  }
  __shared__ double ak[Q * 256 * 4];
  __shared__ double cs[Q * 256 * 4];
  __shared__ double red[2][K][4];
  __shared__ double bold[4 * K];
  FusePipe<Q, K> F;
  F.C = C;
  F.n2 = n2;
  F.k2 = k2;
  F.eps = eps;
  F.log_mu = log_mu;
  F.mu = mu;
  F.gc = gc;
  F.c = c;
  F.tag = tag;
  F.spin_limit = spin_limit;
  F.glog = glog;
  F.gs = fuse_stride(gc);
  F.row0 = static_cast<int64_t>(r) * n1 / gr;
  F.row1 = static_cast<int64_t>(r + 1) * n1 / gr;
  F.b = b;
  F.part = part;
  F.ctl = ctl;
  F.ak = ak;
  F.cs = cs;
  F.bold = bold;
  F.faulted = false;
  const int nb = static_cast<int>((F.row1 - F.row0 + K - 1) / K);
  const int nq = n2 >> 2;
  const int q0 = static_cast<int>(static_cast<int64_t>(c) * nq / gc);
  const int q1 = static_cast<int>(static_cast<int64_t>(c + 1) * nq / gc);
  bool qv[Q];
#pragma unroll
  for (int u = 0; u < Q; ++u) {
    const int q = q0 + static_cast<int>(threadIdx.x) + 256 * u;
    qv[u] = q < q1;
    F.jq[u] = 4 * (q < q1 ? q : (q1 > q0 ? q1 - 1 : 0));  // masked quads re-read a valid one
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      ak[(u * 256 + threadIdx.x) * 4 + v] = qv[u] ? a[F.jq[u] + v] * k2 : -INFINITY;
      cs[(u * 256 + threadIdx.x) * 4 + v] = 0.0;
    }
  }
  __syncthreads();
  if (nb > 0) {
    f32x4 x0[K][Q], x1[K][Q], x2[K][Q], x3[K][Q];
    double b0[K], b1[K], b2[K], b3[K];
    F.load(0, x0, b0);
    F.load(1, x1, b1);
    F.load(2, x2, b2);
    F.produce(0, x0, b0, red[0]);
    if (nb > 1) F.produce(1, x1, b1, red[1]);
    for (int t = 0; t < nb; t += 4) {
      F.step(t, nb, x0, b0, x2, b2, x3, b3, red);
      if (t + 1 >= nb) break;
      F.step(t + 1, nb, x1, b1, x3, b3, x0, b0, red);
      if (t + 2 >= nb) break;
      F.step(t + 2, nb, x2, b2, x0, b0, x1, b1, red);
      if (t + 3 >= nb) break;
      F.step(t + 3, nb, x3, b3, x1, b1, x2, b2, red);
    }
  }
#pragma unroll
  for (int u = 0; u < Q; ++u)
    if (qv[u])
#pragma unroll
      for (int v = 0; v < 4; ++v)
        pcol[static_cast<int64_t>(r) * n2 + F.jq[u] + v] = cs[(u * 256 + threadIdx.x) * 4 + v];
}

// Column sums of the plan after the b-update: fold the gr row-group sums of each
// column in order, form the candidate a_j (into the other buffer) and the column's
// marginal violation; k_error_finish then forms the total and applies the stop rule.
__global__ __launch_bounds__(256) void k_fused_merge(int32_t n2, int32_t gr, const double *__restrict__ pcol,
                                                     double *__restrict__ bufA0, double *__restrict__ bufA1,
                                                     int32_t cur, double eps, double log_nu, double nu,
                                                     double *__restrict__ errp, const SinkCtl *__restrict__ ctl) {
  if (ctl->done) return;
  const double *a = cur ? bufA1 : bufA0;
  double *an = cur ? bufA0 : bufA1;
  const int j = blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (j < n2) {
    double sum = 0.0;
    for (int q = 0; q < gr; ++q) sum += pcol[static_cast<int64_t>(q) * n2 + j];
    an[j] = a[j] + eps * (log_nu - log(sum));
    e = fabs(sum - nu);
  }
  block_error(e, errp);
}

// Grid of the single-pass iteration on the current device: gc partners per row,
// gr row groups, every workgroup co-resident (occupancy x compute units, looked up
// once per device).  FA_ERR_SHAPE when the shape or the device does not allow it.
struct FuseGrid {
  int gc, gr;
};

namespace {
constexpr int kMaxDev = 64;
std::mutex g_fuse_mu;
int g_fuse_slots[kMaxDev] = {};
}  // namespace

static int fuse_slots(int *slots) {
  int dev = -1;
  FA_HIP(hipGetDevice(&dev));
  FA_REQUIRE(dev >= 0 && dev < kMaxDev, FA_ERR_ARG, "single-pass Sinkhorn: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_fuse_mu);
  if (!g_fuse_slots[dev]) {
    int per_cu = 0, cus = 0, coop = 0;
    FA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(&k_sink_fused<kFuseQ, kFuseK>), 256, 0));
    FA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    FA_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    const int64_t n = coop ? static_cast<int64_t>(per_cu) * cus : 0;
    g_fuse_slots[dev] = static_cast<int>(n < kFuseMaxGrid ? n : kFuseMaxGrid);
    if (!g_fuse_slots[dev]) g_fuse_slots[dev] = -1;
  }
  *slots = g_fuse_slots[dev];
  return FA_OK;
}

static int fuse_grid(int32_t n1, int32_t n2, FuseGrid *g) {
  FA_REQUIRE(n1 > 0 && n2 > 0 && n2 % 4 == 0, FA_ERR_SHAPE,
             "single-pass Sinkhorn: n2 = %d must be a positive multiple of 4", n2);
  int slots = 0;
  FA_TRY(fuse_slots(&slots));
  const int gc = fuse_partners(n2);
  FA_REQUIRE(slots > 0 && gc <= slots && gc <= n2 / 4, FA_ERR_SHAPE,
             "single-pass Sinkhorn: %d partners per row do not fit %d co-resident workgroups", gc, slots);
  int64_t gr = slots / gc;
  const int64_t cap = fuse_groups_cap(n1, n2);  // also no more groups than batches of rows
  if (gr > cap) gr = cap;
  if (gr >= 8) gr -= gr % 8;
  // A pass takes as long as a row group needs for its rows.  The partners of a row
  // group share an XCD, so at most (slots / 8) / gc groups fit per XCD; where that
  // layout fills under 5/8 of the co-resident slots (33..39 partners: one group
  // per XCD), the two-pass form is faster and the single pass is not used.
  const int64_t xcd_groups = 8 * ((slots / 8) / gc);
  FA_REQUIRE(8 * xcd_groups * gc >= 5 * static_cast<int64_t>(slots), FA_ERR_SHAPE,
             "single-pass Sinkhorn: %d partners per row fill %lld of %d co-resident slots", gc,
             static_cast<long long>(xcd_groups * gc), slots);
  g->gc = gc;
  g->gr = static_cast<int>(gr);
  return FA_OK;
}

static std::atomic<int32_t> g_fuse_spin{kFuseSpinDefault};

int run_sinkhorn(const float *C, const float *Ct, int32_t n1, int32_t n2, double eps, double *a, double *b,
                 int32_t max_iter, double tol, int32_t check_every, int32_t *dev_iters, double *dev_err, SinkWs &w,
                 hipStream_t s, KTimer *tm) {
  SinkLayout L = sink_layout(n1, n2);
  SinkCtl *ctl = reinterpret_cast<SinkCtl *>(w.ctl);
  const double k2 = kLog2e / eps;
  const double log_nu = -log(static_cast<double>(n2)), nu = 1.0 / n2;
  const double log_mu = -log(static_cast<double>(n1));
  FA_LAUNCH(k_sink_reset, dim3(1), dim3(1), 0, s, ctl);
  const dim3 gcol(L.ncolblk, L.nsplit), gmerge(L.nmerge), grow(ceil_div(n1, kRowsPerWg));
  // Single-pass form: iterations 0 and 1 run the two passes (iteration 0's b-update
  // makes every row sum of the plan mu_i, which bounds the row sums the single pass
  // sees from iteration 2 on), then one pass per iteration.
  FuseGrid fg{0, 0};
  const bool fused = w.part != nullptr && max_iter >= 2 && fuse_grid(n1, n2, &fg) == FA_OK;
  // clear the exchange slots (tag 0 is never a pass's tag)
  if (fused)
    FA_TRY(launch_fill_f64(reinterpret_cast<double *>(w.part), static_cast<int64_t>(n1) * fuse_stride(fg.gc), 0.0, s));
  const double mu = 1.0 / n1;
  const int32_t spin = g_fuse_spin.load();
  for (int it = 0; it <= max_iter; ++it) {
    const int cur = it & 1;
    const int is_final = it == max_iter;
    const int is_check = it > 0 && (it % check_every == 0);
    if (fused && it >= 2) {
      const float *cC = C;
      int32_t cn1 = n1, cn2 = n2, ccur = cur, gc = fg.gc, gr = fg.gr, sp = spin, glog = 0;
      while ((1 << glog) < gc) ++glog;
      uint32_t tag = static_cast<uint32_t>((it - 2) % 255 + 1);  // consecutive passes never share a tag
      const double *ca0 = a, *ca1 = w.a_next;
      double *cb = b, *cpcol = w.pcol;
      uint64_t *cpart = w.part;
      double ck2 = k2, ceps = eps, clog_mu = log_mu, cmu = mu;
      SinkCtl *cctl = ctl;
      void *args[] = {&cC, &cn1, &cn2, &ca0, &ca1, &ccur, &cb, &ck2, &ceps, &clog_mu, &cmu, &gc, &glog, &gr, &tag,
                      &cpart, &cpcol, &cctl, &sp};
      FA_TIMED(tm, KK_FUSED, s,
               FA_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_sink_fused<kFuseQ, kFuseK>),
                                                 dim3(fg.gr * fg.gc), dim3(256), args, 0, s)));
      const int nm = ceil_div(n2, 256);
      FA_TIMED(tm, KK_COL_MERGE, s,
               FA_LAUNCH(k_fused_merge, dim3(nm), dim3(256), 0, s, n2, fg.gr, w.pcol, a, w.a_next, cur, eps, log_nu, nu,
                         w.errp, ctl));
      FA_TIMED(tm, KK_COL_MERGE, s,
               FA_LAUNCH(k_error_finish, dim3(1), dim3(256), 0, s, w.errp, nm, ctl, it, is_check, is_final, tol, cur,
                         dev_iters, dev_err));
      if (is_final) break;
      continue;
    }
    if (Ct) {
      const dim3 gct(L.ncolt);
      if (n1 % 4 == 0)
        FA_TIMED(tm, KK_COL_T, s,
                 FA_LAUNCH((k_lse_col_t<4, kColTRowsPerWg>), gct, dim3(256), 0, s, Ct, n1, n2, a, w.a_next, cur, b,
                           k2, eps, log_nu, nu, w.errp, ctl));
      else
        FA_TIMED(tm, KK_COL_T, s,
                 FA_LAUNCH((k_lse_col_t<1, kColTRowsPerWg>), gct, dim3(256), 0, s, Ct, n1, n2, a, w.a_next, cur, b,
                           k2, eps, log_nu, nu, w.errp, ctl));
      FA_TIMED(tm, KK_COL_MERGE, s,
               FA_LAUNCH(k_error_finish, dim3(1), dim3(256), 0, s, w.errp, L.ncolt, ctl, it, is_check, is_final, tol,
                         cur, dev_iters, dev_err));
    } else {
      if (L.V == 4)
        FA_TIMED(tm, KK_COL_PARTIAL, s,
                 FA_LAUNCH((k_lse_col_partial<4, kColRowsPerStep>), gcol, dim3(256), 0, s, C, n1, n2, a, w.a_next, cur, b, k2,
                           L.rows_per_split, w.pm, w.ps, ctl));
      else
        FA_TIMED(tm, KK_COL_PARTIAL, s,
                 FA_LAUNCH((k_lse_col_partial<1, kColRowsPerStep>), gcol, dim3(256), 0, s, C, n1, n2, a, w.a_next, cur, b, k2,
                           L.rows_per_split, w.pm, w.ps, ctl));
      FA_TIMED(tm, KK_COL_MERGE, s,
               FA_LAUNCH(k_lse_col_merge, gmerge, dim3(256), 0, s, n2, L.nsplit, w.pm, w.ps, a, w.a_next, cur, eps,
                         log_nu, nu, w.errp, ctl, it, is_check, is_final, tol, dev_iters, dev_err));
    }
    if (is_final) break;
    if (fused && it == 1) continue;  // iteration 2's b-update is the first single pass
    if (L.V == 4)
      FA_TIMED(tm, KK_ROW, s,
               FA_LAUNCH((k_lse_row<4, kRowsPerWg>), grow, dim3(256), 0, s, C, n1, n2, a, w.a_next, 1 - cur, b, k2, eps, log_mu,
                         ctl));
    else
      FA_TIMED(tm, KK_ROW, s,
               FA_LAUNCH((k_lse_row<1, kRowsPerWg>), grow, dim3(256), 0, s, C, n1, n2, a, w.a_next, 1 - cur, b, k2, eps, log_mu,
                         ctl));
  }
  FA_LAUNCH(k_final_a, dim3(ceil_div(n2, 256)), dim3(256), 0, s, a, w.a_next, n2, ctl, dev_iters, dev_err);
  return FA_OK;
}

// Plan S = exp2((a_j + b_i - C_ij) * log2(e)/eps), optional row argmax of the FP64 exponent.
// With truth/rank: the rank of each row's true partner t among the row's scores,
// 1 + #{j : y_ij > y_it} (the §4 ranking behind Hits@K and MRR), counted in the
// same pass on the FP64 exponents; y_it is formed with exactly the operations of
// the main loop, so the partner never counts itself.  t outside [0, n2) gives 0.
template <int V, typename TS>
__global__ __launch_bounds__(256) void k_plan(const float *__restrict__ C, int32_t n1, int32_t n2,
                                              const double *__restrict__ a, const double *__restrict__ b, double k2,
                                              TS *__restrict__ S, int32_t *__restrict__ argmax,
                                              const int32_t *__restrict__ truth, int32_t *__restrict__ rank) {
  constexpr int R = 4;
  const int i0 = blockIdx.x * R;
  double bk[R], best[R], yt[R];
  int bidx[R], tr[R], cnt[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    bk[r] = (i0 + r < n1) ? b[i0 + r] * k2 : 0.0;
    best[r] = -INFINITY;
    bidx[r] = 0x7fffffff;
    tr[r] = (truth && i0 + r < n1) ? truth[i0 + r] : -1;
    if (tr[r] >= n2) tr[r] = -1;
    // the score is two explicit fmas here and in the main loop, so the compiler
    // has no multiply-add left to contract differently in the two places
    yt[r] = tr[r] >= 0 ? fma(-static_cast<double>(C[static_cast<int64_t>(i0 + r) * n2 + tr[r]]), k2,
                             fma(a[tr[r]], k2, bk[r]))
                       : INFINITY;
    cnt[r] = 0;
  }
  for (int j = threadIdx.x * V; j < n2; j += 256 * V) {
    double aj[V];
#pragma unroll
    for (int v = 0; v < V; ++v) aj[v] = a[j + v];
    float cr[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) Vec<V>::load(C + static_cast<int64_t>(min(i0 + r, n1 - 1)) * n2 + j, cr[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (i0 + r >= n1) continue;
      const int64_t base = static_cast<int64_t>(i0 + r) * n2 + j;
      const float *c = cr[r];
      float sv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double y = fma(-static_cast<double>(c[v]), k2, fma(aj[v], k2, bk[r]));
        sv[v] = exp2_split(y);
        cnt[r] += y > yt[r];
        if (y > best[r]) {
          best[r] = y;
          bidx[r] = j + v;
        }
      }
      VStore<TS, V>::run(S + base, sv);
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (rank) {
    __shared__ int sc[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int c = cnt[r];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
      if (lane == 0) sc[r][w] = c;
    }
    __syncthreads();
    if (threadIdx.x < R && i0 + static_cast<int>(threadIdx.x) < n1) {
      const int r = threadIdx.x;
      rank[i0 + r] = tr[r] >= 0 ? 1 + ((sc[r][0] + sc[r][1]) + (sc[r][2] + sc[r][3])) : 0;
    }
  }
  if (!argmax) return;
  __shared__ double sb[R][4];
  __shared__ int si[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v = best[r];
    int id = bidx[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(v, o, 64);
      const int id2 = __shfl_xor(id, o, 64);
      if (v2 > v || (v2 == v && id2 < id)) {
        v = v2;
        id = id2;
      }
    }
    if (lane == 0) {
      sb[r][w] = v;
      si[r][w] = id;
    }
  }
  __syncthreads();
  if (threadIdx.x < R && i0 + static_cast<int>(threadIdx.x) < n1) {
    const int r = threadIdx.x;
    double v = sb[r][0];
    int id = si[r][0];
    for (int q = 1; q < 4; ++q)
      if (sb[r][q] > v || (sb[r][q] == v && si[r][q] < id)) {
        v = sb[r][q];
        id = si[r][q];
      }
    argmax[i0 + r] = id;
  }
}

int run_plan(const float *C, int32_t n1, int32_t n2, double eps, const double *a, const double *b, void *S,
             int32_t sdt, int32_t *argmax, const int32_t *truth, int32_t *rank, hipStream_t s, KTimer *tm) {
  if (n1 == 0 || n2 == 0) return FA_OK;
  const int tid = tm ? tm->begin(KK_PLAN, s) : -1;
  const double k2 = kLog2e / eps;
  const dim3 g(ceil_div(n1, 4));
  const bool v4 = n2 % 4 == 0;
  if (sdt == FA_BF16) {
    if (v4)
      FA_LAUNCH((k_plan<4, uint16_t>), g, dim3(256), 0, s, C, n1, n2, a, b, k2, static_cast<uint16_t *>(S), argmax, truth, rank);
    else
      FA_LAUNCH((k_plan<1, uint16_t>), g, dim3(256), 0, s, C, n1, n2, a, b, k2, static_cast<uint16_t *>(S), argmax, truth, rank);
  } else {
    if (v4)
      FA_LAUNCH((k_plan<4, float>), g, dim3(256), 0, s, C, n1, n2, a, b, k2, static_cast<float *>(S), argmax, truth, rank);
    else
      FA_LAUNCH((k_plan<1, float>), g, dim3(256), 0, s, C, n1, n2, a, b, k2, static_cast<float *>(S), argmax, truth, rank);
  }
  if (tm) tm->end(tid, s);
  return FA_OK;
}

int sinkhorn_fault(const SinkWs &w, hipStream_t s, int32_t *fault) {
  SinkCtl c;
  FA_HIP(hipMemcpyAsync(&c, w.ctl, sizeof c, hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  *fault = c.fault;
  return FA_OK;
}

}  // namespace fa

using namespace fa;

extern "C" size_t fa_sinkhorn_workspace_size(int32_t n1, int32_t n2) {
  if (n1 <= 0 || n2 <= 0) return 256;
  return sinkhorn_ws_bytes(n1, n2, false);
}

extern "C" size_t fa_sinkhorn_fused_workspace_size(int32_t n1, int32_t n2) {
  if (n1 <= 0 || n2 <= 0) return 256;
  return sinkhorn_ws_bytes(n1, n2, true);
}

extern "C" int fa_sinkhorn_fused_grid(int32_t n1, int32_t n2, int32_t *gr, int32_t *gc) {
  FA_REQUIRE(gr && gc, FA_ERR_ARG, "fa_sinkhorn_fused_grid: null output");
  FuseGrid g;
  FA_TRY(fuse_grid(n1, n2, &g));
  *gr = g.gr;
  *gc = g.gc;
  return FA_OK;
}

extern "C" int32_t fa_set_sync_spin_limit(int32_t polls) {
  return g_fuse_spin.exchange(polls < 1 ? 1 : polls);
}

extern "C" int fa_sinkhorn_fused(const float *C, int32_t n1, int32_t n2, double eps, double *a, double *b,
                                 int32_t max_iter, double tol, int32_t check_every, int32_t *dev_iters,
                                 double *dev_err, int32_t *host_iters, double *host_err, void *ws, size_t ws_bytes,
                                 void *stream) {
  FA_REQUIRE(n1 > 0 && n2 > 0, FA_ERR_SHAPE, "fa_sinkhorn_fused: n1 = %d, n2 = %d must be positive", n1, n2);
  FA_REQUIRE(eps > 0 && max_iter >= 0 && check_every >= 1 && tol >= 0, FA_ERR_ARG,
             "fa_sinkhorn_fused: need eps > 0, max_iter >= 0, check_every >= 1, tol >= 0");
  FA_REQUIRE(C && a && b && dev_iters && dev_err, FA_ERR_ARG, "fa_sinkhorn_fused: null pointer");
  const size_t need = sinkhorn_ws_bytes(n1, n2, true);
  FA_REQUIRE(ws && ws_bytes >= need, FA_ERR_WORKSPACE, "fa_sinkhorn_fused: workspace %zu < %zu", ws_bytes, need);
  Carver cv(ws, ws_bytes);
  SinkWs w;
  FA_TRY(carve_sinkhorn(cv, n1, n2, w, true));
  hipStream_t s = static_cast<hipStream_t>(stream);
  FA_TRY(run_sinkhorn(C, nullptr, n1, n2, eps, a, b, max_iter, tol, check_every, dev_iters, dev_err, w, s));
  if (host_iters || host_err) {
    int32_t fault = 0;
    FA_TRY(sinkhorn_fault(w, s, &fault));
    FA_REQUIRE(!fault, FA_ERR_SYNC, "fa_sinkhorn_fused: a partner wait of the single pass gave up");
    if (host_iters) FA_HIP(hipMemcpy(host_iters, dev_iters, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (host_err) FA_HIP(hipMemcpy(host_err, dev_err, sizeof(double), hipMemcpyDeviceToHost));
  }
  return FA_OK;
}

extern "C" int fa_sinkhorn(const float *C, const float *Ct, int32_t n1, int32_t n2, double eps, double *a, double *b,
                           int32_t max_iter, double tol, int32_t check_every, int32_t *dev_iters, double *dev_err,
                           int32_t *host_iters, double *host_err, void *ws, size_t ws_bytes, void *stream) {
  FA_REQUIRE(n1 > 0 && n2 > 0, FA_ERR_SHAPE, "fa_sinkhorn: n1 = %d, n2 = %d must be positive", n1, n2);
  FA_REQUIRE(eps > 0 && max_iter >= 0 && check_every >= 1 && tol >= 0, FA_ERR_ARG,
             "fa_sinkhorn: need eps > 0, max_iter >= 0, check_every >= 1, tol >= 0");
  FA_REQUIRE(C && a && b && dev_iters && dev_err, FA_ERR_ARG, "fa_sinkhorn: null pointer");
  FA_REQUIRE(ws && ws_bytes >= sinkhorn_ws_bytes(n1, n2, false), FA_ERR_WORKSPACE,
             "fa_sinkhorn: workspace %zu < %zu", ws_bytes, sinkhorn_ws_bytes(n1, n2, false));
  Carver cv(ws, ws_bytes);
  SinkWs w;
  FA_TRY(carve_sinkhorn(cv, n1, n2, w, false));
  hipStream_t s = static_cast<hipStream_t>(stream);
  FA_TRY(run_sinkhorn(C, Ct, n1, n2, eps, a, b, max_iter, tol, check_every, dev_iters, dev_err, w, s));
  if (host_iters || host_err) {
    FA_HIP(hipStreamSynchronize(s));
    if (host_iters) FA_HIP(hipMemcpy(host_iters, dev_iters, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (host_err) FA_HIP(hipMemcpy(host_err, dev_err, sizeof(double), hipMemcpyDeviceToHost));
  }
  return FA_OK;
}

extern "C" int fa_plan(const float *C, int32_t n1, int32_t n2, double eps, const double *a, const double *b, void *S,
                       int32_t s_dtype, int32_t *argmax, const int32_t *truth, int32_t *rank, void *stream) {
  FA_REQUIRE(n1 >= 0 && n2 >= 0 && eps > 0, FA_ERR_ARG, "fa_plan: bad sizes or eps");
  FA_REQUIRE(s_dtype == FA_F32 || s_dtype == FA_BF16, FA_ERR_ARG, "fa_plan: s_dtype %d", s_dtype);
  if (n1 == 0 || n2 == 0) return FA_OK;
  FA_REQUIRE(C && a && b && S, FA_ERR_ARG, "fa_plan: null pointer");
  FA_REQUIRE((truth == nullptr) == (rank == nullptr), FA_ERR_ARG, "fa_plan: truth and rank go together");
  return run_plan(C, n1, n2, eps, a, b, S, s_dtype, argmax, truth, rank, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- no allocation

// Scratch of fa_sinkhorn_noalloc: one copy per GPU, held until the process ends.
// Host code reaches it only through the address hipGetSymbolAddress returns for
// the current device (the array's name on the host is not a device address).
static __device__ __align__(256) unsigned char scratch[FA_SINKHORN_NOALLOC_SCRATCH];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's scratch array, looked up once per device.
int device_scratch(void **out) {
  int dev = -1;
  FA_HIP(hipGetDevice(&dev));
  FA_REQUIRE(dev >= 0 && dev < kMaxDevices, FA_ERR_ARG, "fa_sinkhorn_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    FA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    FA_REQUIRE(ptr != nullptr, FA_ERR_HIP, "fa_sinkhorn_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FA_OK;
}
}  // namespace

extern "C" size_t fa_sinkhorn_noalloc_need(int32_t n1, int32_t n2, int32_t transposed) {
  if (n1 <= 0 || n2 <= 0) return 0;
  return sink_scratch_bytes(n1, n2, transposed != 0 ? SINK_T_ONLY : SINK_TWO_PASS);
}

extern "C" int fa_sinkhorn_noalloc(const float *C, const float *Ct, int32_t n1, int32_t n2, double eps, double *a,
                                   double *b, int32_t max_iter, double tol, int32_t check_every, int32_t *dev_iters,
                                   double *dev_err, void *stream) {
  FA_REQUIRE(n1 > 0 && n2 > 0, FA_ERR_SHAPE, "fa_sinkhorn_noalloc: n1 = %d, n2 = %d must be positive", n1, n2);
  FA_REQUIRE(eps > 0 && max_iter >= 0 && check_every >= 1 && tol >= 0, FA_ERR_ARG,
             "fa_sinkhorn_noalloc: need eps > 0, max_iter >= 0, check_every >= 1, tol >= 0");
  FA_REQUIRE(C && a && b && dev_iters && dev_err, FA_ERR_ARG, "fa_sinkhorn_noalloc: null pointer");
  const bool tr = Ct != nullptr;
  const size_t need = sink_scratch_bytes(n1, n2, tr ? SINK_T_ONLY : SINK_TWO_PASS);
  FA_REQUIRE(need <= FA_SINKHORN_NOALLOC_SCRATCH, FA_ERR_SHAPE,
             "fa_sinkhorn_noalloc: %d x %d needs %zu bytes of scratch %s, the static array holds %zu "
             "(use fa_sinkhorn with a workspace)",
             n1, n2, need, tr ? "with C^T" : "without C^T (column partials)",
             static_cast<size_t>(FA_SINKHORN_NOALLOC_SCRATCH));
  void *ptr = nullptr;
  FA_TRY(device_scratch(&ptr));
  Carver cv(ptr, FA_SINKHORN_NOALLOC_SCRATCH);
  SinkWs w;
  FA_TRY(carve_sink(cv, n1, n2, w, tr ? SINK_T_ONLY : SINK_TWO_PASS));
  return run_sinkhorn(C, Ct, n1, n2, eps, a, b, max_iter, tol, check_every, dev_iters, dev_err, w,
                      static_cast<hipStream_t>(stream));
}
