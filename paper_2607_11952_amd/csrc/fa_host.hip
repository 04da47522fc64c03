// Host-side pieces of the ABI: error text, defaults, device check, CSR build.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fa_common.h"

namespace fa {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

}  // namespace fa

extern "C" const char *fa_last_error(void) { return fa::g_err; }

extern "C" void fa_default_params(fa_params *p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->eps = 0.05;
  p->alpha = 0.5;
  p->beta = 0.15;
  p->lambda_e = 1.0;
  p->lambda_n = 1.0;
  p->lambda_a = 1.0;
  p->lambda_p = p->eps;
  p->eps_anchor = p->eps;
  p->delta_nbr = 1e-30;
  p->tol = 0.0;
  p->k_r = 10;
  p->k_node = 1;
  p->outer_iters = 10;
  p->inner_iters = 50;
  p->check_every = 1;
  p->plan_dtype = FA_F32;
  p->feat_dtype = FA_F32;
  p->feat_l2norm = 1;
  p->warm_start = 0;
  p->chunk_rows = 0;
  p->profile = 0;
  p->dual_start = FA_START_ZERO;
  p->transpose_cost = 0;
  p->plan_in_ct = 0;
  p->warm_fallback = 1;
  p->warm_probe = 0;
  p->sink_fused = 1;
}

extern "C" int fa_device_check(void) {
  int dev = 0;
  FA_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  FA_HIP(hipGetDeviceProperties(&prop, dev));
  FA_REQUIRE(strncmp(prop.gcnArchName, "gfx950", 6) == 0, FA_ERR_DEVICE,
             "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
  return FA_OK;
}

// Counting sort by row, then sort + deduplicate each row.  Written independently
// of any other CSR builder; the result is unique (sorted, duplicate-free rows).
extern "C" int fa_csr_build(int32_t n, int64_t m, const int64_t *edges, int64_t *rowptr,
                            int32_t *colidx, int64_t cap, int64_t *nnz_out) {
  FA_REQUIRE(n >= 0 && m >= 0, FA_ERR_ARG, "fa_csr_build: negative size (n=%d, m=%lld)", n,
             (long long)m);
  FA_REQUIRE(rowptr != nullptr, FA_ERR_ARG, "fa_csr_build: null rowptr_out");
  FA_REQUIRE(m == 0 || edges != nullptr, FA_ERR_ARG, "fa_csr_build: null edge list");
  for (int64_t e = 0; e < m; ++e) {
    int64_t u = edges[2 * e], v = edges[2 * e + 1];
    FA_REQUIRE(u >= 0 && u < n && v >= 0 && v < n, FA_ERR_ARG,
               "fa_csr_build: edge %lld = (%lld, %lld) out of range for n = %d", (long long)e,
               (long long)u, (long long)v, n);
  }
  std::vector<int64_t> start(static_cast<size_t>(n) + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    int64_t u = edges[2 * e], v = edges[2 * e + 1];
    if (u == v) continue;
    start[u + 1]++;
    start[v + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) start[i + 1] += start[i];
  std::vector<int32_t> bucket(static_cast<size_t>(start[n]));
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  for (int64_t e = 0; e < m; ++e) {
    int64_t u = edges[2 * e], v = edges[2 * e + 1];
    if (u == v) continue;
    bucket[fill[u]++] = static_cast<int32_t>(v);
    bucket[fill[v]++] = static_cast<int32_t>(u);
  }
  int64_t nnz = 0;
  rowptr[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    auto b = bucket.begin() + start[i], en = bucket.begin() + start[i + 1];
    std::sort(b, en);
    int64_t kept = std::unique(b, en) - b;
    nnz += kept;
    rowptr[i + 1] = nnz;
  }
  if (nnz_out) *nnz_out = nnz;
  FA_REQUIRE(nnz <= cap, FA_ERR_SHAPE, "fa_csr_build: capacity %lld < nnz %lld", (long long)cap,
             (long long)nnz);
  FA_REQUIRE(nnz == 0 || colidx != nullptr, FA_ERR_ARG, "fa_csr_build: null colidx_out");
  for (int32_t i = 0; i < n; ++i) {
    int64_t kept = rowptr[i + 1] - rowptr[i];
    std::copy(bucket.begin() + start[i], bucket.begin() + start[i] + kept, colidx + rowptr[i]);
  }
  return FA_OK;
}
