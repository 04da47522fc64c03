/* Host-side driver for the address/undefined-behaviour sanitizer build of the
 * library (host code instrumented, device code not).  Every call here returns
 * before any kernel is launched: the CSR builder of the graph input (checked
 * against a dense adjacency matrix), the workspace and scratch size queries
 * over a grid of shapes and options, and the argument and workspace checks of
 * the entry points.  Prints one line per group; exits non-zero on the first
 * wrong result (the sanitizers abort on their own findings). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fastalign.h"

#define CHECK(cond)                                                          \
  do {                                                                       \
    if (!(cond)) {                                                           \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);     \
      exit(1);                                                               \
    }                                                                        \
  } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void) { /* splitmix64 */
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

/* Random edge list with self-loops and repeated edges; the CSR must equal the
 * symmetrised, loop-free adjacency matrix row by row. */
static void csr_case(int32_t n, int64_t m) {
  int64_t *e = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 2));
  unsigned char *adj = (unsigned char *)calloc((size_t)n * (size_t)n + 1, 1);
  for (int64_t k = 0; k < m; ++k) {
    int64_t u = (int64_t)(next_u64() % (uint64_t)n), v = (int64_t)(next_u64() % (uint64_t)n);
    if (k % 7 == 3) v = u;                        /* a loop */
    if (k % 11 == 5 && k > 0) { u = e[2 * k - 1]; v = e[2 * k - 2]; } /* the previous edge reversed */
    e[2 * k] = u;
    e[2 * k + 1] = v;
    if (u != v) adj[u * n + v] = adj[v * n + u] = 1;
  }
  int64_t want = 0;
  for (int64_t i = 0; i < (int64_t)n * n; ++i) want += adj[i];
  int64_t *rowptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t nnz = -1;
  /* capacity one short: rowptr and nnz are valid, colidx untouched */
  if (want > 0) {
    int32_t *small = (int32_t *)malloc(sizeof(int32_t) * (size_t)want);
    CHECK(fa_csr_build(n, m, e, rowptr, small, want - 1, &nnz) == FA_ERR_SHAPE);
    CHECK(nnz == want && rowptr[n] == want);
    CHECK(strlen(fa_last_error()) > 0);
    free(small);
  }
  int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(want + 1));
  nnz = -1;
  CHECK(fa_csr_build(n, m, e, rowptr, col, want, &nnz) == FA_OK);
  CHECK(nnz == want && rowptr[0] == 0 && rowptr[n] == want);
  for (int32_t i = 0; i < n; ++i) {
    int64_t k = rowptr[i];
    for (int32_t j = 0; j < n; ++j)
      if (adj[(int64_t)i * n + j]) {
        CHECK(k < rowptr[i + 1] && col[k] == j);
        ++k;
      }
    CHECK(k == rowptr[i + 1]);
  }
  free(col);
  free(rowptr);
  free(adj);
  free(e);
}

static void csr_group(void) {
  int64_t rowptr[8], nnz = -1;
  int32_t col[8];
  CHECK(fa_csr_build(0, 0, NULL, rowptr, NULL, 0, &nnz) == FA_OK && nnz == 0 && rowptr[0] == 0);
  CHECK(fa_csr_build(3, 0, NULL, rowptr, NULL, 0, &nnz) == FA_OK && nnz == 0 && rowptr[3] == 0);
  const int64_t loops[] = {0, 0, 2, 2};
  CHECK(fa_csr_build(3, 2, loops, rowptr, NULL, 0, &nnz) == FA_OK && nnz == 0);
  const int64_t bad_hi[] = {0, 3};
  CHECK(fa_csr_build(3, 1, bad_hi, rowptr, col, 8, &nnz) == FA_ERR_ARG);
  const int64_t bad_lo[] = {-1, 1};
  CHECK(fa_csr_build(3, 1, bad_lo, rowptr, col, 8, &nnz) == FA_ERR_ARG);
  CHECK(fa_csr_build(-1, 0, NULL, rowptr, col, 8, &nnz) == FA_ERR_ARG);
  CHECK(fa_csr_build(3, -1, NULL, rowptr, col, 8, &nnz) == FA_ERR_ARG);
  CHECK(fa_csr_build(3, 1, NULL, rowptr, col, 8, &nnz) == FA_ERR_ARG);
  CHECK(fa_csr_build(3, 0, NULL, NULL, col, 8, &nnz) == FA_ERR_ARG);
  const int64_t one[] = {0, 1};
  CHECK(fa_csr_build(3, 1, one, rowptr, NULL, 8, &nnz) == FA_ERR_ARG);
  static const int32_t ns[] = {1, 2, 5, 17, 64, 300};
  static const int64_t ms[] = {1, 3, 20, 100, 900, 6000};
  for (int c = 0; c < 6; ++c) csr_case(ns[c], ms[c]);
  printf("csr: ok\n");
}

/* Size queries: positive, monotone in the sizes, and zero for shapes they refuse. */
static void size_group(void) {
  fa_params p;
  fa_default_params(&p);
  CHECK(p.eps > 0 && p.outer_iters > 0 && p.inner_iters > 0 && p.check_every >= 1);
  static const int32_t n1s[] = {1, 7, 256, 1000, 4099, 120000};
  static const int32_t n2s[] = {1, 9, 255, 900, 4097, 110000};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      int32_t n1 = n1s[i], n2 = n2s[j];
      CHECK(fa_sinkhorn_workspace_size(n1, n2) > 0);
      CHECK(fa_sinkhorn_fused_workspace_size(n1, n2) > fa_sinkhorn_workspace_size(n1, n2));
      CHECK(fa_sinkhorn_noalloc_need(n1, n2, 1) > 0);
      CHECK(fa_sinkhorn_noalloc_need(n1, n2, 0) >= fa_sinkhorn_noalloc_need(n1, n2, 1));
      for (int dt = 0; dt < 2; ++dt) {
        int32_t plan = dt ? FA_BF16 : FA_F32;
        CHECK(fa_cost_workspace_size(n1, n2, plan, 0) > 0);
        CHECK(fa_cost_workspace_size(n1, n2, plan, 64) > 0);
      }
      for (int opt = 0; opt < 32; ++opt) {
        fa_params q = p;
        q.plan_dtype = (opt & 1) ? FA_BF16 : FA_F32;
        q.feat_dtype = (opt & 2) ? FA_BF16 : FA_F32;
        q.transpose_cost = (opt & 4) ? 1 : 0;
        q.plan_in_ct = (opt & 8) && q.transpose_cost;
        q.warm_start = (opt & 16) ? 1 : 0;
        q.sink_fused = (opt & 1) ^ ((opt >> 2) & 1);
        for (int ds = 0; ds < 3; ++ds) {
          q.dual_start = ds;
          size_t w = fa_align_workspace_size(n1, n2, 32, 10, 8LL * n1, 8LL * n2, &q);
          size_t w2 = fa_align_workspace_size(n1, n2, 64, 20, 16LL * n1, 16LL * n2, &q);
          CHECK(w > 0 && w2 >= w);
        }
      }
    }
  CHECK(fa_sinkhorn_noalloc_need(0, 10, 1) == 0);
  CHECK(fa_align_workspace_size(0, 10, 4, 1, 1, 1, &p) == 0);
  CHECK(fa_align_workspace_size(10, 10, -1, 1, 1, 1, &p) == 0);
  CHECK(fa_align_workspace_size(10, 10, 4, 1, 1, 1, NULL) == 0);
  CHECK(fa_mlp_param_count() > 0 && fa_node_feature_dim() > 0);
  CHECK(fa_mlp_act_floats(1000) >= fa_mlp_act_floats(10));
  CHECK(fa_node_features_workspace_size(1000) > 0);
  printf("sizes: ok\n");
}

/* A small valid pair of host CSRs (a ring and a path) for the argument checks. */
static int64_t rp1[65], rp2[49];
static int32_t ci1[256], ci2[256];
static fa_csr g1, g2;
static void make_graphs(void) {
  int64_t e1[128], e2[96], nnz = 0;
  for (int i = 0; i < 64; ++i) { e1[2 * i] = i; e1[2 * i + 1] = (i + 1) % 64; }
  for (int i = 0; i < 47; ++i) { e2[2 * i] = i; e2[2 * i + 1] = i + 1; }
  CHECK(fa_csr_build(64, 64, e1, rp1, ci1, 256, &nnz) == FA_OK && nnz == 128);
  g1.n = 64; g1.nnz = nnz; g1.rowptr = rp1; g1.colidx = ci1;
  CHECK(fa_csr_build(48, 47, e2, rp2, ci2, 256, &nnz) == FA_OK && nnz == 94);
  g2.n = 48; g2.nnz = nnz; g2.rowptr = rp2; g2.colidx = ci2;
}

static int is_refusal(int rc) { return rc == FA_ERR_ARG || rc == FA_ERR_SHAPE || rc == FA_ERR_CSR; }

static void arg_group(void) {
  make_graphs();
  fa_params p;
  fa_default_params(&p);
  fa_stats st;
  memset(&st, 0, sizeof st);
  float dummy[4];
  double da[4];
  int32_t di[4];
  /* Top-k: k outside [1, min(64, n2)] and bad shapes */
  CHECK(fa_plan_topk(NULL, 4, 8, 0.1, NULL, NULL, 0, NULL, NULL, NULL) == FA_ERR_ARG);
  CHECK(fa_plan_topk(NULL, 4, 8, 0.1, NULL, NULL, 9, NULL, NULL, NULL) == FA_ERR_ARG);
  CHECK(fa_plan_topk(NULL, 4, 100, 0.1, NULL, NULL, 65, NULL, NULL, NULL) == FA_ERR_ARG);
  /* Sinkhorn: sizes, eps, workspace */
  CHECK(is_refusal(fa_sinkhorn(dummy, NULL, 0, 4, 0.1, da, da, 10, 0, 1, di, da, NULL, NULL, NULL, 0, NULL)));
  CHECK(is_refusal(fa_sinkhorn(dummy, NULL, 4, 4, -1.0, da, da, 10, 0, 1, di, da, NULL, NULL, NULL, 0, NULL)));
  CHECK(fa_sinkhorn(dummy, NULL, 4, 4, 0.1, da, da, 10, 0, 1, di, da, NULL, NULL, NULL, 0, NULL) ==
        FA_ERR_WORKSPACE);
  CHECK(fa_sinkhorn_noalloc(dummy, NULL, 64, 3000000, 0.1, da, da, 10, 0, 1, di, da, NULL) == FA_ERR_SHAPE);
  /* single pass: sizes, eps, pointers, workspace; its grid needs n2 % 4 == 0 */
  CHECK(is_refusal(fa_sinkhorn_fused(dummy, 0, 4, 0.1, da, da, 10, 0, 1, di, da, NULL, NULL, NULL, 0, NULL)));
  CHECK(is_refusal(fa_sinkhorn_fused(dummy, 4, 4, 0.0, da, da, 10, 0, 1, di, da, NULL, NULL, NULL, 0, NULL)));
  CHECK(is_refusal(fa_sinkhorn_fused(NULL, 4, 4, 0.1, da, da, 10, 0, 1, di, da, NULL, NULL, NULL, 0, NULL)));
  CHECK(fa_sinkhorn_fused(dummy, 4, 4, 0.1, da, da, 10, 0, 1, di, da, NULL, NULL, NULL, 0, NULL) == FA_ERR_WORKSPACE);
  int32_t gr = -1, gc = -1;
  CHECK(fa_sinkhorn_fused_grid(10, 6, &gr, &gc) == FA_ERR_SHAPE && gr == -1);
  CHECK(fa_sinkhorn_fused_grid(10, 8, NULL, &gc) == FA_ERR_ARG);
  const int32_t prev = fa_set_sync_spin_limit(0);   /* clamped to one poll */
  CHECK(prev >= 1 && fa_set_sync_spin_limit(prev) == 1);
  /* End to end: parameter checks, then the workspace check */
  fa_params q = p;
  q.eps = 0;
  CHECK(fa_align(&g1, &g2, NULL, NULL, 0, NULL, 0, &q, NULL, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, NULL, 0,
                 NULL) == FA_ERR_ARG);
  q = p; q.dual_start = 3;
  CHECK(fa_align(&g1, &g2, NULL, NULL, 0, NULL, 0, &q, NULL, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, NULL, 0,
                 NULL) == FA_ERR_ARG);
  q = p; q.warm_probe = -1;
  CHECK(fa_align(&g1, &g2, NULL, NULL, 0, NULL, 0, &q, NULL, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, NULL, 0,
                 NULL) == FA_ERR_ARG);
  q = p; q.transpose_cost = 0; q.plan_in_ct = 1;
  CHECK(fa_align(&g1, &g2, NULL, NULL, 0, NULL, 0, &q, NULL, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, NULL, 0,
                 NULL) == FA_ERR_ARG);
  q = p; q.sink_fused = 1; q.transpose_cost = 0; q.plan_in_ct = 1;
  CHECK(fa_align(&g1, &g2, NULL, NULL, 0, NULL, 0, &q, NULL, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, NULL, 0,
                 NULL) == FA_ERR_ARG);
  q = p; q.check_every = 0;
  CHECK(fa_align(&g1, &g2, NULL, NULL, 0, NULL, 0, &q, NULL, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, NULL, 0,
                 NULL) == FA_ERR_ARG);
  fa_csr broken = g1;
  broken.rowptr = NULL;
  CHECK(is_refusal(fa_align(&broken, &g2, NULL, NULL, 0, NULL, 0, &p, NULL, dummy, da, da, di, NULL, NULL, 0, NULL,
                            NULL, &st, NULL, 0, NULL)));
  broken = g1;
  broken.n = -5;
  CHECK(is_refusal(fa_align(&broken, &g2, NULL, NULL, 0, NULL, 0, &p, NULL, dummy, da, da, di, NULL, NULL, 0, NULL,
                            NULL, &st, NULL, 0, NULL)));
  size_t need = fa_align_workspace_size(g1.n, g2.n, 0, 0, g1.nnz, g2.nnz, &p);
  CHECK(need > 0);
  void *ws = malloc(need);
  CHECK(fa_align(&g1, &g2, NULL, NULL, 0, NULL, 0, &p, NULL, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, ws,
                 need - 1, NULL) == FA_ERR_WORKSPACE);
  CHECK(fa_align_begin(&g1, &g2, NULL, NULL, 0, NULL, 0, &p, dummy, da, da, &st, ws, need - 1, NULL) ==
        FA_ERR_WORKSPACE);
  CHECK(fa_align_step(&g1, &g2, 0, 0, &p, NULL, 0, dummy, da, da, di, NULL, NULL, &st, NULL, 0, NULL) ==
        FA_ERR_WORKSPACE);
  CHECK(fa_align_end(&g1, &g2, 0, 0, &p, 0, dummy, da, da, di, NULL, NULL, 0, NULL, NULL, &st, NULL, 0, NULL) ==
        FA_ERR_WORKSPACE);
  free(ws);
  CHECK(strlen(fa_last_error()) > 0);
  printf("arguments: ok\n");
}

int main(void) {
  csr_group();
  size_group();
  arg_group();
  return 0;
}
