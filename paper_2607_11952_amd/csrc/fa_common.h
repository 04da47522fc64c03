// Internal helpers shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "fastalign.h"

namespace fa {

void set_error(const char *fmt, ...);

#define FA_HIP(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      ::fa::set_error("%s failed: %s", #x, hipGetErrorString(e_));                  \
      return FA_ERR_HIP;                                                            \
    }                                                                               \
  } while (0)

#define FA_REQUIRE(cond, code, ...)                                                 \
  do {                                                                              \
    if (!(cond)) {                                                                  \
      ::fa::set_error(__VA_ARGS__);                                                 \
      return code;                                                                  \
    }                                                                               \
  } while (0)

#define FA_TRY(x)                                                                   \
  do {                                                                              \
    int s_ = (x);                                                                   \
    if (s_ < 0) return s_;                                                          \
  } while (0)

// Launch and check that the launch itself was accepted.
// A dispatch counts its work-items per dimension in 32 bits: a launch past 2^32
// work-items in one dimension does not fail, it covers only part of the range.
// Every launch is checked here; element-wise kernels over n1 * n2 entries use
// grid-stride loops on a capped grid (stride_grid) instead.
#define FA_LAUNCH(kernel, grid, block, shmem, stream, ...)                          \
  do {                                                                              \
    const dim3 fa_g_ = (grid), fa_b_ = (block);                                     \
    FA_REQUIRE(static_cast<uint64_t>(fa_g_.x) * fa_b_.x < (1ull << 32) &&           \
                   static_cast<uint64_t>(fa_g_.y) * fa_b_.y < (1ull << 32) &&       \
                   static_cast<uint64_t>(fa_g_.z) * fa_b_.z < (1ull << 32),         \
               FA_ERR_SHAPE, "launch of %s exceeds 2^32 work-items in one dimension", \
               #kernel);                                                            \
    hipLaunchKernelGGL(kernel, fa_g_, fa_b_, shmem, stream, __VA_ARGS__);           \
    FA_HIP(hipGetLastError());                                                      \
  } while (0)

constexpr double kLog2e = 1.4426950408889634073599246810019;
constexpr double kLn2 = 0.69314718055994530941723212145818;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Simple bump allocator over a caller workspace.
struct Carver {
  char *base;
  size_t cap;
  size_t off = 0;
  bool ok = true;
  Carver(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
  template <typename T>
  T *take(size_t count) {
    size_t start = align_up(off, 256);
    size_t bytes = align_up(count * sizeof(T), 256);
    off = start + bytes;
    if (!base || off > cap) {
      ok = false;
      return nullptr;
    }
    return reinterpret_cast<T *>(base + start);
  }
};

// Size-only twin of Carver for the *_workspace_size queries.
struct Sizer {
  size_t off = 0;
  template <typename T>
  void take(size_t count) {
    off = align_up(off, 256) + align_up(count * sizeof(T), 256);
  }
};

// ---------------------------------------------------------------- bf16

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
#else
  uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
#endif
}

// Round to nearest even; NaN stays a quiet NaN.
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t u = __float_as_uint(f);
#else
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
#endif
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

template <typename T>
__device__ inline void store_from_f32(T *p, int64_t i, float v);
template <>
__device__ inline void store_from_f32<float>(float *p, int64_t i, float v) { p[i] = v; }
template <>
__device__ inline void store_from_f32<uint16_t>(uint16_t *p, int64_t i, float v) { p[i] = f32_to_bf16(v); }

// Streaming (non-temporal) accesses for dense n1 x n2 operands that are touched
// once per pass: at production sizes they cannot stay in L2 or MALL, so their
// lines are marked to be evicted first and leave the caches to the dual vectors,
// neighbour lists and gathered rows that are reused.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ inline float ld_stream(const float *p) { return __builtin_nontemporal_load(p); }
__device__ inline f32x4 ld_stream4(const float *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
}
__device__ inline void st_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ inline void st_stream(uint16_t *p, float v) { __builtin_nontemporal_store(f32_to_bf16(v), p); }

// V consecutive floats of a streamed row (V = 1, 4, 8).
template <int V>
struct Vec;
template <>
struct Vec<1> {
  static __device__ inline void load(const float *p, float *o) { o[0] = ld_stream(p); }
};
template <>
struct Vec<4> {
  static __device__ inline void load(const float *p, float *o) {
    const f32x4 t = ld_stream4(p);
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
  }
};

template <>
struct Vec<8> {
  static __device__ inline void load(const float *p, float *o) {
    const f32x4 t = ld_stream4(p), u = ld_stream4(p + 4);
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
    o[4] = u.x;
    o[5] = u.y;
    o[6] = u.z;
    o[7] = u.w;
  }
};

// 2^y for an FP64 exponent: integer part exact (ldexp), fraction through FP32 exp2.
__device__ inline float exp2_split(double y) {
  if (!(y > -1000.0)) return 0.0f;
  if (y > 200.0) return INFINITY;
  const double fl = floor(y);
  return ldexpf(exp2f(static_cast<float>(y - fl)), static_cast<int>(fl));
}

// ---------------------------------------------------------------- reductions

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Merge two log2-domain partial sums (m, s) meaning s * 2^m.
__device__ inline void lse2_merge(double &m, double &s, double m2, double s2) {
  if (m2 > m) {
    s = s * exp2(m - m2) + s2;
    m = m2;
  } else if (m2 > -INFINITY) {
    s = s + s2 * exp2(m2 - m);
  }
}

__device__ inline void wave_lse2(double &m, double &s) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double m2 = __shfl_xor(m, o, 64);
    double s2 = __shfl_xor(s, o, 64);
    lse2_merge(m, s, m2, s2);
  }
}

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// Grid of an element-wise kernel over n items, 256 threads per workgroup: at most
// 65,536 workgroups, the kernel walks [0, n) in grid strides.
constexpr int64_t kStrideBlocks = 1 << 16;
inline dim3 stride_grid(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return dim3(static_cast<unsigned>(b < kStrideBlocks ? b : kStrideBlocks));
}
#define FA_GRID_STRIDE(i, n)                                                                 \
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); \
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// Optional per-kernel timing with HIP events recorded on the launch stream around
// individual launches.  Events come from a fixed pool; collect() must be called
// after the stream has reached the last recorded event.
enum KernelKind {
  KK_COL_PARTIAL = 0,
  KK_COL_MERGE,
  KK_ROW,
  KK_STAGE1,
  KK_STAGE2,
  KK_PLAN,
  KK_FEATSIM,
  KK_COL_T,
  KK_TRANSPOSE,
  KK_TOPK,
  KK_FUSED,
  KK_COUNT
};
struct KTimer {
  static constexpr int kPool = 2048;
  hipEvent_t ev[kPool];
  int kind[kPool / 2];
  int used = 0, created = 0;
  double ms[KK_COUNT] = {0};
  int calls[KK_COUNT] = {0};
  bool init() {
    for (; created < kPool; ++created)
      if (hipEventCreate(&ev[created]) != hipSuccess) return false;
    return true;
  }
  ~KTimer() {
    for (int q = 0; q < created; ++q) (void)hipEventDestroy(ev[q]);
  }
  // Returns a slot id or -1 when the pool is full (that launch is then untimed).
  int begin(int k, hipStream_t s) {
    if (used + 2 > created) return -1;
    const int id = used / 2;
    kind[id] = k;
    (void)hipEventRecord(ev[used], s);
    used += 2;
    return id;
  }
  void end(int id, hipStream_t s) {
    if (id >= 0) (void)hipEventRecord(ev[2 * id + 1], s);
  }
  void collect() {
    for (int id = 0; id < used / 2; ++id) {
      float x = 0.f;
      if (hipEventElapsedTime(&x, ev[2 * id], ev[2 * id + 1]) == hipSuccess) {
        ms[kind[id]] += x;
        calls[kind[id]] += 1;
      }
    }
    used = 0;
  }
};
#define FA_TIMED(tm, kk, s, launch)                                                 \
  do {                                                                              \
    const int tid_ = (tm) ? (tm)->begin((kk), (s)) : -1;                            \
    launch;                                                                         \
    if (tm) (tm)->end(tid_, (s));                                                   \
  } while (0)

// Validate a device CSR descriptor's host-visible fields.
inline int check_csr(const fa_csr *A, const char *name) {
  FA_REQUIRE(A != nullptr, FA_ERR_ARG, "%s: null CSR", name);
  FA_REQUIRE(A->n >= 0 && A->nnz >= 0, FA_ERR_CSR, "%s: negative size", name);
  FA_REQUIRE(A->n == 0 || A->rowptr != nullptr, FA_ERR_CSR, "%s: null rowptr", name);
  FA_REQUIRE(A->nnz == 0 || A->colidx != nullptr, FA_ERR_CSR, "%s: null colidx", name);
  return FA_OK;
}

}  // namespace fa
