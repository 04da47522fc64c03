// Node similarity of Algorithm 1, Phase 1:
//   C_node = alpha * exp(-R1 R2^T) + (1 - alpha) * exp(-X1 X2^T)
// Both products are dense contractions, so they run on the matrix cores: FP32
// operands with v_mfma_f32_32x32x2_f32, BF16 operands with gfx950's
// v_mfma_f32_32x32x16_bf16, FP32 accumulation either way.  One workgroup owns a
// 128x128 output tile (four waves, 64x64 each as 2x2 blocks of 32x32), runs both
// K loops into two accumulator sets and applies the exponential mix once, so
// C_node is written a single time.  Workgroup ids are remapped so tiles that
// share operand panels run on the same XCD (its own L2).
#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T>
struct GemmTraits;
template <>
struct GemmTraits<float> {
  static constexpr int KC = 16;    // K elements per LDS stage
  static constexpr int KSTEP = 2;  // K per MFMA
  static constexpr int WPR = 16;   // 32-bit words per tile row (KC * 4 / 4)
};
template <>
struct GemmTraits<uint16_t> {
  static constexpr int KC = 32;
  static constexpr int KSTEP = 16;
  static constexpr int WPR = 16;   // KC * 2 / 4
};

constexpr int kTile = 128;
constexpr int kLdsStride = 17;  // words per LDS row: 16 + 1 pad (odd stride, no bank conflicts)

// Stage a 128 x KC tile of a row-major [rows x K] operand into LDS as 32-bit words.
template <typename T>
__device__ inline void stage_tile(const T *__restrict__ M, int32_t rows, int32_t K, int row0, int k0,
                                  uint32_t *__restrict__ lds) {
  constexpr int EPW = 4 / sizeof(T);  // elements per word
  constexpr int WPR = GemmTraits<T>::WPR;
  for (int wd = threadIdx.x; wd < kTile * WPR; wd += 256) {
    const int r = wd / WPR, c = wd % WPR;
    const int grow = row0 + r;
    const int gk = k0 + c * EPW;
    uint32_t v = 0;
    if (grow < rows) {
      const T *p = M + static_cast<int64_t>(grow) * K + gk;
      if (EPW == 1) {
        if (gk < K) v = reinterpret_cast<const uint32_t *>(p)[0];
      } else {
        const uint16_t *h = reinterpret_cast<const uint16_t *>(p);
        const uint32_t lo = gk < K ? h[0] : 0u;
        const uint32_t hi = gk + 1 < K ? h[1] : 0u;
        v = lo | (hi << 16);
      }
    }
    lds[r * kLdsStride + c] = v;
  }
}

template <typename T>
__device__ inline void mma_step(const uint32_t *__restrict__ la, const uint32_t *__restrict__ lb, int ks,
                                int wm, int wn, int lane, floatx16 (&acc)[2][2]);

template <>
__device__ inline void mma_step<float>(const uint32_t *__restrict__ la, const uint32_t *__restrict__ lb, int ks,
                                       int wm, int wn, int lane, floatx16 (&acc)[2][2]) {
  // 32x32x2: lane holds A[m = lane%32][k = lane/32] and B[k = lane/32][n = lane%32].
  const int k = ks * 2 + (lane >> 5);
  float av[2], bv[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    av[q] = __uint_as_float(la[(wm * 64 + q * 32 + (lane & 31)) * kLdsStride + k]);
    bv[q] = __uint_as_float(lb[(wn * 64 + q * 32 + (lane & 31)) * kLdsStride + k]);
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[p], bv[q], acc[p][q], 0, 0, 0);
}

template <>
__device__ inline void mma_step<uint16_t>(const uint32_t *__restrict__ la, const uint32_t *__restrict__ lb, int ks,
                                          int wm, int wn, int lane, floatx16 (&acc)[2][2]) {
  // 32x32x16: lane holds A[m = lane%32][k = 8*(lane/32) .. +8] (4 words), same for B.
  const int w0 = ks * 8 + (lane >> 5) * 4;
  bf16x8 av[2], bv[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    uint32_t wa[4], wb[4];
    const uint32_t *pa = la + (wm * 64 + q * 32 + (lane & 31)) * kLdsStride + w0;
    const uint32_t *pb = lb + (wn * 64 + q * 32 + (lane & 31)) * kLdsStride + w0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      wa[t] = pa[t];
      wb[t] = pb[t];
    }
    __builtin_memcpy(&av[q], wa, 16);
    __builtin_memcpy(&bv[q], wb, 16);
  }
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[p], bv[q], acc[p][q], 0, 0, 0);
}

template <typename T>
__device__ inline void gemm_nt(const T *__restrict__ A, const T *__restrict__ B, int32_t n1, int32_t n2, int32_t K,
                               int m0, int n0, uint32_t *la, uint32_t *lb, floatx16 (&acc)[2][2]) {
  constexpr int KC = GemmTraits<T>::KC, KSTEP = GemmTraits<T>::KSTEP;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
    stage_tile<T>(A, n1, K, m0, k0, la);
    stage_tile<T>(B, n2, K, n0, k0, lb);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / KSTEP; ++ks) mma_step<T>(la, lb, ks, wm, wn, lane, acc);
  }
}

template <typename TX, typename TR>
__global__ __launch_bounds__(256) void k_featsim(const TX *__restrict__ X1, const TX *__restrict__ X2, int32_t d,
                                                 const TR *__restrict__ R1, const TR *__restrict__ R2, int32_t nL,
                                                 int32_t n1, int32_t n2, float alpha, float *__restrict__ C) {
  __shared__ uint32_t la[kTile * kLdsStride];
  __shared__ uint32_t lb[kTile * kLdsStride];
  const int ntm = (n1 + kTile - 1) / kTile, ntn = (n2 + kTile - 1) / kTile;
  const int nb = ntm * ntn;
  // XCD-aware id: consecutive ids land on different XCDs; give each XCD a
  // contiguous range of the grouped tile order instead.
  int bid = blockIdx.x;
  const int full = (nb / 8) * 8;
  if (bid < full) bid = (bid % 8) * (full / 8) + bid / 8;
  // grouped order: 8 tile-rows at a time share B panels
  constexpr int GM = 8;
  const int group = bid / (GM * ntn);
  const int first_m = group * GM;
  const int gsz = min(ntm - first_m, GM);
  const int tm = first_m + (bid % (GM * ntn)) % gsz;
  const int tn = (bid % (GM * ntn)) / gsz;
  const int m0 = tm * kTile, n0 = tn * kTile;
  floatx16 accR[2][2], accX[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        accR[p][q][r] = 0.f;
        accX[p][q][r] = 0.f;
      }
  if (nL > 0) gemm_nt<TR>(R1, R2, n1, n2, nL, m0, n0, la, lb, accR);
  if (d > 0) gemm_nt<TX>(X1, X2, n1, n2, d, m0, n0, la, lb, accX);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const float beta = 1.0f - alpha;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int col = n0 + wn * 64 + q * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 64 + p * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (row < n1 && col < n2)
          C[static_cast<int64_t>(row) * n2 + col] = alpha * expf(-accR[p][q][r]) + beta * expf(-accX[p][q][r]);
      }
    }
}

int launch_feature_sim(const void *X1, const void *X2, int32_t n1, int32_t n2, int32_t d, int32_t xdt,
                       const void *R1, const void *R2, int32_t nL, int32_t rdt, double alpha, float *C,
                       hipStream_t s) {
  if (n1 == 0 || n2 == 0) return FA_OK;
  const int nb = ceil_div(n1, kTile) * ceil_div(n2, kTile);
  const float al = static_cast<float>(alpha);
  if (xdt == FA_BF16 && rdt == FA_BF16)
    FA_LAUNCH((k_featsim<uint16_t, uint16_t>), dim3(nb), dim3(256), 0, s, static_cast<const uint16_t *>(X1),
              static_cast<const uint16_t *>(X2), d, static_cast<const uint16_t *>(R1),
              static_cast<const uint16_t *>(R2), nL, n1, n2, al, C);
  else if (xdt == FA_BF16)
    FA_LAUNCH((k_featsim<uint16_t, float>), dim3(nb), dim3(256), 0, s, static_cast<const uint16_t *>(X1),
              static_cast<const uint16_t *>(X2), d, static_cast<const float *>(R1), static_cast<const float *>(R2),
              nL, n1, n2, al, C);
  else if (rdt == FA_BF16)
    FA_LAUNCH((k_featsim<float, uint16_t>), dim3(nb), dim3(256), 0, s, static_cast<const float *>(X1),
              static_cast<const float *>(X2), d, static_cast<const uint16_t *>(R1),
              static_cast<const uint16_t *>(R2), nL, n1, n2, al, C);
  else
    FA_LAUNCH((k_featsim<float, float>), dim3(nb), dim3(256), 0, s, static_cast<const float *>(X1),
              static_cast<const float *>(X2), d, static_cast<const float *>(R1), static_cast<const float *>(R2), nL,
              n1, n2, al, C);
  return FA_OK;
}

}  // namespace fa

using namespace fa;

extern "C" int fa_feature_sim(const void *X1, const void *X2, int32_t n1, int32_t n2, int32_t d, int32_t x_dtype,
                              const void *R1, const void *R2, int32_t nL, int32_t r_dtype, double alpha,
                              float *C_node, void *stream) {
  FA_REQUIRE(n1 >= 0 && n2 >= 0 && d >= 0 && nL >= 0, FA_ERR_ARG, "fa_feature_sim: negative size");
  FA_REQUIRE((x_dtype == FA_F32 || x_dtype == FA_BF16) && (r_dtype == FA_F32 || r_dtype == FA_BF16), FA_ERR_ARG,
             "fa_feature_sim: dtype must be FA_F32 or FA_BF16");
  if (n1 == 0 || n2 == 0) return FA_OK;
  FA_REQUIRE(C_node && (d == 0 || (X1 && X2)) && (nL == 0 || (R1 && R2)), FA_ERR_ARG, "fa_feature_sim: null pointer");
  return launch_feature_sim(X1, X2, n1, n2, d, x_dtype, R1, R2, nL, r_dtype, alpha, C_node,
                            static_cast<hipStream_t>(stream));
}
