// Node similarity of Algorithm 1, Phase 1:
//   C_node = alpha * exp(-R1 R2^T) + (1 - alpha) * exp(-X1 X2^T)
// Both products are dense contractions, so they run on the matrix cores: FP32
// operands with v_mfma_f32_32x32x2_f32, BF16 operands with gfx950's
// v_mfma_f32_32x32x16_bf16, FP32 accumulation either way.  One workgroup owns a
// 128x128 output tile (four waves, 64x64 each as 2x2 blocks of 32x32), runs both
// K loops into two accumulator sets and applies the exponential mix once, so
// C_node is written a single time.  Operands move in 16-byte pieces: 128 bytes of
// K per row and step, staged through padded LDS rows, with the next step's
// global loads in flight during the current step's MFMAs.  Workgroup ids are
// remapped so tiles that share operand panels run on the same XCD (its own L2).
#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTile = 128;              // output tile per workgroup (4 waves, 64 x 64 each)
constexpr int kChunkBytes = 128;        // K bytes of each operand row staged per step
constexpr int kLdsRow = kChunkBytes + 16;  // padded LDS row: 16-byte fragment reads stay conflict-free

// One step's operand tile (kTile rows x kChunkBytes) held in registers while the
// previous step computes: 1024 16-byte pieces, four per thread.
struct Stage {
  uint4 v[4];
};

// Load rows [row0, row0+128) x K elements [k0, k0 + kChunkBytes/sizeof(T)) of a
// row-major [rows x K] operand.  vec: every row starts 16-byte aligned and K is a
// whole number of 16-byte pieces, so pieces are single vector loads; otherwise the
// pieces are assembled element by element.  Out-of-range rows and K are zero.
template <typename T>
__device__ inline void load_stage(const T *__restrict__ M, int32_t rows, int32_t K, int row0, int k0, bool vec,
                                  Stage &st) {
  constexpr int EPP = 16 / sizeof(T);  // elements per piece
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = threadIdx.x + 256 * i;
    const int r = q >> 3, piece = q & 7;
    const int grow = row0 + r, gk = k0 + piece * EPP;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (grow < rows && gk < K) {
      const T *p = M + static_cast<int64_t>(grow) * K + gk;
      if (vec) {
        v = *reinterpret_cast<const uint4 *>(p);
      } else {
        T e[EPP];
#pragma unroll
        for (int t = 0; t < EPP; ++t) e[t] = gk + t < K ? p[t] : T(0);
        __builtin_memcpy(&v, e, 16);
      }
    }
    st.v[i] = v;
  }
}

__device__ inline void store_stage(const Stage &st, uint8_t *__restrict__ lds) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = threadIdx.x + 256 * i;
    *reinterpret_cast<uint4 *>(lds + (q >> 3) * kLdsRow + (q & 7) * 16) = st.v[i];
  }
}

// The MFMA steps of one staged chunk for a wave's 64 x 64 block (2 x 2 blocks of 32 x 32).
template <typename T>
__device__ inline void mma_chunk(const uint8_t *__restrict__ la, const uint8_t *__restrict__ lb, int wm, int wn,
                                 int lane, floatx16 (&acc)[2][2]);

// FP32, v_mfma_f32_32x32x2_f32: in each step lane l supplies A[m = l%32][k] and
// B[k][n = l%32] for one k of a pair.  The sum over K is order-free, so each
// 8-element group of K is split as lanes 0-31 -> k0..k0+3, lanes 32-63 -> k0+4..k0+7
// (one 16-byte LDS read per fragment) and step t pairs k0+t with k0+4+t.
template <>
__device__ inline void mma_chunk<float>(const uint8_t *__restrict__ la, const uint8_t *__restrict__ lb, int wm,
                                        int wn, int lane, floatx16 (&acc)[2][2]) {
  const int half = lane >> 5, r = lane & 31;
#pragma unroll
  for (int g = 0; g < kChunkBytes / 32; ++g) {
    float4 av[2], bv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      av[q] = *reinterpret_cast<const float4 *>(la + (wm * 64 + q * 32 + r) * kLdsRow + g * 32 + half * 16);
      bv[q] = *reinterpret_cast<const float4 *>(lb + (wn * 64 + q * 32 + r) * kLdsRow + g * 32 + half * 16);
    }
    const float *a0 = reinterpret_cast<const float *>(&av[0]), *a1 = reinterpret_cast<const float *>(&av[1]);
    const float *b0 = reinterpret_cast<const float *>(&bv[0]), *b1 = reinterpret_cast<const float *>(&bv[1]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[t], b0[t], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[t], b1[t], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[t], b0[t], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[t], b1[t], acc[1][1], 0, 0, 0);
    }
  }
}

// BF16, v_mfma_f32_32x32x16_bf16: lane l supplies A[m = l%32][k = 8(l/32) .. +8] and
// the same slice of B, one 16-byte LDS read each.
template <>
__device__ inline void mma_chunk<uint16_t>(const uint8_t *__restrict__ la, const uint8_t *__restrict__ lb, int wm,
                                           int wn, int lane, floatx16 (&acc)[2][2]) {
  const int half = lane >> 5, r = lane & 31;
#pragma unroll
  for (int ks = 0; ks < kChunkBytes / 32; ++ks) {
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      av[q] = *reinterpret_cast<const bf16x8 *>(la + (wm * 64 + q * 32 + r) * kLdsRow + ks * 32 + half * 16);
      bv[q] = *reinterpret_cast<const bf16x8 *>(lb + (wn * 64 + q * 32 + r) * kLdsRow + ks * 32 + half * 16);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[p], bv[q], acc[p][q], 0, 0, 0);
  }
}

// acc += A[m0.., :] B[n0.., :]^T over all of K.  The next chunk's global loads are
// issued before the current chunk's MFMAs, so they are in flight during the math.
template <typename T>
__device__ inline void gemm_nt(const T *__restrict__ A, const T *__restrict__ B, int32_t n1, int32_t n2, int32_t K,
                               int m0, int n0, uint8_t *la, uint8_t *lb, floatx16 (&acc)[2][2]) {
  constexpr int KE = kChunkBytes / sizeof(T);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const bool vec = (static_cast<int64_t>(K) * sizeof(T)) % 16 == 0 &&
                   (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  Stage sa, sb;
  load_stage<T>(A, n1, K, m0, 0, vec, sa);
  load_stage<T>(B, n2, K, n0, 0, vec, sb);
  for (int k0 = 0; k0 < K; k0 += KE) {
    __syncthreads();  // the previous chunk's LDS reads are done
    store_stage(sa, la);
    store_stage(sb, lb);
    __syncthreads();
    if (k0 + KE < K) {
      load_stage<T>(A, n1, K, m0, k0 + KE, vec, sa);
      load_stage<T>(B, n2, K, n0, k0 + KE, vec, sb);
    }
    mma_chunk<T>(la, lb, wm, wn, lane, acc);
  }
}

template <typename TX, typename TR>
__global__ __launch_bounds__(256) void k_featsim(const TX *__restrict__ X1, const TX *__restrict__ X2, int32_t d,
                                                 const TR *__restrict__ R1, const TR *__restrict__ R2, int32_t nL,
                                                 int32_t n1, int32_t n2, float alpha, float *__restrict__ C) {
  __shared__ __align__(16) uint8_t la[kTile * kLdsRow];
  __shared__ __align__(16) uint8_t lb[kTile * kLdsRow];
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
