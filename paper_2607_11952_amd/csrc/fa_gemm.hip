// Node similarity of Algorithm 1, Phase 1:
//   C_node = alpha * exp(-R1 R2^T) + (1 - alpha) * exp(-X1 X2^T)
// Both products are dense contractions, so they run on the matrix cores: FP32
// operands with v_mfma_f32_32x32x2_f32, BF16 operands with gfx950's
// v_mfma_f32_32x32x16_bf16, FP32 accumulation either way.  Each workgroup runs
// both K loops into two accumulator sets and applies the exponential mix once, so
// C_node is written a single time, and workgroup ids are remapped so tiles that
// share operand panels run on the same XCD (its own L2).
//   k_featsim_dma (BF16 operands in whole 16-byte pieces, the form the alignment
//     uses): 256 x 128 tiles, eight waves, operands loaded straight into a
//     three-stage LDS ring by buffer loads with an LDS destination, so two K steps
//     are in flight while a third is multiplied.
//   k_featsim (FP32 operands, or K not a multiple of 8): 128 x 128 tiles, four
//     waves, operands staged through registers into padded LDS rows with the next
//     step's global loads in flight during the current step's MFMAs.
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

// ---------------------------------------------------------------- BF16, direct-to-LDS
// Both operands BF16 with K a multiple of 8 and 16-byte aligned rows (every 16-byte
// piece lies wholly inside or wholly past K): a 256 x 128 tile per workgroup, eight
// waves of 64 x 64, and the operands moved by direct-to-LDS buffer loads
// (buffer_load_dwordx4 ... lds: no registers in between) into a three-stage ring, so
// two 64-element steps of K are in flight while the third is multiplied, with one
// barrier per step.  One workgroup per CU (144 KB of LDS), two waves per SIMD.
constexpr int kDmaBM = 256, kDmaBN = 128;
constexpr int kDmaStep = 64;                       // K elements per stage: 128 bytes per row
constexpr int kDmaLoads = (kDmaBM + kDmaBN) / 64;  // load instructions per wave per stage (1 KB each)

// Buffer resource over the rows [row0, row0 + nr) of a row-major [rows x K] BF16
// operand that one tile reads, nr = min(tile_rows, rows - row0) (row0 < rows): a
// load at or past its end returns zero, and offsets stay below tile_rows * K * 2
// bytes whatever the operand's size.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t dma_rsrc(const uint16_t *M, int32_t rows, int32_t K, int row0,
                                                           int tile_rows) {
  const int nr = rows - row0 < tile_rows ? rows - row0 : tile_rows;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(M + static_cast<int64_t>(row0) * K), 0, nr * K * 2,
                                           0x00020000);
}

// The 16-byte piece p of row r of a stage sits in slot p ^ dma_swz(r) of the row's
// 128 bytes, so the fragment reads (32 consecutive rows, one piece each) spread over
// all banks whether the LDS serves 16 or 32 lanes per cycle.
__device__ __forceinline__ int dma_swz(int r) { return (r ^ (r >> 3)) & 7; }

// The tile's ROWS rows x K elements [k0, k0 + 64) of the operand (resource rs from
// dma_rsrc, nr valid rows) into a stage (ROWS x 128 bytes).  Each instruction
// writes 1 KB (eight rows) of LDS, lane l at byte 16 l, so lane l fetches the piece
// its slot holds; pieces past K or past the last row are given an offset past the
// end and arrive as zeros.
template <int ROWS>
__device__ __forceinline__ void dma_stage(__amdgpu_buffer_rsrc_t rs, int32_t nr, int32_t K, int k0, uint8_t *lds,
                                          int wv, int lane) {
#pragma unroll
  for (int i = 0; i < ROWS / 64; ++i) {
    const int g = i * 8 + wv;  // 1 KB block: rows 8g .. 8g+7
    const int r = 8 * g + (lane >> 3);
    const int k = k0 + 8 * ((lane & 7) ^ dma_swz(r));
    const uint32_t off = r < nr && k < K ? (static_cast<uint32_t>(r) * K + k) * 2u : 0x80000000u;
    // the LDS operand is the wave's block base (M0); a generic-to-LDS address-space cast
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)(lds + g * 1024), 16, off, 0,
                                             0, 0);
  }
}

__device__ __forceinline__ bf16x8 dma_frag(const uint8_t *lds, int r, int piece) {
  return *reinterpret_cast<const bf16x8 *>(lds + r * 128 + 16 * (piece ^ dma_swz(r)));
}

// One stage's MFMAs for the wave's 64 x 64 block: all sixteen fragments of the
// stage are read first, then the sixteen MFMAs issue back to back (the scheduling
// groups stop the compiler from interleaving each read just before its MFMA, which
// left the LDS latency in the MFMA chain).
__device__ __forceinline__ void dma_mma(const uint8_t *la, const uint8_t *lb, int wm, int wn, int lane,
                                        floatx16 (&acc)[2][2]) {
  const int half = lane >> 5, r = lane & 31;
  bf16x8 av[kDmaStep / 16][2], bv[kDmaStep / 16][2];
#pragma unroll
  for (int ks = 0; ks < kDmaStep / 16; ++ks)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      av[ks][q] = dma_frag(la, wm * 64 + q * 32 + r, 2 * ks + half);
      bv[ks][q] = dma_frag(lb, wn * 64 + q * 32 + r, 2 * ks + half);
    }
#pragma unroll
  for (int ks = 0; ks < kDmaStep / 16; ++ks)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[ks][p], bv[ks][q], acc[p][q], 0, 0, 0);
  __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);  // 16 LDS reads
  __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);  // then 16 MFMAs
}

// e^-x as 2^(-x log2 e) with the hardware exp2 (about one ulp of its own): rounding
// the FP32 argument adds at most |x| 2^-24 relative error, i.e. at most
// |x| 2^-24 e^-x <= 2^-24 / e absolute for x >= 0.
__device__ __forceinline__ float exp_neg(float x) { return __builtin_amdgcn_exp2f(-x * 1.44269504088896341f); }

__global__ __launch_bounds__(512, 1) void k_featsim_dma(const uint16_t *__restrict__ X1, const uint16_t *__restrict__ X2,
                                                        int32_t d, const uint16_t *__restrict__ R1,
                                                        const uint16_t *__restrict__ R2, int32_t nL, int32_t n1,
                                                        int32_t n2, float alpha, float *__restrict__ C) {
  // three stages, each an A panel (256 rows x 128 bytes) then a B panel (128 rows x 128 bytes)
  __shared__ __align__(1024) uint8_t ring[3][(kDmaBM + kDmaBN) * 128];
  const int ntm = (n1 + kDmaBM - 1) / kDmaBM, ntn = (n2 + kDmaBN - 1) / kDmaBN;
  const int nb = ntm * ntn;
  // XCD-aware id, then groups of 8 tile-rows sharing B panels (as in k_featsim)
  int bid = blockIdx.x;
  const int full = (nb / 8) * 8;
  if (bid < full) bid = (bid % 8) * (full / 8) + bid / 8;
  constexpr int GM = 8;
  const int group = bid / (GM * ntn);
  const int first_m = group * GM;
  const int gsz = min(ntm - first_m, GM);
  const int tm = first_m + (bid % (GM * ntn)) % gsz;
  const int tn = (bid % (GM * ntn)) / gsz;
  const int m0 = tm * kDmaBM, n0 = tn * kDmaBN;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wv >> 1, wn = wv & 1;
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
  // the K steps of the encoding product, then those of the attribute product
  const int nR = (nL + kDmaStep - 1) / kDmaStep, nX = (d + kDmaStep - 1) / kDmaStep;
  const int nc = nR + nX;
  // resources over this tile's rows of each operand (m0 < n1, n0 < n2)
  const int nm = n1 - m0 < kDmaBM ? n1 - m0 : kDmaBM, nn = n2 - n0 < kDmaBN ? n2 - n0 : kDmaBN;
  const __amdgpu_buffer_rsrc_t rR1 = dma_rsrc(R1, n1, nL, m0, kDmaBM), rR2 = dma_rsrc(R2, n2, nL, n0, kDmaBN);
  const __amdgpu_buffer_rsrc_t rX1 = dma_rsrc(X1, n1, d, m0, kDmaBM), rX2 = dma_rsrc(X2, n2, d, n0, kDmaBN);
  auto issue = [&](int c) {
    uint8_t *la = ring[c % 3], *lb = la + kDmaBM * 128;
    if (c < nR) {
      dma_stage<kDmaBM>(rR1, nm, nL, c * kDmaStep, la, wv, lane);
      dma_stage<kDmaBN>(rR2, nn, nL, c * kDmaStep, lb, wv, lane);
    } else {
      dma_stage<kDmaBM>(rX1, nm, d, (c - nR) * kDmaStep, la, wv, lane);
      dma_stage<kDmaBN>(rX2, nn, d, (c - nR) * kDmaStep, lb, wv, lane);
    }
  };
  // Step c: wait for this wave's loads of step c (those of step c+1 may stay in
  // flight; vector-memory loads complete in issue order), barrier (every wave's
  // pieces have landed, and every wave is done with the buffer of step c-1: its
  // fragment reads fed MFMAs already issued), load step c+2 into that buffer,
  // multiply step c.  A bare s_barrier: __syncthreads' fence would wait for every
  // load in flight.  The compiler barriers keep LDS accesses on their side of it.
  auto step = [&](int c, floatx16(&acc)[2][2]) {
    if (c + 1 < nc)
      __builtin_amdgcn_s_waitcnt(0x0F70 | kDmaLoads);  // vmcnt(kDmaLoads)
    else
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (c + 2 < nc) issue(c + 2);
    const uint8_t *la = ring[c % 3];
    dma_mma(la, la + kDmaBM * 128, wm, wn, lane, acc);
  };
  if (nc > 0) issue(0);
  if (nc > 1) issue(1);
  for (int c = 0; c < nR; ++c) step(c, accR);
  for (int c = nR; c < nc; ++c) step(c, accX);
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
          C[static_cast<int64_t>(row) * n2 + col] = alpha * exp_neg(accR[p][q][r]) + beta * exp_neg(accX[p][q][r]);
      }
    }
}

// Operands the direct-to-LDS kernel takes: whole 16-byte pieces (K a multiple of
// 8, 16-byte aligned rows) and a tile's rows under 2^31 bytes (32-bit buffer offsets).
static bool dma_operands(const void *A, const void *B, int32_t K) {
  return K == 0 || (K % 8 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                    (reinterpret_cast<uintptr_t>(B) & 15) == 0 && int64_t(kDmaBM) * K * 2 < (int64_t(1) << 31));
}

int launch_feature_sim(const void *X1, const void *X2, int32_t n1, int32_t n2, int32_t d, int32_t xdt,
                       const void *R1, const void *R2, int32_t nL, int32_t rdt, double alpha, float *C,
                       hipStream_t s) {
  if (n1 == 0 || n2 == 0) return FA_OK;
  const int nb = ceil_div(n1, kTile) * ceil_div(n2, kTile);
  const float al = static_cast<float>(alpha);
  if (xdt == FA_BF16 && rdt == FA_BF16 && dma_operands(X1, X2, d) && dma_operands(R1, R2, nL))
    FA_LAUNCH(k_featsim_dma, dim3(ceil_div(n1, kDmaBM) * ceil_div(n2, kDmaBN)), dim3(512), 0, s,
              static_cast<const uint16_t *>(X1), static_cast<const uint16_t *>(X2), d,
              static_cast<const uint16_t *>(R1), static_cast<const uint16_t *>(R2), nL, n1, n2, al, C);
  else if (xdt == FA_BF16 && rdt == FA_BF16)
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
