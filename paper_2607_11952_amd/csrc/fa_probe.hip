// Measurement utility: the achievable HBM read rate of this part, as a reference
// next to the vendor peak for the streaming kernels (both Sinkhorn passes read
// the cost once with 16-byte non-temporal loads; this kernel does nothing else).
#include "fa_common.h"
#include "fa_internal.h"

namespace fa {

// Grid-stride sum of a float buffer: eight 16-byte streaming loads in flight per
// thread per step (the fastest plain read found on this part: 2-8 loads in flight,
// 2k-64k workgroups, streaming or cached loads were compared), one partial per
// thread (so nothing is optimised away).
__global__ __launch_bounds__(256) void k_stream_read(const float *__restrict__ x, size_t n4,
                                                     float *__restrict__ partial) {
  constexpr int U = 8;
  const size_t tid = blockIdx.x * 256ull + threadIdx.x;
  const size_t stride = gridDim.x * 256ull;
  float s = 0.f;
  size_t i = tid;
  for (; i + (U - 1) * stride < n4; i += U * stride) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ld_stream4(x + 4 * (i + u * stride));
#pragma unroll
    for (int u = 0; u < U; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n4; i += stride) {
    const f32x4 v = ld_stream4(x + 4 * i);
    s += (v.x + v.y) + (v.z + v.w);
  }
  partial[tid] = s;
}

}  // namespace fa

using namespace fa;

extern "C" int fa_stream_read(const float *x, size_t n, float *partial, int32_t nblocks, void *stream) {
  FA_REQUIRE(x && partial, FA_ERR_ARG, "fa_stream_read: null pointer");
  FA_REQUIRE(n % 4 == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0, FA_ERR_ARG,
             "fa_stream_read: n must be a multiple of 4 and x 16-byte aligned");
  FA_REQUIRE(nblocks >= 1 && nblocks <= 65536, FA_ERR_ARG, "fa_stream_read: nblocks %d not in [1, 65536]", nblocks);
  if (n == 0) return FA_OK;
  FA_LAUNCH(k_stream_read, dim3(nblocks), dim3(256), 0, static_cast<hipStream_t>(stream), x, n / 4, partial);
  return FA_OK;
}
