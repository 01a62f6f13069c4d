// Rows scaled to unit length, for the angular HD metric: the distance
// |x_i/|x_i| - x_j/|x_j||^2 is the squared Euclidean distance of these rows,
// so the refinement kernels run on them unchanged.
#include "fsne_kernels.h"

namespace fsne {

// xu_i = x_i / |x_i| in FP32, the norm accumulated in FP32 from the stored
// values (BF16 widened exactly); a zero row stays zero.  One wave per row.
template <typename TX>
__global__ __launch_bounds__(kBlock) void k_unit_rows(const TX* __restrict__ X,
                                                      float* __restrict__ Xu, int D, int32_t i0,
                                                      int32_t n) {
  const int32_t w = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (w >= n) return;
  const int64_t row = (int64_t)(i0 + w) * D;
  const int lane = lane_id();
  float acc = 0.0f;
  for (int e = lane; e < D; e += kWave) {
    const float v = to_unit_f32(X[row + e]);
    acc = fmaf(v, v, acc);
  }
  const float nrm = wave_sum(acc);
  const float sc = nrm > 0.0f ? 1.0f / sqrtf(nrm) : 0.0f;
  for (int e = lane; e < D; e += kWave) Xu[row + e] = to_unit_f32(X[row + e]) * sc;
}

hipError_t launch_unit_rows(const void* X, int32_t xdtype, float* Xu, int32_t D, int32_t i0,
                            int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock));
  if (xdtype == 0)
    hipLaunchKernelGGL((k_unit_rows<float>), grid, dim3(kBlock), 0, s,
                       static_cast<const float*>(X), Xu, D, i0, n);
  else
    hipLaunchKernelGGL((k_unit_rows<uint16_t>), grid, dim3(kBlock), 0, s,
                       static_cast<const uint16_t*>(X), Xu, D, i0, n);
  return hipGetLastError();
}

}  // namespace fsne
