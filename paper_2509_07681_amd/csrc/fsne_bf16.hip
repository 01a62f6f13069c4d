// Squared norms of the BF16 rows (for the expanded-form screen of the BF16 form).
#include "fsne_kernels.h"

namespace fsne {

// Squared norms of BF16 rows, accumulated in FP32 from the BF16 values.
__global__ void k_xnorm(const uint16_t* __restrict__ X, int D, int32_t i0, int32_t n,
                        float* __restrict__ xnorm) {
  const int32_t i = i0 + (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= i0 + n) return;
  const int lane = lane_id();
  float acc = 0.0f;
  for (int e = lane; e < D; e += kWave) {
    const float v = __uint_as_float(((uint32_t)X[(int64_t)i * D + e]) << 16);
    acc = fmaf(v, v, acc);
  }
  acc = wave_sum(acc);
  if (lane == 0) xnorm[i] = acc;
}

hipError_t launch_xnorm(const StepArgs& a, float* xnorm, int32_t i0, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xnorm, dim3((unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock)),
                     dim3(kBlock), 0, s, static_cast<const uint16_t*>(a.X), a.D, i0, n, xnorm);
  return hipGetLastError();
}

}  // namespace fsne
