// Measurement aid, not part of the FUnc-SNE library: the rate at which one
// MI355X gathers rows of a given size from random positions of a table, in
// the same access shape the step kernels use (a row split over row_bytes/16
// lanes, one 16-byte load per lane, so one wave load instruction fetches
// 64 / (row_bytes/16) rows).  It gives the ceiling that the neighbour-row
// gathers of the LD pass can reach, which for small rows lies well below
// the streaming bandwidth of HBM.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Wave w gathers `rows` rows at pseudo-random positions in [0, nrows); the
// sum is stored only if it equals a value the zero table cannot produce, so
// nothing is written but the loads cannot be removed.
template <int LPR>   // lanes per row
__global__ __launch_bounds__(256) void k_gather_probe(const float4* __restrict__ T, uint32_t nrows,
                                                      int rows, int nw, uint32_t salt,
                                                      float* sink) {
  const int w = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (w >= nw) return;
  constexpr int RPI = 64 / LPR;
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int p = 0; p < rows; p += RPI) {
    const uint32_t r = mix32((uint32_t)w * 977u + (uint32_t)(p + lane / LPR) * 131u + salt) % nrows;
    const float4 v = T[(size_t)r * LPR + (lane % LPR)];
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  const float s = acc.x + acc.y + acc.z + acc.w;
  if (s == 123.456f) sink[w] = s;
}

}  // namespace

extern "C" {

// Gathers `rows_per_wave` random rows of row_bytes (16, 32, 64, 128, 256 or
// 512) per wave over nwaves waves from a zeroed device table of table_bytes,
// `reps` times; *ms gets the mean time of one launch (HIP events).  Returns
// 0, or -1 for bad arguments, -3 for a HIP error.
int fsne_probe_gather(int64_t table_bytes, int32_t row_bytes, int32_t rows_per_wave,
                      int32_t nwaves, int32_t reps, float* ms) {
  if (!ms || reps < 1 || nwaves < 1 || rows_per_wave < 1 || table_bytes < row_bytes) return -1;
  const int lpr = row_bytes / 16;
  if (row_bytes % 16 || lpr < 1 || lpr > 32 || (lpr & (lpr - 1))) return -1;
  const uint64_t nrows64 = (uint64_t)table_bytes / (uint64_t)row_bytes;
  if (nrows64 > 0xFFFFFFFFull) return -1;
  const uint32_t nrows = (uint32_t)nrows64;
  float4* T = nullptr;
  float* sink = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  int rc = 0;
  auto ok = [&](hipError_t e) { if (e != hipSuccess) rc = -3; return e == hipSuccess; };
  if (ok(hipMalloc(&T, (size_t)nrows * row_bytes)) && ok(hipMalloc(&sink, sizeof(float) * nwaves)) &&
      ok(hipMemset(T, 0, (size_t)nrows * row_bytes)) && ok(hipEventCreate(&a)) &&
      ok(hipEventCreate(&b))) {
    const dim3 grid((unsigned)((nwaves + 3) / 4)), block(256);
    for (int pass = 0; pass < 2 && rc == 0; ++pass) {   // pass 0 warms up
      ok(hipEventRecord(a));
      for (int r = 0; r < reps; ++r) {
        const uint32_t salt = (uint32_t)(pass * 7919 + r * 104729);
        switch (lpr) {
          case 1: hipLaunchKernelGGL(k_gather_probe<1>, grid, block, 0, 0, T, nrows, rows_per_wave, nwaves, salt, sink); break;
          case 2: hipLaunchKernelGGL(k_gather_probe<2>, grid, block, 0, 0, T, nrows, rows_per_wave, nwaves, salt, sink); break;
          case 4: hipLaunchKernelGGL(k_gather_probe<4>, grid, block, 0, 0, T, nrows, rows_per_wave, nwaves, salt, sink); break;
          case 8: hipLaunchKernelGGL(k_gather_probe<8>, grid, block, 0, 0, T, nrows, rows_per_wave, nwaves, salt, sink); break;
          case 16: hipLaunchKernelGGL(k_gather_probe<16>, grid, block, 0, 0, T, nrows, rows_per_wave, nwaves, salt, sink); break;
          default: hipLaunchKernelGGL(k_gather_probe<32>, grid, block, 0, 0, T, nrows, rows_per_wave, nwaves, salt, sink); break;
        }
        ok(hipGetLastError());
      }
      ok(hipEventRecord(b));
      ok(hipEventSynchronize(b));
      float t = 0.0f;
      ok(hipEventElapsedTime(&t, a, b));
      *ms = t / (float)reps;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (T) (void)hipFree(T);
  if (sink) (void)hipFree(sink);
  return rc;
}

}  // extern "C"
