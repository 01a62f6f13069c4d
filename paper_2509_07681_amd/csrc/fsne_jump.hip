// Jump start by a random linear projection (Sec. 3, paragraph on helping the
// first iterations): the embedding is replaced by a projection of the
// centred data, so that LD neighbours, and their neighbours, already carry
// some of the HD structure when the lists are still random.
//   y_ic = s sum_k (x_ik - mu_k) r_kc,   r_kc = +1 or -1,
//   s = sigma / sqrt(tr Sigma),  tr Sigma = (1/N) sum_i |x_i - mu|^2,
// with r_kc = -1 when bit 0 of the first word of Philox block
// (k, c, 9, projection) is set.  Column means and the trace are summed in
// double in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fsne_context.h"

namespace {

using namespace fsne;

constexpr int kColTile = 64;      // columns per block
constexpr int kRowLanes = 4;      // row lanes per block (256 threads)
constexpr int kRowChunks = 256;   // row chunks (blockIdx.y)
constexpr uint32_t kStreamJump = 9;

__device__ __forceinline__ float load_x(const void* X, int xdtype, int64_t q) {
  return xdtype == 0 ? static_cast<const float*>(X)[q]
                     : __uint_as_float((uint32_t) static_cast<const uint16_t*>(X)[q] << 16);
}

// part[chunk][k] = sum over the chunk's rows of (x_ik - mu_k)^p, p = 1 with
// mu = NULL (plain sums), p = 2 otherwise; rows in a fixed order.
__global__ __launch_bounds__(256) void k_col_part(const void* X, int xdtype, int64_t N, int D,
                                                  const double* mu, double* part) {
  __shared__ double red[kRowLanes][kColTile];
  const int col = blockIdx.x * kColTile + (threadIdx.x % kColTile);
  const int rl = threadIdx.x / kColTile;
  const int64_t per = (N + kRowChunks - 1) / kRowChunks;
  const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min(N, r0 + per);
  double s = 0.0;
  if (col < D) {
    const double m = mu ? mu[col] : 0.0;
    for (int64_t r = r0 + rl; r < r1; r += kRowLanes) {
      const double v = (double)load_x(X, xdtype, r * D + col);
      s += mu ? (v - m) * (v - m) : v;
    }
  }
  red[rl][threadIdx.x % kColTile] = s;
  __syncthreads();
  if (rl == 0 && col < D) {
    double t = 0.0;
    for (int k = 0; k < kRowLanes; ++k) t += red[k][threadIdx.x];
    part[(int64_t)blockIdx.y * D + col] = t;
  }
}

// out[k] = (sum over chunks of part[.][k]) / N, in chunk order.
__global__ void k_col_final(const double* part, int D, int64_t N, double* out) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= D) return;
  double t = 0.0;
  for (int c = 0; c < kRowChunks; ++c) t += part[(int64_t)c * D + col];
  out[col] = t / (double)N;
}

// scale = sigma / sqrt(sum_k var_k) (0 when the data have no spread), and
// the sign matrix r (D x d).
__global__ void k_jump_setup(const double* var, const double* mu, int D, int d, float sigma,
                             uint32_t projection, uint32_t k0, uint32_t k1, float* muf,
                             float* r, float* scale) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < D * d) {
    const int k = q / d, c = q % d;
    const uint4 u = philox((uint32_t)k, (uint32_t)c, kStreamJump, projection, k0, k1);
    r[q] = (u.x & 1u) ? -1.0f : 1.0f;
  }
  if (q < D) muf[q] = (float)mu[q];
  if (q == 0) {
    double tr = 0.0;
    for (int k = 0; k < D; ++k) tr += var[k];
    *scale = tr > 0.0 ? (float)((double)sigma / sqrt(tr)) : 0.0f;
  }
}

// Y[i][c] = scale sum_k (x_ik - mu_k) r_kc for c < d; V[i] = 0.  One thread
// per (point, component).
__global__ void k_project(const void* X, int xdtype, int64_t N, int D, int d, int DP,
                          const float* muf, const float* r, const float* scale, float* Y,
                          float* V) {
  const int64_t total = N * (int64_t)DP;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / DP;
    const int c = (int)(q % DP);
    if (c < d) {
      float s = 0.0f;
      for (int k = 0; k < D; ++k) s = fmaf(load_x(X, xdtype, i * D + k) - muf[k], r[k * d + c], s);
      Y[q] = *scale * s;
    }
    V[q] = 0.0f;
  }
}

}  // namespace

extern "C" fsne_status fsne_jump_start(fsne_ctx* c, int32_t projection, float sigma) {
  if (!c) return FSNE_EINVAL;
  if (projection < 0 || !(sigma > 0.0f) || !std::isfinite(sigma)) {
    c->err = "fsne_jump_start: projection must be >= 0 and sigma > 0";
    return FSNE_EINVAL;
  }
  const int D = c->D, d = c->d;
  const int64_t N = c->N;
  double *part = nullptr, *mu = nullptr, *var = nullptr;
  float *muf = nullptr, *r = nullptr, *scale = nullptr;
  fsne_status st = FSNE_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == FSNE_OK) {
      c->err = std::string("fsne_jump_start: ") + what + ": " + hipGetErrorString(e);
      st = FSNE_EHIP;
    }
    return st == FSNE_OK;
  };
  if (chk(hipMalloc(&part, sizeof(double) * kRowChunks * D), "hipMalloc") &&
      chk(hipMalloc(&mu, sizeof(double) * D), "hipMalloc") &&
      chk(hipMalloc(&var, sizeof(double) * D), "hipMalloc") &&
      chk(hipMalloc(&muf, sizeof(float) * D), "hipMalloc") &&
      chk(hipMalloc(&r, sizeof(float) * D * d), "hipMalloc") &&
      chk(hipMalloc(&scale, sizeof(float)), "hipMalloc")) {
    const dim3 grid((unsigned)((D + kColTile - 1) / kColTile), kRowChunks);
    const unsigned gd = (unsigned)((D + 255) / 256);
    hipLaunchKernelGGL(k_col_part, grid, dim3(256), 0, c->stream, c->X, c->xdtype, N, D,
                       (const double*)nullptr, part);
    hipLaunchKernelGGL(k_col_final, dim3(gd), dim3(256), 0, c->stream, part, D, N, mu);
    hipLaunchKernelGGL(k_col_part, grid, dim3(256), 0, c->stream, c->X, c->xdtype, N, D,
                       (const double*)mu, part);
    hipLaunchKernelGGL(k_col_final, dim3(gd), dim3(256), 0, c->stream, part, D, N, var);
    hipLaunchKernelGGL(k_jump_setup, dim3((unsigned)((D * d + 255) / 256 + 1)), dim3(256), 0,
                       c->stream, var, mu, D, d, sigma, (uint32_t)projection, (uint32_t)c->seed,
                       (uint32_t)(c->seed >> 32), muf, r, scale);
    const int64_t total = N * (int64_t)c->DP;
    const unsigned gp = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_project, dim3(gp), dim3(256), 0, c->stream, c->X, c->xdtype, N, D, d,
                       c->DP, muf, r, scale, c->Y, c->V);
    chk(hipGetLastError(), "launch");
    chk(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  }
  for (void* p : {(void*)part, (void*)mu, (void*)var, (void*)muf, (void*)r, (void*)scale})
    if (p) (void)hipFree(p);
  return st;
}
