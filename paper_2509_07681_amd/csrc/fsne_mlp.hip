// Placement network for dynamic data: D -> H1 -> H2 -> d with ReLU hidden
// layers, trained by mean squared error on (x, standardised y) pairs of a
// context's embedding with Adam, then used to place inserted or drifted
// points.  The three large products run as BF16 MFMA GEMMs with FP32
// accumulation (operands rounded to nearest even when staged into LDS); the
// d-wide output layer, the loss, the reductions and Adam are FP32 vector
// code.  Parameters are one flat FP32 buffer:
//   W1 (H1 x D), b1 (H1), W2 (H2 x H1), b2 (H2), W3 (d x H2), b3 (d).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "fsne_context.h"

struct fsne_mlp {
  int32_t D = 0, H1 = 0, H2 = 0, d = 0, DP = 0, xdtype = 0;
  fsne_mlp_opts opts{};
  int64_t np = 0;
  int64_t t = 0;               // Adam steps taken
  hipStream_t stream = nullptr;
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;   // params, grad, Adam moments
  float *ymean = nullptr, *ystd = nullptr;                            // d each
  float *Xb = nullptr, *Tb = nullptr, *H1b = nullptr, *H2b = nullptr; // batch buffers
  float *Ob = nullptr, *dOb = nullptr, *dH1 = nullptr, *dH2 = nullptr;
  float* lpart = nullptr;      // loss partial sums
  float* ws = nullptr;         // split-K partial products
  float* part = nullptr;       // row-chunk partial sums (bias and output-layer gradients)
  void* xstage = nullptr;      // host-batch staging (input dtype)
  std::string err;
};

namespace {

using namespace fsne;

constexpr int kBM = 64, kBN = 64, kBK = 32, kLDP = kBK + 8;
constexpr int kTM = 64, kTN = 64, kTK = 64, kTP = kTK + 8;   // vector-staged tiles
constexpr int kMaxSplit = 8;      // split-K factor limit of the weight-gradient products
constexpr int kRowChunk = 16;     // rows per partial sum of the column reductions
constexpr int kLossBlocks = 256;
enum { kEpiBias = 1, kEpiRelu = 2, kEpiMask = 4 };

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

struct GemmArgs {
  const float* A;
  int64_t sam, sak;        // A(m, k) = A[m sam + k sak]
  const float* B;
  int64_t sbk, sbn;        // B(k, n) = B[k sbk + n sbn]
  float* C;
  int64_t ldc;             // C(m, n) = C[m ldc + n]
  int M, N, K;
  const float* bias;       // C(m, n) += bias[n]
  const float* mask;       // C(m, n) = 0 where mask[m ldm + n] <= 0
  int64_t ldm;
  int epi;
  float* ws;               // split-K: partial C of split z at ws + z M N (row stride N)
  int kchunk;              // split-K: K range of one split (a multiple of kTK)
};

__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// C = A B (+ bias, ReLU, mask).  64 x 64 tiles, 4 waves of 32 x 32, K steps
// of 32 staged in LDS as bfloat16, v_mfma_f32_32x32x16_bf16.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kBM][kLDP];   // [m][k]
  __shared__ __align__(16) uint16_t Bs[kBN][kLDP];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int bm = blockIdx.y * kBM, bn = blockIdx.x * kBN;
  const bool a_k = g.sak == 1, b_k = g.sbk == 1;     // contiguous index of each operand
  f32x16 acc = {};
  for (int k0 = 0; k0 < g.K; k0 += kBK) {
    for (int e = tid; e < kBM * kBK; e += 256) {
      const int m = a_k ? e / kBK : e % kBM, k = a_k ? e % kBK : e / kBM;
      const int gm = bm + m, gk = k0 + k;
      const float v = (gm < g.M && gk < g.K) ? g.A[(int64_t)gm * g.sam + (int64_t)gk * g.sak] : 0.0f;
      As[m][k] = to_bf16(v);
    }
    for (int e = tid; e < kBN * kBK; e += 256) {
      const int n = b_k ? e / kBK : e % kBN, k = b_k ? e % kBK : e / kBN;
      const int gn = bn + n, gk = k0 + k;
      const float v = (gn < g.N && gk < g.K) ? g.B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn] : 0.0f;
      Bs[n][k] = to_bf16(v);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kBK; s += 16) {
      const int kk = s + (lane >> 5) * 8;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + (lane & 31)][kk]);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + (lane & 31)][kk]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int n = bn + wn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = bm + wm * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
    if (m < g.M && n < g.N) {
      float v = acc[r];
      if (g.epi & kEpiBias) v += g.bias[n];
      if (g.epi & kEpiRelu) v = v > 0.0f ? v : 0.0f;
      if (g.epi & kEpiMask) v = g.mask[(int64_t)m * g.ldm + n] > 0.0f ? v : 0.0f;
      g.C[(int64_t)m * g.ldc + n] = v;
    }
  }
}

// Four consecutive elements p[0..3] of an operand along its contiguous index,
// which starts at c; elements at or beyond lim read as 0.
__device__ __forceinline__ float4 load4(const float* p, int c, int lim) {
  if (c + 3 < lim) return *reinterpret_cast<const float4*>(p);
  float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (c < lim) v.x = p[0];
  if (c + 1 < lim) v.y = p[1];
  if (c + 2 < lim) v.z = p[2];
  return v;
}

__device__ __forceinline__ uint2 pack4_bf16(float4 v) {
  return make_uint2((uint32_t)to_bf16(v.x) | ((uint32_t)to_bf16(v.y) << 16),
                    (uint32_t)to_bf16(v.z) | ((uint32_t)to_bf16(v.w) << 16));
}

// One 64 x 64 FP32 tile of an operand as 4 float4 per thread.  KC: the
// operand is contiguous along k (rows r of the tile are its m or n index),
// and each thread loads 4 rows of 4 k; otherwise it is contiguous along
// m / n, and each thread loads a 4 (k) x 4 (r) block, so that it can store
// 4 consecutive k of one row at once.
template <bool KC>
__device__ __forceinline__ void tile_load(const float* __restrict__ P, int64_t s_r, int64_t s_k,
                                          int r0, int rlim, int k0, int klim, float4* v) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int idx = tid + 256 * j;
    if constexpr (KC) {
      const int r = idx >> 4, k = (idx & 15) << 2;
      const int gr = r0 + r, gk = k0 + k;
      v[j] = gr < rlim ? load4(P + (int64_t)gr * s_r + gk, gk, klim)
                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    } else {
      const int k = ((tid >> 4) << 2) + j, r = (tid & 15) << 2;
      const int gr = r0 + r, gk = k0 + k;
      v[j] = gk < klim ? load4(P + (int64_t)gk * s_k + gr, gr, rlim)
                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  }
}

// Rounds the tile to bfloat16 into LDS, laid out [row][k].
template <bool KC>
__device__ __forceinline__ void tile_store(uint16_t (*L)[kTP], const float4* v) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int idx = tid + 256 * j;
    if constexpr (KC) {
      const int r = idx >> 4, k = (idx & 15) << 2;
      *reinterpret_cast<uint2*>(&L[r][k]) = pack4_bf16(v[j]);
    }
  }
  if constexpr (!KC) {
    // v[j] holds rows r .. r+3 at k + j: row r + i gets k .. k+3 in one store
    const int k = (tid >> 4) << 2, r = (tid & 15) << 2;
    const float c[4][4] = {{v[0].x, v[1].x, v[2].x, v[3].x}, {v[0].y, v[1].y, v[2].y, v[3].y},
                           {v[0].z, v[1].z, v[2].z, v[3].z}, {v[0].w, v[1].w, v[2].w, v[3].w}};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      *reinterpret_cast<uint2*>(&L[r + i][k]) =
          pack4_bf16(make_float4(c[i][0], c[i][1], c[i][2], c[i][3]));
  }
}

// C = A B (+ bias, ReLU, mask) with 16-byte operand loads and the next K tile
// loaded into registers while the current one is multiplied.  AK / BK: A / B
// contiguous along k (else along m / n).  With gridDim.z > 1 each z-slice
// multiplies one K range and writes its partial product to ws (no epilogue).
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm_v(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kTM][kTP];
  __shared__ __align__(16) uint16_t Bs[kTN][kTP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int bm = blockIdx.y * kTM, bn = blockIdx.x * kTN;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int64_t a_r = AK ? g.sam : 0, a_k = AK ? 0 : g.sak;
  const int64_t b_r = BK ? g.sbn : 0, b_k = BK ? 0 : g.sbk;
  float4 ra[4], rb[4];
  tile_load<AK>(g.A, a_r, a_k, bm, g.M, kbeg, kend, ra);
  tile_load<BK>(g.B, b_r, b_k, bn, g.N, kbeg, kend, rb);
  f32x16 acc = {};
  for (int k0 = kbeg; k0 < kend; k0 += kTK) {
    tile_store<AK>(As, ra);
    tile_store<BK>(Bs, rb);
    __syncthreads();
    if (k0 + kTK < kend) {
      tile_load<AK>(g.A, a_r, a_k, bm, g.M, k0 + kTK, kend, ra);
      tile_load<BK>(g.B, b_r, b_k, bn, g.N, k0 + kTK, kend, rb);
    }
#pragma unroll
    for (int s = 0; s < kTK; s += 16) {
      const int kk = s + (lane >> 5) * 8;
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + (lane & 31)][kk]);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + (lane & 31)][kk]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int n = bn + wn * 32 + (lane & 31);
  if (gridDim.z > 1) {
    float* w = g.ws + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = bm + wm * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
      if (m < g.M && n < g.N) w[(int64_t)m * g.N + n] = acc[r];
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = bm + wm * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
    if (m < g.M && n < g.N) {
      float v = acc[r];
      if (g.epi & kEpiBias) v += g.bias[n];
      if (g.epi & kEpiRelu) v = v > 0.0f ? v : 0.0f;
      if (g.epi & kEpiMask) v = g.mask[(int64_t)m * g.ldm + n] > 0.0f ? v : 0.0f;
      g.C[(int64_t)m * g.ldc + n] = v;
    }
  }
}

// C(m, n) = sum over z of the split-K partials, in split order.
__global__ void k_splitk_sum(const float* ws, int S, int M, int N, float* C, int64_t ldc) {
  const int64_t total = (int64_t)M * N;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.0f;
    for (int z = 0; z < S; ++z) v += ws[(int64_t)z * total + q];
    C[(q / N) * ldc + q % N] = v;
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

hipError_t gemm(hipStream_t s, const float* A, int64_t sam, int64_t sak, const float* B,
                int64_t sbk, int64_t sbn, float* C, int64_t ldc, int M, int N, int K, int epi,
                const float* bias = nullptr, const float* mask = nullptr, int64_t ldm = 0,
                float* ws = nullptr) {
  GemmArgs g{A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, bias, mask, ldm, epi, ws, K};
  const bool ak = sak == 1, bk = sbk == 1;
  const bool a_ok = ak ? (sam % 4 == 0) : (sam == 1 && sak % 4 == 0);
  const bool b_ok = bk ? (sbn % 4 == 0) : (sbn == 1 && sbk % 4 == 0);
  if (!(a_ok && b_ok && aligned16(A) && aligned16(B))) {
    const dim3 grid((unsigned)((N + kBN - 1) / kBN), (unsigned)((M + kBM - 1) / kBM));
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
    return hipGetLastError();
  }
  const int tiles = ((N + kTN - 1) / kTN) * ((M + kTM - 1) / kTM);
  int S = 1;
  if (epi == 0 && ws && tiles < 256) {
    // enough slices to fill the chip, each still at least 256 deep in K
    S = std::min(kMaxSplit, std::max(1, 512 / tiles));
    while (S > 1 && K / S < 256) --S;
  }
  g.kchunk = S > 1 ? ((K + S - 1) / S + kTK - 1) / kTK * kTK : K;
  S = (K + g.kchunk - 1) / g.kchunk;
  const dim3 grid((unsigned)((N + kTN - 1) / kTN), (unsigned)((M + kTM - 1) / kTM), (unsigned)S);
  if (ak && bk)
    hipLaunchKernelGGL((k_gemm_v<true, true>), grid, dim3(256), 0, s, g);
  else if (ak && !bk)
    hipLaunchKernelGGL((k_gemm_v<true, false>), grid, dim3(256), 0, s, g);
  else if (!ak && bk)
    hipLaunchKernelGGL((k_gemm_v<false, true>), grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((k_gemm_v<false, false>), grid, dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  hipLaunchKernelGGL(k_splitk_sum, dim3(1024), dim3(256), 0, s, ws, S, M, N, C, ldc);
  return hipGetLastError();
}

// Batch rows: row k is source row (off + k) mod N of X (FP32 or BF16 bits),
// converted to FP32; targets (y - mean) / std from Y (padded stride DP).
// One block per row at a time.
__global__ void k_gather(const void* X, int xdtype, int D, int64_t N, int64_t off, int n,
                         const float* Y, int DP, int d, const float* mean, const float* sd,
                         float* Xb, float* Tb) {
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const int64_t r = (off + k) % N;
    float* dst = Xb + (int64_t)k * D;
    if (xdtype == 0) {
      const float* src = static_cast<const float*>(X) + r * D;
      for (int c = threadIdx.x; c < D; c += blockDim.x) dst[c] = src[c];
    } else {
      const uint16_t* src = static_cast<const uint16_t*>(X) + r * D;
      for (int c = threadIdx.x; c < D; c += blockDim.x)
        dst[c] = __uint_as_float((uint32_t)src[c] << 16);
    }
    if (Y && (int)threadIdx.x < d) {
      const int c = threadIdx.x;
      Tb[(int64_t)k * d + c] = (Y[r * DP + c] - mean[c]) / sd[c];
    }
  }
}

// Output layer: O[r][j] = b3[j] + sum_k H2[r][k] W3[j][k]; one wave per row.
__global__ void k_out_layer(const float* H2, const float* W3, const float* b3, int n, int H,
                            int d, float* O) {
  const int r = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (r >= n) return;
  const int lane = lane_id();
  for (int j = 0; j < d; ++j) {
    float s = 0.0f;
    for (int k = lane; k < H; k += kWave) s = fmaf(H2[(int64_t)r * H + k], W3[(int64_t)j * H + k], s);
    s = wave_sum_uniform(s);
    if (lane == 0) O[(int64_t)r * d + j] = s + b3[j];
  }
}

// dO = 2 (O - T) / (n d); per-block partial sums of (O - T)^2, added to the
// block's running sum when accumulate is set.
__global__ void k_dout(const float* O, const float* T, int64_t cnt, float scale, float* dO,
                       float* lpart, int accumulate) {
  __shared__ float sl[256];
  float l = 0.0f;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < cnt; q += (int64_t)gridDim.x * 256) {
    const float e = O[q] - T[q];
    dO[q] = 2.0f * e * scale;
    l = fmaf(e, e, l);
  }
  sl[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) sl[threadIdx.x] += sl[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = (accumulate ? lpart[blockIdx.x] : 0.0f) + sl[0];
}

// Output-layer gradient over one chunk of rows (blockIdx.y), in row order:
//   part[c][j (H+1) + k] = sum_r dO[r][j] H2[r][k]   (k < H)
//   part[c][j (H+1) + H] = sum_r dO[r][j]
__global__ void k_grad_out_part(const float* dO, const float* H2, int n, int H, int d,
                                float* part) {
  const int Q = d * (H + 1);
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  const int j = q / (H + 1), k = q % (H + 1);
  const int r0 = blockIdx.y * kRowChunk, r1 = min(n, r0 + kRowChunk);
  float s = 0.0f;
  if (k < H) {
    for (int r = r0; r < r1; ++r) s = fmaf(dO[(int64_t)r * d + j], H2[(int64_t)r * H + k], s);
  } else {
    for (int r = r0; r < r1; ++r) s += dO[(int64_t)r * d + j];
  }
  part[(int64_t)blockIdx.y * Q + q] = s;
}

// Sum over the nchunk partials part[c * stride + q] of one output q: one
// wave, lane l taking chunks l, l + 64, ... in order, then a fixed tree.
__device__ __forceinline__ float sum_chunks(const float* part, int nchunk, int64_t stride,
                                            int q) {
  float s = 0.0f;
  for (int c = lane_id(); c < nchunk; c += kWave) s += part[(int64_t)c * stride + q];
  return wave_sum_uniform(s);
}

// gW3 / gb3 from the chunk partials; one wave per output.
__global__ void k_grad_out_sum(const float* part, int nchunk, int H, int d, float* gW3,
                               float* gb3) {
  const int Q = d * (H + 1);
  const int q = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (q >= Q) return;
  const float s = sum_chunks(part, nchunk, Q, q);
  if (lane_id() != 0) return;
  const int j = q / (H + 1), k = q % (H + 1);
  if (k < H)
    gW3[(int64_t)j * H + k] = s;
  else
    gb3[j] = s;
}

// dH2[r][k] = (sum_j dO[r][j] W3[j][k]) where H2[r][k] > 0, else 0.
__global__ void k_back_out(const float* dO, const float* W3, const float* H2, int n, int H, int d,
                           float* dH2) {
  const int64_t total = (int64_t)n * H;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q / H, k = q % H;
    float s = 0.0f;
    for (int j = 0; j < d; ++j) s = fmaf(dO[r * d + j], W3[(int64_t)j * H + k], s);
    dH2[q] = H2[q] > 0.0f ? s : 0.0f;
  }
}

// Column sums of M (n x cols) over one chunk of rows (blockIdx.y), in row order.
__global__ void k_colsum_part(const float* M, int n, int cols, float* part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const int r0 = blockIdx.y * kRowChunk, r1 = min(n, r0 + kRowChunk);
  float s = 0.0f;
  for (int r = r0; r < r1; ++r) s += M[(int64_t)r * cols + c];
  part[(int64_t)blockIdx.y * cols + c] = s;
}

// out[c] = sum of the chunk partials of column c; one wave per column.
__global__ void k_sum_parts(const float* part, int nchunk, int cols, float* out) {
  const int c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (c >= cols) return;
  const float s = sum_chunks(part, nchunk, cols, c);
  if (lane_id() == 0) out[c] = s;
}

// Adam (Kingma and Ba 2015) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void k_adam(float* p, float* m, float* v, const float* g, int64_t np, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < np;
       k += (int64_t)gridDim.x * blockDim.x) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  }
}

// He-uniform initialisation: w = (2u - 1) sqrt(6 / fan_in) with u = (draw >> 8)
// 2^-24 from Philox block (index, layer, 8, 0); biases 0.
__global__ void k_init(float* p, int64_t n_w, int64_t n_b, int layer, int fan_in, uint32_t k0,
                       uint32_t k1) {
#pragma clang fp contract(off)
  const float ratio = 6.0f / (float)fan_in;
  const float bound = sqrtf(ratio);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_w + n_b;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (k < n_w) {
      const uint4 u = philox((uint32_t)k, (uint32_t)layer, 8u, 0u, k0, k1);
      const float unit = (float)(u.x >> 8) * 5.9604644775390625e-08f;
      const float two_u = 2.0f * unit;
      const float centred = two_u - 1.0f;
      p[k] = centred * bound;
    } else {
      p[k] = 0.0f;
    }
  }
}

// Per-component mean and standard deviation of Y (N rows, stride DP), two
// passes, fixed order; one block per component.
__global__ void k_ystats(const float* Y, int64_t N, int DP, float* mean, float* sd) {
  __shared__ float s[256];
  const int c = blockIdx.x;
  float a = 0.0f;
  for (int64_t r = threadIdx.x; r < N; r += 256) a += Y[r * DP + c];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  const float mu = s[0] / (float)N;
  __syncthreads();
  float b = 0.0f;
  for (int64_t r = threadIdx.x; r < N; r += 256) {
    const float e = Y[r * DP + c] - mu;
    b = fmaf(e, e, b);
  }
  s[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[c] = mu;
    const float v = s[0] / (float)N;
    sd[c] = v > 0.0f ? sqrtf(v) : 1.0f;
  }
}

// y = O * std + mean.
__global__ void k_unstandardise(const float* O, int n, int d, const float* mean, const float* sd,
                                float* Y) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n * d) Y[q] = O[q] * sd[q % d] + mean[q % d];
}

fsne_status mfail(fsne_mlp* m, fsne_status st, const std::string& msg) {
  if (m) m->err = msg;
  return st;
}

#define MCHK(m, expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return mfail(m, FSNE_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define MTRY(expr)                 \
  do {                             \
    fsne_status s_ = (expr);       \
    if (s_ != FSNE_OK) return s_;  \
  } while (0)

struct Views {
  float *W1, *b1, *W2, *b2, *W3, *b3;
};

Views views(const fsne_mlp* m, float* base) {
  Views v;
  v.W1 = base;
  v.b1 = v.W1 + (int64_t)m->H1 * m->D;
  v.W2 = v.b1 + m->H1;
  v.b2 = v.W2 + (int64_t)m->H2 * m->H1;
  v.W3 = v.b2 + m->H2;
  v.b3 = v.W3 + (int64_t)m->d * m->H2;
  return v;
}

// Forward of n batch rows already in Xb: H1b, H2b, Ob.
fsne_status forward(fsne_mlp* m, int n) {
  hipStream_t s = m->stream;
  const Views P = views(m, m->P);
  MCHK(m, gemm(s, m->Xb, m->D, 1, P.W1, 1, m->D, m->H1b, m->H1, n, m->H1, m->D,
               kEpiBias | kEpiRelu, P.b1));
  MCHK(m, gemm(s, m->H1b, m->H1, 1, P.W2, 1, m->H1, m->H2b, m->H2, n, m->H2, m->H1,
               kEpiBias | kEpiRelu, P.b2));
  hipLaunchKernelGGL(k_out_layer, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, m->H2b, P.W3,
                     P.b3, n, m->H2, m->d, m->Ob);
  MCHK(m, hipGetLastError());
  return FSNE_OK;
}

// Column sums of an n x cols batch matrix into out, via row-chunk partials.
fsne_status colsum(fsne_mlp* m, const float* M, int n, int cols, float* out) {
  const int nchunk = (n + kRowChunk - 1) / kRowChunk;
  const unsigned gx = (unsigned)((cols + 255) / 256);
  hipLaunchKernelGGL(k_colsum_part, dim3(gx, (unsigned)nchunk), dim3(256), 0, m->stream, M, n,
                     cols, m->part);
  MCHK(m, hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((cols + 3) / 4)), dim3(256), 0, m->stream,
                     m->part, nchunk, cols, out);
  MCHK(m, hipGetLastError());
  return FSNE_OK;
}

// Loss and gradient (into G) of n batch rows with targets in Tb; the loss
// partials are added to the running sums when accumulate is set.
fsne_status backward(fsne_mlp* m, int n, int accumulate = 0) {
  hipStream_t s = m->stream;
  const Views P = views(m, m->P);
  const Views Gv = views(m, m->G);
  const int64_t cnt = (int64_t)n * m->d;
  hipLaunchKernelGGL(k_dout, dim3(kLossBlocks), dim3(256), 0, s, m->Ob, m->Tb, cnt,
                     1.0f / (float)cnt, m->dOb, m->lpart, accumulate);
  MCHK(m, hipGetLastError());
  const int q = m->d * (m->H2 + 1);
  const int nchunk = (n + kRowChunk - 1) / kRowChunk;
  hipLaunchKernelGGL(k_grad_out_part, dim3((unsigned)((q + 255) / 256), (unsigned)nchunk),
                     dim3(256), 0, s, m->dOb, m->H2b, n, m->H2, m->d, m->part);
  MCHK(m, hipGetLastError());
  hipLaunchKernelGGL(k_grad_out_sum, dim3((unsigned)((q + 3) / 4)), dim3(256), 0, s, m->part,
                     nchunk, m->H2, m->d, Gv.W3, Gv.b3);
  MCHK(m, hipGetLastError());
  hipLaunchKernelGGL(k_back_out, dim3(1024), dim3(256), 0, s, m->dOb, P.W3, m->H2b, n, m->H2,
                     m->d, m->dH2);
  MCHK(m, hipGetLastError());
  // gW2 = dH2^T H1, gb2 = column sums of dH2
  MCHK(m, gemm(s, m->dH2, 1, m->H2, m->H1b, m->H1, 1, Gv.W2, m->H1, m->H2, m->H1, n, 0,
               nullptr, nullptr, 0, m->ws));
  MTRY(colsum(m, m->dH2, n, m->H2, Gv.b2));
  // dH1 = (dH2 W2) where H1 > 0
  MCHK(m, gemm(s, m->dH2, m->H2, 1, P.W2, m->H1, 1, m->dH1, m->H1, n, m->H1, m->H2, kEpiMask,
               nullptr, m->H1b, m->H1));
  // gW1 = dH1^T X, gb1 = column sums of dH1
  MCHK(m, gemm(s, m->dH1, 1, m->H1, m->Xb, m->D, 1, Gv.W1, m->D, m->H1, m->D, n, 0,
               nullptr, nullptr, 0, m->ws));
  MTRY(colsum(m, m->dH1, n, m->H1, Gv.b1));
  return FSNE_OK;
}

fsne_status adam(fsne_mlp* m) {
  m->t += 1;
  const fsne_mlp_opts& o = m->opts;
  const float c1 = 1.0f - powf(o.beta1, (float)m->t), c2 = 1.0f - powf(o.beta2, (float)m->t);
  hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, m->stream, m->P, m->Mo, m->Vo, m->G, m->np,
                     o.lr, o.beta1, o.beta2, o.eps, c1, c2);
  MCHK(m, hipGetLastError());
  return FSNE_OK;
}

template <typename T>
fsne_status malloc_dev(fsne_mlp* m, T** p, size_t n) {
  void* q = nullptr;
  if (hipMalloc(&q, sizeof(T) * (n ? n : 1)) != hipSuccess)
    return mfail(m, FSNE_ENOMEM, "hipMalloc failed");
  *p = static_cast<T*>(q);
  return FSNE_OK;
}


// Host batch (n rows of the input dtype, targets T n x d or NULL) to Xb / Tb.
fsne_status upload_batch(fsne_mlp* m, const void* X, const float* T, int64_t n) {
  const size_t xb = m->xdtype == FSNE_F32 ? 4 : 2;
  MCHK(m, hipMemcpyAsync(m->xstage, X, (size_t)n * m->D * xb, hipMemcpyHostToDevice, m->stream));
  hipLaunchKernelGGL(k_gather, dim3(1024), dim3(256), 0, m->stream, m->xstage, m->xdtype, m->D,
                     n, (int64_t)0, (int)n, nullptr, 0, 0, nullptr, nullptr, m->Xb, nullptr);
  MCHK(m, hipGetLastError());
  if (T)
    MCHK(m, hipMemcpyAsync(m->Tb, T, sizeof(float) * n * m->d, hipMemcpyHostToDevice, m->stream));
  return FSNE_OK;
}

float loss_of(fsne_mlp* m, int64_t cnt) {
  float part[kLossBlocks];
  if (hipMemcpyAsync(part, m->lpart, sizeof part, hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return NAN;
  double s = 0.0;
  for (float v : part) s += v;
  return (float)(s / (double)cnt);
}

}  // namespace

extern "C" {

fsne_status fsne_mlp_default_opts(fsne_mlp_opts* o) {
  if (!o) return FSNE_EINVAL;
  o->hidden1 = 512;
  o->hidden2 = 512;
  o->epochs = 5;
  o->batch = 4096;
  o->lr = 1e-3f;
  o->beta1 = 0.9f;
  o->beta2 = 0.999f;
  o->eps = 1e-8f;
  o->seed = 1;
  return FSNE_OK;
}

fsne_status fsne_mlp_create(const fsne_ctx* ctx, const fsne_mlp_opts* opts, fsne_mlp** out) {
  if (!out) return FSNE_EINVAL;
  *out = nullptr;
  if (!ctx || !opts) return FSNE_EINVAL;
  if (opts->hidden1 < 1 || opts->hidden2 < 1 || opts->hidden1 > 16384 || opts->hidden2 > 16384 ||
      opts->epochs < 0 || opts->batch < 1 || opts->batch > (1 << 20) || !(opts->lr >= 0.0f) ||
      !(opts->beta1 >= 0.0f && opts->beta1 < 1.0f) || !(opts->beta2 >= 0.0f && opts->beta2 < 1.0f) ||
      !(opts->eps > 0.0f))
    return FSNE_EINVAL;
  fsne_mlp* m = new (std::nothrow) fsne_mlp();
  if (!m) return FSNE_ENOMEM;
  m->D = ctx->D;
  m->d = ctx->d;
  m->DP = ctx->DP;
  m->xdtype = ctx->xdtype;
  m->H1 = opts->hidden1;
  m->H2 = opts->hidden2;
  m->opts = *opts;
  m->np = (int64_t)m->H1 * m->D + m->H1 + (int64_t)m->H2 * m->H1 + m->H2 + (int64_t)m->d * m->H2 + m->d;
  const size_t B = (size_t)opts->batch;
  auto bad = [&](fsne_status st) {
    fsne_mlp_destroy(m);
    return st;
  };
  if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) return bad(FSNE_EHIP);
  fsne_status st;
  if ((st = malloc_dev(m, &m->P, m->np)) || (st = malloc_dev(m, &m->G, m->np)) ||
      (st = malloc_dev(m, &m->Mo, m->np)) || (st = malloc_dev(m, &m->Vo, m->np)) ||
      (st = malloc_dev(m, &m->ymean, m->d)) || (st = malloc_dev(m, &m->ystd, m->d)) ||
      (st = malloc_dev(m, &m->Xb, B * m->D)) || (st = malloc_dev(m, &m->Tb, B * m->d)) ||
      (st = malloc_dev(m, &m->H1b, B * m->H1)) || (st = malloc_dev(m, &m->H2b, B * m->H2)) ||
      (st = malloc_dev(m, &m->Ob, B * m->d)) || (st = malloc_dev(m, &m->dOb, B * m->d)) ||
      (st = malloc_dev(m, &m->dH1, B * m->H1)) || (st = malloc_dev(m, &m->dH2, B * m->H2)) ||
      (st = malloc_dev(m, &m->lpart, kLossBlocks)) ||
      (st = malloc_dev(m, &m->ws, (size_t)kMaxSplit *
                                      std::max<size_t>((size_t)m->H1 * m->D, (size_t)m->H2 * m->H1))) ||
      (st = malloc_dev(m, &m->part, ((B + kRowChunk - 1) / kRowChunk) *
                                        std::max<size_t>(std::max(m->H1, m->H2),
                                                         (size_t)m->d * (m->H2 + 1)))) ||
      (st = malloc_dev(m, reinterpret_cast<uint8_t**>(&m->xstage), B * m->D * 4)))
    return bad(st);
  if (hipMemsetAsync(m->Mo, 0, sizeof(float) * m->np, m->stream) != hipSuccess ||
      hipMemsetAsync(m->Vo, 0, sizeof(float) * m->np, m->stream) != hipSuccess)
    return bad(FSNE_EHIP);
  const Views P = views(m, m->P);
  float* layer_base[3] = {P.W1, P.W2, P.W3};
  const int64_t n_w[3] = {(int64_t)m->H1 * m->D, (int64_t)m->H2 * m->H1, (int64_t)m->d * m->H2};
  const int64_t n_b[3] = {m->H1, m->H2, m->d};
  const int fan[3] = {m->D, m->H1, m->H2};
  for (int l = 0; l < 3; ++l) {
    hipLaunchKernelGGL(k_init, dim3(1024), dim3(256), 0, m->stream, layer_base[l], n_w[l], n_b[l], l,
                       fan[l], (uint32_t)opts->seed, (uint32_t)(opts->seed >> 32));
    if (hipGetLastError() != hipSuccess) return bad(FSNE_EHIP);
  }
  // standardisation defaults: mean 0, std 1 (train sets them from the data)
  float zeros[64] = {0}, ones[64];
  for (float& v : ones) v = 1.0f;
  if (m->d > 64 ||
      hipMemcpyAsync(m->ymean, zeros, sizeof(float) * m->d, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
      hipMemcpyAsync(m->ystd, ones, sizeof(float) * m->d, hipMemcpyHostToDevice, m->stream) != hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess)
    return bad(FSNE_EHIP);
  *out = m;
  return FSNE_OK;
}

int64_t fsne_mlp_num_params(const fsne_mlp* m) { return m ? m->np : -1; }

fsne_status fsne_mlp_train(fsne_mlp* m, fsne_ctx* ctx, float* final_loss) {
  if (!m || !ctx) return FSNE_EINVAL;
  if (ctx->D != m->D || ctx->d != m->d || ctx->xdtype != m->xdtype)
    return mfail(m, FSNE_EINVAL, "context does not match the network's shape");
  MCHK(m, hipStreamSynchronize(ctx->stream));
  const int64_t N = ctx->N;
  hipLaunchKernelGGL(k_ystats, dim3((unsigned)m->d), dim3(256), 0, m->stream, ctx->Y, N, ctx->DP,
                     m->ymean, m->ystd);
  MCHK(m, hipGetLastError());
  const int64_t B = m->opts.batch;
  const int64_t nb = (N + B - 1) / B;
  MCHK(m, hipMemsetAsync(m->lpart, 0, sizeof(float) * kLossBlocks, m->stream));
  for (int e = 0; e < m->opts.epochs; ++e) {
    const int64_t off = ((int64_t)e * 104729) % N;
    const int last = e == m->opts.epochs - 1;
    for (int64_t b = 0; b < nb; ++b) {
      const int n = (int)std::min<int64_t>(B, N - b * B);
      hipLaunchKernelGGL(k_gather, dim3(1024), dim3(256), 0, m->stream, ctx->X, ctx->xdtype, m->D,
                         N, off + b * B, n, ctx->Y, ctx->DP, m->d, m->ymean, m->ystd, m->Xb, m->Tb);
      MCHK(m, hipGetLastError());
      MTRY(forward(m, n));
      MTRY(backward(m, n, last));
      MTRY(adam(m));
    }
  }
  // mean squared error over the last epoch (each of the N rows once)
  if (final_loss) *final_loss = m->opts.epochs > 0 ? loss_of(m, N * m->d) : NAN;
  MCHK(m, hipStreamSynchronize(m->stream));
  return FSNE_OK;
}

fsne_status fsne_mlp_predict(fsne_mlp* m, const void* X, int64_t n, float* Y) {
  if (!m) return FSNE_EINVAL;
  if (!X || !Y || n < 0) return mfail(m, FSNE_EINVAL, "bad arguments to fsne_mlp_predict");
  const int64_t B = m->opts.batch;
  const size_t xb = m->xdtype == FSNE_F32 ? 4 : 2;
  for (int64_t s = 0; s < n; s += B) {
    const int k = (int)std::min<int64_t>(B, n - s);
    MTRY(upload_batch(m, static_cast<const uint8_t*>(X) + (size_t)s * m->D * xb, nullptr, k));
    MTRY(forward(m, k));
    hipLaunchKernelGGL(k_unstandardise, dim3((unsigned)((k * m->d + 255) / 256)), dim3(256), 0,
                       m->stream, m->Ob, k, m->d, m->ymean, m->ystd, m->dOb);
    MCHK(m, hipGetLastError());
    MCHK(m, hipMemcpyAsync(Y + s * m->d, m->dOb, sizeof(float) * k * m->d, hipMemcpyDeviceToHost,
                           m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
  }
  return FSNE_OK;
}

fsne_status fsne_mlp_get_params(fsne_mlp* m, float* params, float* ymean, float* ystd) {
  if (!m) return FSNE_EINVAL;
  if (params) MCHK(m, hipMemcpyAsync(params, m->P, sizeof(float) * m->np, hipMemcpyDeviceToHost, m->stream));
  if (ymean) MCHK(m, hipMemcpyAsync(ymean, m->ymean, sizeof(float) * m->d, hipMemcpyDeviceToHost, m->stream));
  if (ystd) MCHK(m, hipMemcpyAsync(ystd, m->ystd, sizeof(float) * m->d, hipMemcpyDeviceToHost, m->stream));
  MCHK(m, hipStreamSynchronize(m->stream));
  return FSNE_OK;
}

fsne_status fsne_mlp_set_params(fsne_mlp* m, const float* params, const float* ymean,
                                const float* ystd) {
  if (!m) return FSNE_EINVAL;
  if (params) MCHK(m, hipMemcpyAsync(m->P, params, sizeof(float) * m->np, hipMemcpyHostToDevice, m->stream));
  if (ymean) MCHK(m, hipMemcpyAsync(m->ymean, ymean, sizeof(float) * m->d, hipMemcpyHostToDevice, m->stream));
  if (ystd) MCHK(m, hipMemcpyAsync(m->ystd, ystd, sizeof(float) * m->d, hipMemcpyHostToDevice, m->stream));
  MCHK(m, hipStreamSynchronize(m->stream));
  return FSNE_OK;
}

fsne_status fsne_mlp_loss_grad(fsne_mlp* m, const void* X, const float* T, int64_t n, float* grad,
                               float* loss) {
  if (!m) return FSNE_EINVAL;
  if (!X || !T || n < 1 || n > m->opts.batch)
    return mfail(m, FSNE_EINVAL, "bad arguments to fsne_mlp_loss_grad");
  MTRY(upload_batch(m, X, T, n));
  MTRY(forward(m, (int)n));
  MTRY(backward(m, (int)n));
  if (grad)
    MCHK(m, hipMemcpyAsync(grad, m->G, sizeof(float) * m->np, hipMemcpyDeviceToHost, m->stream));
  const float l = loss_of(m, n * m->d);
  if (loss) *loss = l;
  return FSNE_OK;
}

fsne_status fsne_mlp_train_batch(fsne_mlp* m, const void* X, const float* T, int64_t n) {
  if (!m) return FSNE_EINVAL;
  if (!X || !T || n < 1 || n > m->opts.batch)
    return mfail(m, FSNE_EINVAL, "bad arguments to fsne_mlp_train_batch");
  MTRY(upload_batch(m, X, T, n));
  MTRY(forward(m, (int)n));
  MTRY(backward(m, (int)n));
  MTRY(adam(m));
  MCHK(m, hipStreamSynchronize(m->stream));
  return FSNE_OK;
}

void fsne_mlp_destroy(fsne_mlp* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  void* bufs[] = {m->P, m->G, m->Mo, m->Vo, m->ymean, m->ystd, m->Xb, m->Tb, m->H1b, m->H2b,
                  m->Ob, m->dOb, m->dH1, m->dH2, m->lpart, m->ws, m->part, m->xstage};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

const char* fsne_mlp_last_error(const fsne_mlp* m) { return m ? m->err.c_str() : "null network"; }

}  // extern "C"
