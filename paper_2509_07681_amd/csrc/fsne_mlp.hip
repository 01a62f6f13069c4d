// Placement network for dynamic data: D -> H1 -> H2 -> d with ReLU hidden
// layers, trained by mean squared error on (x, standardised y) pairs of a
// context's embedding with Adam, then used to place inserted or drifted
// points.  The three large products run as BF16 MFMA GEMMs with FP32
// accumulation; their operands are kept in memory as bfloat16 (rounded to
// nearest even once, where they are produced: the batch rows by the gather,
// W1 and W2 by the optimiser step, H1, dH1 and dH2 by the kernels that
// compute them), so a GEMM reads half the bytes and converts nothing.  The
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
  float *Tb = nullptr, *H2b = nullptr, *Ob = nullptr, *dOb = nullptr, *dH2 = nullptr;  // batch, FP32
  uint16_t *Xb = nullptr, *H1b = nullptr, *dH1b = nullptr, *dH2b = nullptr;        // batch, BF16
  uint16_t *W1b = nullptr, *W2b = nullptr;   // W1, W2 rounded to BF16
  bool wdirty = true;          // W1b / W2b must be rounded again from P
  float* lpart = nullptr;      // loss partial sums
  float* ws = nullptr;         // split-K partial products of the W1 gradient
  float* ws2 = nullptr;        // split-K partial products of the W2 gradient
  float* part = nullptr;       // row-chunk partial sums of the b2 gradient
  float* part3 = nullptr;      // row-chunk partial sums of the W3 / b3 gradients
  float* colpart = nullptr;    // 64-row-block partial sums of the b1 gradient
  float* lchunk = nullptr;     // loss of each row chunk
  bool fused_head = false;     // output layer, loss and dH2 in one kernel (k_head)
  void* xstage = nullptr;      // host-batch staging (input dtype)
  std::string err;
};

namespace {

using namespace fsne;

constexpr int kBM = 64, kBN = 64, kBK = 32, kLDP = kBK + 8;
constexpr int kTM = 64, kTN = 64, kTK = 64;   // vector-staged tiles: 64 x 64 per sub-tile
constexpr int kMaxSplit = 8;      // split-K factor limit of the weight-gradient products
constexpr int kRowChunk = 16;     // rows per partial sum of the column reductions
constexpr int kLossBlocks = 256;
enum { kEpiBias = 1, kEpiRelu = 2, kEpiMask = 4, kEpiColSum = 8 };

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

struct GemmArgs {
  const uint16_t* A;       // bfloat16 bits
  int64_t sam, sak;        // A(m, k) = A[m sam + k sak]
  const uint16_t* B;       // bfloat16 bits
  int64_t sbk, sbn;        // B(k, n) = B[k sbk + n sbn]
  float* C;                // FP32 output, or
  uint16_t* Cb;            // bfloat16 output (rounded to nearest even)
  int64_t ldc;             // C(m, n) = C[m ldc + n]
  int M, N, K;
  const float* bias;       // C(m, n) += bias[n]
  const uint16_t* mask;    // C(m, n) = 0 unless the bfloat16 mask[m ldm + n] > 0
  int64_t ldm;
  int epi;
  float* ws;               // partials mode: the product of split z (no epilogue) at
                           // ws + z M N (row stride N), split z covering one K range
  int kchunk;              // K range of one split (a multiple of the K step)
  float* colpart;          // with kEpiColSum: colpart[by N + n] = sum over the 64
                           // rows of row block by of C(m, n) after the epilogue
};

// bfloat16 bits of f, rounded to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// True where the bfloat16 value is > 0 (sign clear, not zero).
__device__ __forceinline__ bool bf16_pos(uint16_t b) { return b != 0 && !(b & 0x8000u); }

// The tile (bx, by, bz) a block computes.  Workgroups go to the chip's
// eight XCDs in turn (linear id mod 8), each XCD with its own L2; when the
// tiles divide evenly, XCD x takes the x-th contiguous eighth of the tiles
// in row-major order, so that the blocks sharing a row of A tiles (and most
// of B) read them through one L2 instead of eight.
struct Tile {
  int bx, by, bz;
};
__device__ __forceinline__ Tile block_tile() {
  const int gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const int T = gx * gy * gz;
  int t = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if ((T & 7) == 0) t = (t & 7) * (T >> 3) + (t >> 3);
  Tile r;
  r.bz = t / (gx * gy);
  const int rem = t - r.bz * gx * gy;
  r.by = rem / gx;
  r.bx = rem - r.by * gx;
  return r;
}

// Writes a block's 64 x 64 tile of C from the accumulators of its four
// waves (wave (wm, wn) holds rows wm 32 .. +32 and columns wn 32 .. +32;
// lane l, register r: column l mod 32, row (r mod 4) + 8 (r / 4) + 4 (l / 32)).
// Partials mode (g.ws): the raw product of this K split.  Otherwise bias,
// ReLU and mask as g.epi says, and with kEpiColSum the column sums of the
// tile, in a fixed order, to g.colpart.
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, const f32x16& acc, Tile tl,
                                              int wm, int wn, int lane, float (*colacc)[kBN]) {
  const int bm = tl.by * kBM, bn = tl.bx * kBN;
  const int n = bn + wn * 32 + (lane & 31);
  if (g.ws) {
    float* w = g.ws + (int64_t)tl.bz * g.M * g.N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = bm + wm * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
      if (m < g.M && n < g.N) w[(int64_t)m * g.N + n] = acc[r];
    }
    return;
  }
  float cs = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = bm + wm * 32 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
    if (m < g.M && n < g.N) {
      float v = acc[r];
      if (g.epi & kEpiBias) v += g.bias[n];
      if (g.epi & kEpiRelu) v = v > 0.0f ? v : 0.0f;
      if (g.epi & kEpiMask) v = bf16_pos(g.mask[(int64_t)m * g.ldm + n]) ? v : 0.0f;
      if (g.Cb)
        g.Cb[(int64_t)m * g.ldc + n] = to_bf16(v);
      else
        g.C[(int64_t)m * g.ldc + n] = v;
      cs += v;
    }
  }
  if (g.epi & kEpiColSum) {
    // lanes l and l + 32 hold the same column: add them, then the two waves
    // of a column half through LDS
    cs += __shfl_xor(cs, 32);
    if (lane < 32) colacc[wm][wn * 32 + lane] = cs;
    __syncthreads();
    const int c = threadIdx.x;
    if (c < kBN && bn + c < g.N) g.colpart[(int64_t)tl.by * g.N + bn + c] = colacc[0][c] + colacc[1][c];
  }
}

// C = A B (+ bias, ReLU, mask).  64 x 64 tiles, 4 waves of 32 x 32, K steps
// of 32 staged in LDS, v_mfma_f32_32x32x16_bf16; any strides.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kBM][kLDP];   // [m][k]
  __shared__ __align__(16) uint16_t Bs[kBN][kLDP];   // [n][k]
  __shared__ float colacc[2][kBN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const Tile tl = block_tile();
  const int bm = tl.by * kBM, bn = tl.bx * kBN;
  const bool a_k = g.sak == 1, b_k = g.sbk == 1;     // contiguous index of each operand
  const int kbeg = tl.bz * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  f32x16 acc = {};
  for (int k0 = kbeg; k0 < kend; k0 += kBK) {
    for (int e = tid; e < kBM * kBK; e += 256) {
      const int m = a_k ? e / kBK : e % kBM, k = a_k ? e % kBK : e / kBM;
      const int gm = bm + m, gk = k0 + k;
      As[m][k] = (gm < g.M && gk < kend) ? g.A[(int64_t)gm * g.sam + (int64_t)gk * g.sak] : 0;
    }
    for (int e = tid; e < kBN * kBK; e += 256) {
      const int n = b_k ? e / kBK : e % kBN, k = b_k ? e % kBK : e / kBN;
      const int gn = bn + n, gk = k0 + k;
      Bs[n][k] = (gn < g.N && gk < kend) ? g.B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn] : 0;
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
  gemm_epilogue(g, acc, tl, wm, wn, lane, colacc);
}

// Eight consecutive bfloat16 elements p[0..7] of an operand along its
// contiguous index, which starts at c; elements at or beyond lim read as 0.
__device__ __forceinline__ uint4 load8(const uint16_t* p, int c, int lim) {
  if (c + 7 < lim) return *reinterpret_cast<const uint4*>(p);
  uint16_t e[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) e[i] = c + i < lim ? p[i] : 0;
  return make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                    e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
}

__device__ __forceinline__ uint32_t half_of(const uint4& v, int i) {
  const uint32_t w = i < 2 ? v.x : i < 4 ? v.y : i < 6 ? v.z : v.w;
  return (i & 1) ? w >> 16 : w & 0xFFFFu;
}

// One 64 x 64 bfloat16 tile of an operand as two 16-byte loads per thread.
// KC: the operand is contiguous along k (rows r of the tile are its m or n
// index): each load takes 8 k of one row.  Otherwise it is contiguous along
// m / n: the thread loads 8 rows at k and at k + 1, so that it can store
// both k of one row at once.
template <bool KC>
__device__ __forceinline__ void tile_load(const uint16_t* __restrict__ P, int64_t s_r,
                                          int64_t s_k, int r0, int rlim, int k0, int klim,
                                          uint4* v) {
  const int tid = threadIdx.x;
  if constexpr (KC) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int idx = tid + 256 * j;
      const int r = idx >> 3, k = (idx & 7) << 3;
      const int gr = r0 + r, gk = k0 + k;
      v[j] = gr < rlim ? load8(P + (int64_t)gr * s_r + gk, gk, klim) : make_uint4(0, 0, 0, 0);
    }
  } else {
    const int k = (tid >> 3) << 1, r = (tid & 7) << 3;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gk = k0 + k + j, gr = r0 + r;
      v[j] = gk < klim ? load8(P + (int64_t)gk * s_k + gr, gr, rlim) : make_uint4(0, 0, 0, 0);
    }
  }
}

// Column of element k of tile row `row` in LDS.  A tile stored by the
// transposing path below (8 rows of one thread, a word each, rows 8 apart
// across lanes) has the 16-byte chunks of each row (8 k each) permuted by
// XOR with bits 3..5 of the row, so that those stores spread over all banks
// instead of hitting 4 of them; a tile stored row-contiguous keeps the plain
// layout, whose 16-byte stores and MFMA operand reads are conflict-free.
template <bool KC>
__device__ __forceinline__ int tile_col(int row, int k) {
  if constexpr (KC) return k;
  return (((k >> 3) ^ ((row >> 3) & 7)) << 3) | (k & 7);
}

// Stores the tile into LDS columns k0 .. k0+63, laid out [row][tile_col(k)].
template <bool KC, int TP>
__device__ __forceinline__ void tile_store(uint16_t (*L)[TP], int k0, const uint4* v) {
  const int tid = threadIdx.x;
  if constexpr (KC) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int idx = tid + 256 * j;
      const int row = idx >> 3;
      *reinterpret_cast<uint4*>(&L[row][tile_col<KC>(row, k0 + ((idx & 7) << 3))]) = v[j];
    }
  } else {
    const int k = (tid >> 3) << 1, r = (tid & 7) << 3;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      *reinterpret_cast<uint32_t*>(&L[r + i][tile_col<KC>(r + i, k0 + k)]) =
          half_of(v[0], i) | (half_of(v[1], i) << 16);
  }
}

// C = A B (+ bias, ReLU, mask, column sums) with 16-byte bfloat16 operand
// loads.  A K step covers R sub-tiles of 64 (R kTK columns of A and rows of B in LDS),
// and the next step's operands are loaded into registers while the current
// one is multiplied: the fewer, deeper steps leave fewer waits on a load.
// AK / BK: A / B contiguous along k (else along m / n).  gridDim.z splits K
// into ranges of g.kchunk (partials mode, g.ws).
template <bool AK, bool BK, int R>
__global__ __launch_bounds__(256) void k_gemm_v(GemmArgs g) {
  constexpr int TK = kTK * R, TP = TK + 8;
  __shared__ __align__(16) uint16_t As[kTM][TP];
  __shared__ __align__(16) uint16_t Bs[kTN][TP];
  __shared__ float colacc[2][kBN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const Tile tl = block_tile();
  const int bm = tl.by * kTM, bn = tl.bx * kTN;
  const int kbeg = tl.bz * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int64_t a_r = AK ? g.sam : 0, a_k = AK ? 0 : g.sak;
  const int64_t b_r = BK ? g.sbn : 0, b_k = BK ? 0 : g.sbk;
  uint4 ra[R][2], rb[R][2];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    tile_load<AK>(g.A, a_r, a_k, bm, g.M, kbeg + kTK * q, kend, ra[q]);
    tile_load<BK>(g.B, b_r, b_k, bn, g.N, kbeg + kTK * q, kend, rb[q]);
  }
  f32x16 acc = {};
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      tile_store<AK, TP>(As, kTK * q, ra[q]);
      tile_store<BK, TP>(Bs, kTK * q, rb[q]);
    }
    __syncthreads();
    if (k0 + TK < kend) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        tile_load<AK>(g.A, a_r, a_k, bm, g.M, k0 + TK + kTK * q, kend, ra[q]);
        tile_load<BK>(g.B, b_r, b_k, bn, g.N, k0 + TK + kTK * q, kend, rb[q]);
      }
    }
    // sub-tiles past the end of the range hold zeros
    const int steps = kend - k0;
#pragma unroll
    for (int s = 0; s < TK; s += 16) {
      if (s < steps) {
        const int kk = s + (lane >> 5) * 8;
        const int ra = wm * 32 + (lane & 31), rb = wn * 32 + (lane & 31);
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[ra][tile_col<AK>(ra, kk)]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[rb][tile_col<BK>(rb, kk)]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  gemm_epilogue(g, acc, tl, wm, wn, lane, colacc);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// C = A B with the epilogue `epi` (bias, mask, column sums to colpart), or,
// with ws (partials mode), the products of *splits K ranges into ws (no
// epilogue; the caller sums them in split order).  Deep K steps where K is
// long; split K where the tiles alone would not fill the chip.
hipError_t gemm(hipStream_t s, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
                int64_t sbk, int64_t sbn, float* C, uint16_t* Cb, int64_t ldc, int M, int N,
                int K, int epi, const float* bias = nullptr, const uint16_t* mask = nullptr,
                int64_t ldm = 0, float* ws = nullptr, int* splits = nullptr,
                float* colpart = nullptr) {
  GemmArgs g{A, sam, sak, B, sbk, sbn, C, Cb, ldc, M, N, K, bias, mask, ldm, epi, ws, K, colpart};
  const bool ak = sak == 1, bk = sbk == 1;
  const bool a_ok = ak ? (sam % 8 == 0) : (sam == 1 && sak % 8 == 0);
  const bool b_ok = bk ? (sbn % 8 == 0) : (sbn == 1 && sbk % 8 == 0);
  const bool vec = a_ok && b_ok && aligned16(A) && aligned16(B);
  const int tiles = ((N + kTN - 1) / kTN) * ((M + kTM - 1) / kTM);
  int S = 1;
  if (ws && tiles < 256) {
    // enough splits to fill the chip, each still at least 256 deep in K
    S = std::min(kMaxSplit, std::max(1, 512 / tiles));
    while (S > 1 && K / S < 256) --S;
  }
  // K step: two sub-tiles of 64 where a split has at least 128 of K (four
  // measured slower: their LDS leaves room for fewer blocks per CU)
  const int R = vec && (K + S - 1) / S >= 128 ? 2 : 1;
  const int step = vec ? kTK * R : kBK;
  g.kchunk = ((K + S - 1) / S + step - 1) / step * step;
  S = (K + g.kchunk - 1) / g.kchunk;
  if (splits) *splits = S;
  const dim3 grid((unsigned)((N + kTN - 1) / kTN), (unsigned)((M + kTM - 1) / kTM), (unsigned)S);
  if (!vec) {
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
    return hipGetLastError();
  }
#define FSNE_GEMM_V(AKv, BKv)                                                        \
  do {                                                                               \
    if (R == 2)                                                                      \
      hipLaunchKernelGGL((k_gemm_v<AKv, BKv, 2>), grid, dim3(256), 0, s, g);         \
    else                                                                             \
      hipLaunchKernelGGL((k_gemm_v<AKv, BKv, 1>), grid, dim3(256), 0, s, g);         \
  } while (0)
  if (ak && bk)
    FSNE_GEMM_V(true, true);
  else if (ak && !bk)
    FSNE_GEMM_V(true, false);
  else if (!ak && bk)
    FSNE_GEMM_V(false, true);
  else
    FSNE_GEMM_V(false, false);
#undef FSNE_GEMM_V
  return hipGetLastError();
}

// Batch rows: row k is source row (off + k) mod N of X (FP32 or BF16 bits),
// rounded to bfloat16 into Xb (skipped when Xb is null: the rows are read in
// place); targets (y - mean) / std from Y (padded stride DP).  One block per
// row at a time.
__global__ void k_gather(const void* X, int xdtype, int D, int64_t N, int64_t off, int n,
                         const float* Y, int DP, int d, const float* mean, const float* sd,
                         uint16_t* Xb, float* Tb) {
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const int64_t r = (off + k) % N;
    if (Xb) {
      uint16_t* dst = Xb + (int64_t)k * D;
      if (xdtype == 0 && (D & 3) == 0) {
        const float4* src = reinterpret_cast<const float4*>(static_cast<const float*>(X) + r * D);
        for (int c = threadIdx.x; c < (D >> 2); c += blockDim.x) {
          const float4 v = src[c];
          reinterpret_cast<uint2*>(dst)[c] =
              make_uint2(to_bf16(v.x) | ((uint32_t)to_bf16(v.y) << 16),
                         to_bf16(v.z) | ((uint32_t)to_bf16(v.w) << 16));
        }
      } else if (xdtype == 0) {
        const float* src = static_cast<const float*>(X) + r * D;
        for (int c = threadIdx.x; c < D; c += blockDim.x) dst[c] = to_bf16(src[c]);
      } else {
        const uint16_t* src = static_cast<const uint16_t*>(X) + r * D;
        for (int c = threadIdx.x; c < D; c += blockDim.x) dst[c] = src[c];
      }
    }
    if (Y && (int)threadIdx.x < d) {
      const int c = threadIdx.x;
      Tb[(int64_t)k * d + c] = (Y[r * DP + c] - mean[c]) / sd[c];
    }
  }
}

// dst[k] = src[k] rounded to bfloat16, k < n.
__global__ void k_to_bf16(const float* src, uint16_t* dst, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = to_bf16(src[k]);
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

// dH2[r][k] = (sum_j dO[r][j] W3[j][k]) where H2[r][k] > 0, else 0 (and
// its bfloat16 rounding, the operand of the products that follow).
__global__ void k_back_out(const float* dO, const float* W3, const float* H2, int n, int H, int d,
                           float* dH2, uint16_t* dH2b) {
  const int64_t total = (int64_t)n * H;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q / H, k = q % H;
    float s = 0.0f;
    for (int j = 0; j < d; ++j) s = fmaf(dO[r * d + j], W3[(int64_t)j * H + k], s);
    const float v = H2[q] > 0.0f ? s : 0.0f;
    dH2[q] = v;
    dH2b[q] = to_bf16(v);
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

// The output layer and the loss gradient of one chunk of kRowChunk rows per
// block, in one pass over H2 (S = columns per thread / 256, H <= 256 S):
//   O[r][j] = b3[j] + sum_k H2[r][k] W3[j][k],  e = O - T,  dO = 2 e scale,
//   dH2[r][k] = (sum_j dO[r][j] W3[j][k]) where H2[r][k] > 0, else 0
//               (stored rounded to bfloat16: it is only a product operand),
// and the chunk's partial sums, each over its rows in order:
//   part2[c][k] = sum_r dH2[r][k]                      (b2 gradient)
//   part3[c][j (H+1) + k] = sum_r dO[r][j] H2[r][k]    (W3 gradient)
//   part3[c][j (H+1) + H] = sum_r dO[r][j]             (b3 gradient)
//   lchunk[c] = sum over the chunk of e^2.
// red needs kRowChunk d (4 + 2) floats of shared memory.
// The targets of row r: T[r] (tgt.Y null) or, while training on a context,
// (y - mean) / std of its point (off + r) mod N.
struct Targets {
  const float* T;
  const float* Y;
  int64_t N, off;
  int DP;
  const float *mean, *sd;
  __device__ float operator()(int r, int j, int d) const {
    if (!Y) return T[(int64_t)r * d + j];
    const int64_t p = (off + r) % N;
    return (Y[p * DP + j] - mean[j]) / sd[j];
  }
};

template <int S>
__global__ __launch_bounds__(256) void k_head(const float* H2, const float* W3, const float* b3,
                                              Targets tgt, int n, int H, int d, float scale,
                                              uint16_t* dH2, float* part2, float* part3,
                                              float* lchunk) {
  extern __shared__ float red[];            // [4 waves][rows d], then dO, then e^2
  float* sdo = red + 4 * kRowChunk * d;
  float* se2 = sdo + kRowChunk * d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = blockIdx.x, r0 = c * kRowChunk;
  const int rows = min(kRowChunk, n - r0);
  float h[kRowChunk][S];
#pragma unroll
  for (int r = 0; r < kRowChunk; ++r)
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int k = tid + 256 * q;
      h[r][q] = (r < rows && k < H) ? H2[(int64_t)(r0 + r) * H + k] : 0.0f;
    }
  // O: per output j, every row's partial dot product, summed over the wave
  // and then over the four waves
  for (int j = 0; j < d; ++j) {
    float w[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int k = tid + 256 * q;
      w[q] = k < H ? W3[(int64_t)j * H + k] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < kRowChunk; ++r) {
      float p = 0.0f;
#pragma unroll
      for (int q = 0; q < S; ++q) p = fmaf(h[r][q], w[q], p);
      p = wave_sum_uniform(p);
      if (lane == 0) red[(wave * kRowChunk + r) * d + j] = p;
    }
  }
  __syncthreads();
  for (int q = tid; q < kRowChunk * d; q += 256) {
    const int r = q / d, j = q - r * d;
    float dov = 0.0f, e2 = 0.0f;
    if (r < rows) {
      const float o = ((red[q] + red[kRowChunk * d + q]) + (red[2 * kRowChunk * d + q] +
                       red[3 * kRowChunk * d + q])) + b3[j];
      const float e = o - tgt(r0 + r, j, d);
      dov = 2.0f * e * scale;
      e2 = e * e;
    }
    sdo[q] = dov;
    se2[q] = e2;
  }
  __syncthreads();
  // dH2 rows and the partial sums of this chunk
  float dh[kRowChunk][S];
#pragma unroll
  for (int r = 0; r < kRowChunk; ++r)
#pragma unroll
    for (int q = 0; q < S; ++q) dh[r][q] = 0.0f;
  for (int j = 0; j < d; ++j) {
    float w[S], g3[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int k = tid + 256 * q;
      w[q] = k < H ? W3[(int64_t)j * H + k] : 0.0f;
      g3[q] = 0.0f;
    }
#pragma unroll
    for (int r = 0; r < kRowChunk; ++r) {
      const float dv = sdo[r * d + j];
#pragma unroll
      for (int q = 0; q < S; ++q) {
        dh[r][q] = fmaf(dv, w[q], dh[r][q]);
        g3[q] = fmaf(dv, h[r][q], g3[q]);
      }
    }
    float* p3 = part3 + (int64_t)c * d * (H + 1) + (int64_t)j * (H + 1);
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int k = tid + 256 * q;
      if (k < H) p3[k] = g3[q];
    }
    if (tid == 0) {
      float sb = 0.0f;
      for (int r = 0; r < kRowChunk; ++r) sb += sdo[r * d + j];
      p3[H] = sb;
    }
  }
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int k = tid + 256 * q;
    float cs = 0.0f;
#pragma unroll
    for (int r = 0; r < kRowChunk; ++r) {
      const float v = h[r][q] > 0.0f ? dh[r][q] : 0.0f;
      if (r < rows && k < H) dH2[(int64_t)(r0 + r) * H + k] = to_bf16(v);
      cs += v;
    }
    if (k < H) part2[(int64_t)c * H + k] = cs;
  }
  if (tid == 0) {
    float l = 0.0f;
    for (int q = 0; q < kRowChunk * d; ++q) l += se2[q];
    lchunk[c] = l;
  }
}

// Gradient assembly and the optimiser step, one launch.  Blocks below nbd:
// one thread per W1 / W2 entry, the sum of its split-K partials in split
// order.  The rest: one wave per b1, b2, W3, b3 entry (and one for the loss),
// the sum of its row-block partials (lanes take blocks l, l + 64, ..., then
// a fixed tree).  Every gradient goes to G; with adam the parameters take
// their Adam step (Kingma and Ba 2015; c1 = 1 - b1^t, c2 = 1 - b2^t), and the
// new W1 and W2 are rounded to bfloat16 for the next products.
struct FinishArgs {
  float *P, *M, *V, *G;
  uint16_t *W1b, *W2b;             // with adam: the stepped W1, W2 rounded to bfloat16
  int H1, D, H2, d;
  const float* ws1; int S1;        // W1 partials: [S1][H1 D]
  const float* ws2; int S2;        // W2 partials: [S2][H2 H1]
  const float* colpart; int nb1;   // b1 partials: [nb1][H1]
  const float* part2; const float* part3; int nchunk;   // b2: [nchunk][H2]; W3, b3: [nchunk][d (H2+1)]
  const float* lchunk; float* lpart; int accumulate;    // loss (lchunk may be null)
  int nbd;
  int adam; float lr, b1, b2, eps, c1, c2;
};

__device__ __forceinline__ float adam_step(const FinishArgs& f, int64_t k, float gk) {
  f.G[k] = gk;
  if (!f.adam) return 0.0f;
  const float mk = f.b1 * f.M[k] + (1.0f - f.b1) * gk;
  const float vk = f.b2 * f.V[k] + (1.0f - f.b2) * gk * gk;
  f.M[k] = mk;
  f.V[k] = vk;
  const float p = f.P[k] - f.lr * (mk / f.c1) / (sqrtf(vk / f.c2) + f.eps);
  f.P[k] = p;
  return p;
}

__global__ __launch_bounds__(256) void k_finish(FinishArgs f) {
  const int64_t nw1 = (int64_t)f.H1 * f.D, nw2 = (int64_t)f.H2 * f.H1;
  const int64_t o_b1 = nw1, o_w2 = o_b1 + f.H1, o_b2 = o_w2 + nw2, o_w3 = o_b2 + f.H2;
  const int64_t o_b3 = o_w3 + (int64_t)f.d * f.H2;
  if ((int)blockIdx.x < f.nbd) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nw1 + nw2;
         q += (int64_t)f.nbd * 256) {
      float g = 0.0f;
      if (q < nw1) {
        for (int z = 0; z < f.S1; ++z) g += f.ws1[(int64_t)z * nw1 + q];
        const float p = adam_step(f, q, g);
        if (f.adam) f.W1b[q] = to_bf16(p);
      } else {
        const int64_t q2 = q - nw1;
        for (int z = 0; z < f.S2; ++z) g += f.ws2[(int64_t)z * nw2 + q2];
        const float p = adam_step(f, o_w2 + q2, g);
        if (f.adam) f.W2b[q2] = to_bf16(p);
      }
    }
    return;
  }
  const int w = ((int)blockIdx.x - f.nbd) * 4 + (int)(threadIdx.x >> 6);
  const int n3 = f.d * (f.H2 + 1);
  if (w < f.H1) {
    const float g = sum_chunks(f.colpart, f.nb1, f.H1, w);
    if (lane_id() == 0) adam_step(f, o_b1 + w, g);
  } else if (w < f.H1 + f.H2) {
    const int k = w - f.H1;
    const float g = sum_chunks(f.part2, f.nchunk, f.H2, k);
    if (lane_id() == 0) adam_step(f, o_b2 + k, g);
  } else if (w < f.H1 + f.H2 + n3) {
    const int q = w - f.H1 - f.H2;
    const float g = sum_chunks(f.part3, f.nchunk, n3, q);
    const int j = q / (f.H2 + 1), k = q - j * (f.H2 + 1);
    if (lane_id() == 0) adam_step(f, k < f.H2 ? o_w3 + (int64_t)j * f.H2 + k : o_b3 + j, g);
  } else if (w == f.H1 + f.H2 + n3 && f.lchunk) {
    const float l = sum_chunks(f.lchunk, f.nchunk, 1, 0);
    if (lane_id() == 0) f.lpart[0] = (f.accumulate ? f.lpart[0] : 0.0f) + l;
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

// Forward of n batch rows (bfloat16, row stride D: Xb, or xin when given):
// H1b (bfloat16), H2b, and with out the network's output Ob (training takes
// the output inside the loss kernel).
fsne_status forward(fsne_mlp* m, int n, bool out = true, const uint16_t* xin = nullptr) {
  hipStream_t s = m->stream;
  const Views P = views(m, m->P);
  if (m->wdirty) {
    hipLaunchKernelGGL(k_to_bf16, dim3(1024), dim3(256), 0, s, P.W1, m->W1b,
                       (int64_t)m->H1 * m->D);
    hipLaunchKernelGGL(k_to_bf16, dim3(1024), dim3(256), 0, s, P.W2, m->W2b,
                       (int64_t)m->H2 * m->H1);
    MCHK(m, hipGetLastError());
    m->wdirty = false;
  }
  const uint16_t* X = xin ? xin : m->Xb;
  MCHK(m, gemm(s, X, m->D, 1, m->W1b, 1, m->D, nullptr, m->H1b, m->H1, n, m->H1, m->D,
               kEpiBias | kEpiRelu, P.b1));
  MCHK(m, gemm(s, m->H1b, m->H1, 1, m->W2b, 1, m->H1, m->H2b, nullptr, m->H2, n, m->H2, m->H1,
               kEpiBias | kEpiRelu, P.b2));
  if (out || !m->fused_head) {
    hipLaunchKernelGGL(k_out_layer, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, m->H2b, P.W3,
                       P.b3, n, m->H2, m->d, m->Ob);
    MCHK(m, hipGetLastError());
  }
  return FSNE_OK;
}

// Loss and gradient (into G) of n batch rows with targets in Tb, and with
// adam the Adam step; the loss of the batch is added to the running sum when
// accumulate is set.  Launches: the output layer and loss gradient (one
// kernel), the W2 gradient (split-K partials), dH1 with the b1 column sums,
// the W1 gradient (partials), and one kernel that sums every gradient and
// steps the parameters.
fsne_status backward(fsne_mlp* m, int n, int accumulate, bool adam_step_on,
                     const uint16_t* xin = nullptr, Targets tgt = Targets{}) {
  hipStream_t s = m->stream;
  const uint16_t* X = xin ? xin : m->Xb;
  const Views P = views(m, m->P);
  const int64_t cnt = (int64_t)n * m->d;
  const int nchunk = (n + kRowChunk - 1) / kRowChunk;
  if (m->fused_head) {
    const size_t shm = sizeof(float) * 6 * kRowChunk * m->d;
    const float sc = 1.0f / (float)cnt;
    if (!tgt.Y) tgt.T = m->Tb;
#define FSNE_HEAD(Sv)                                                                            \
  hipLaunchKernelGGL((k_head<Sv>), dim3((unsigned)nchunk), dim3(256), shm, s, m->H2b, P.W3, P.b3,  \
                     tgt, n, m->H2, m->d, sc, m->dH2b, m->part, m->part3, m->lchunk)
    if (m->H2 <= 256)
      FSNE_HEAD(1);
    else if (m->H2 <= 512)
      FSNE_HEAD(2);
    else
      FSNE_HEAD(4);
#undef FSNE_HEAD
    MCHK(m, hipGetLastError());
  } else {
    hipLaunchKernelGGL(k_dout, dim3(kLossBlocks), dim3(256), 0, s, m->Ob, m->Tb, cnt,
                       1.0f / (float)cnt, m->dOb, m->lpart, accumulate);
    MCHK(m, hipGetLastError());
    const int q = m->d * (m->H2 + 1);
    hipLaunchKernelGGL(k_grad_out_part, dim3((unsigned)((q + 255) / 256), (unsigned)nchunk),
                       dim3(256), 0, s, m->dOb, m->H2b, n, m->H2, m->d, m->part3);
    MCHK(m, hipGetLastError());
    hipLaunchKernelGGL(k_back_out, dim3(1024), dim3(256), 0, s, m->dOb, P.W3, m->H2b, n, m->H2,
                       m->d, m->dH2, m->dH2b);
    MCHK(m, hipGetLastError());
    hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((m->H2 + 255) / 256), (unsigned)nchunk),
                       dim3(256), 0, s, m->dH2, n, m->H2, m->part);
    MCHK(m, hipGetLastError());
  }
  // W2 gradient dH2^T H1 as split-K partials
  int S2 = 1, S1 = 1;
  MCHK(m, gemm(s, m->dH2b, 1, m->H2, m->H1b, m->H1, 1, nullptr, nullptr, m->H1, m->H2, m->H1,
               n, 0, nullptr, nullptr, 0, m->ws2, &S2));
  // dH1 = (dH2 W2) where H1 > 0, with its column sums per 64-row block (b1)
  MCHK(m, gemm(s, m->dH2b, m->H2, 1, m->W2b, m->H1, 1, nullptr, m->dH1b, m->H1, n, m->H1, m->H2,
               kEpiMask | kEpiColSum, nullptr, m->H1b, m->H1, nullptr, nullptr, m->colpart));
  // W1 gradient dH1^T X as split-K partials
  MCHK(m, gemm(s, m->dH1b, 1, m->H1, X, m->D, 1, nullptr, nullptr, m->D, m->H1, m->D, n, 0,
               nullptr, nullptr, 0, m->ws, &S1));
  FinishArgs f{};
  f.P = m->P;
  f.W1b = m->W1b;
  f.W2b = m->W2b;
  f.M = m->Mo;
  f.V = m->Vo;
  f.G = m->G;
  f.H1 = m->H1;
  f.D = m->D;
  f.H2 = m->H2;
  f.d = m->d;
  f.ws1 = m->ws;
  f.S1 = S1;
  f.ws2 = m->ws2;
  f.S2 = S2;
  f.colpart = m->colpart;
  f.nb1 = (n + kTM - 1) / kTM;
  f.part2 = m->part;
  f.part3 = m->part3;
  f.nchunk = nchunk;
  f.lchunk = m->fused_head ? m->lchunk : nullptr;
  f.lpart = m->lpart;
  f.accumulate = accumulate;
  f.nbd = 1024;
  f.adam = adam_step_on ? 1 : 0;
  if (adam_step_on) {
    m->t += 1;
    const fsne_mlp_opts& o = m->opts;
    f.lr = o.lr;
    f.b1 = o.beta1;
    f.b2 = o.beta2;
    f.eps = o.eps;
    f.c1 = 1.0f - powf(o.beta1, (float)m->t);
    f.c2 = 1.0f - powf(o.beta2, (float)m->t);
  }
  const int waves = m->H1 + m->H2 + m->d * (m->H2 + 1) + 1;
  hipLaunchKernelGGL(k_finish, dim3((unsigned)(f.nbd + (waves + 3) / 4)), dim3(256), 0, s, f);
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

// Adam steps over opts.epochs passes of batches (rows: the context's points
// as bfloat16, or null: gathered per batch).
fsne_status train_epochs(fsne_mlp* m, fsne_ctx* ctx, const uint16_t* rows, int64_t N, int64_t B,
                         int64_t nb) {
  for (int e = 0; e < m->opts.epochs; ++e) {
    const int64_t off = ((int64_t)e * 104729) % N;
    const int last = e == m->opts.epochs - 1;
    for (int64_t b = 0; b < nb; ++b) {
      const int n = (int)std::min<int64_t>(B, N - b * B);
      const int64_t row0 = (off + b * B) % N;
      // bfloat16 rows of a batch that does not wrap around are read in place
      const uint16_t* xin = rows && row0 + n <= N ? rows + row0 * m->D : nullptr;
      // with the fused loss kernel the targets are read there from Y
      Targets tgt{};
      if (m->fused_head) tgt = Targets{nullptr, ctx->Y, N, off + b * B, ctx->DP, m->ymean, m->ystd};
      if (!xin || !m->fused_head) {
        hipLaunchKernelGGL(k_gather, dim3(1024), dim3(256), 0, m->stream, ctx->X, ctx->xdtype,
                           m->D, N, off + b * B, n, ctx->Y, ctx->DP, m->d, m->ymean, m->ystd,
                           xin ? nullptr : m->Xb, m->Tb);
        MCHK(m, hipGetLastError());
      }
      MTRY(forward(m, n, false, xin));
      MTRY(backward(m, n, last, true, xin, tgt));
    }
  }
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
  const size_t nchunk_max = (B + kRowChunk - 1) / kRowChunk;
  // the output layer goes into one kernel while H2 fits four columns a thread
  m->fused_head = m->H2 <= 1024 && m->d <= 64;
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
      (st = malloc_dev(m, &m->dH1b, B * m->H1)) || (st = malloc_dev(m, &m->dH2b, B * m->H2)) ||
      (st = malloc_dev(m, &m->W1b, (size_t)m->H1 * m->D)) ||
      (st = malloc_dev(m, &m->W2b, (size_t)m->H2 * m->H1)) ||
      (st = malloc_dev(m, &m->Ob, B * m->d)) || (st = malloc_dev(m, &m->dOb, B * m->d)) ||
      (st = malloc_dev(m, &m->dH2, B * m->H2)) ||
      (st = malloc_dev(m, &m->lpart, kLossBlocks)) ||
      (st = malloc_dev(m, &m->ws, (size_t)kMaxSplit * m->H1 * m->D)) ||
      (st = malloc_dev(m, &m->ws2, (size_t)kMaxSplit * m->H2 * m->H1)) ||
      (st = malloc_dev(m, &m->part, nchunk_max * m->H2)) ||
      (st = malloc_dev(m, &m->part3, nchunk_max * m->d * (m->H2 + 1))) ||
      (st = malloc_dev(m, &m->colpart, ((B + kTM - 1) / kTM) * m->H1)) ||
      (st = malloc_dev(m, &m->lchunk, nchunk_max)) ||
      (st = malloc_dev(m, reinterpret_cast<uint8_t**>(&m->xstage), B * m->D * 4)))
    return bad(st);
  if (hipMemsetAsync(m->Mo, 0, sizeof(float) * m->np, m->stream) != hipSuccess ||
      hipMemsetAsync(m->Vo, 0, sizeof(float) * m->np, m->stream) != hipSuccess ||
      hipMemsetAsync(m->lpart, 0, sizeof(float) * kLossBlocks, m->stream) != hipSuccess)
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
  // The product operands are bfloat16: BF16 rows are read in place, FP32
  // rows are rounded once into a copy held for this call (every epoch reads
  // each row twice), or, if that copy cannot be allocated, per batch.
  const uint16_t* rows = nullptr;
  uint16_t* copy = nullptr;
  if ((m->D & 7) == 0) {
    if (ctx->xdtype == FSNE_BF16) {
      rows = static_cast<const uint16_t*>(ctx->X);
    } else if (m->opts.epochs > 1 &&
               hipMalloc(reinterpret_cast<void**>(&copy), sizeof(uint16_t) * N * m->D) == hipSuccess) {
      hipLaunchKernelGGL(k_to_bf16, dim3(4096), dim3(256), 0, m->stream,
                         static_cast<const float*>(ctx->X), copy, N * m->D);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        (void)hipFree(copy);
        return mfail(m, FSNE_EHIP, std::string("k_to_bf16: ") + hipGetErrorString(e));
      }
      rows = copy;
    } else {
      (void)hipGetLastError();   // a failed allocation leaves its error behind
    }
  }
  const fsne_status st = train_epochs(m, ctx, rows, N, B, nb);
  if (copy) {
    (void)hipStreamSynchronize(m->stream);
    (void)hipFree(copy);
  }
  MTRY(st);
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
  if (params) {
    MCHK(m, hipMemcpyAsync(m->P, params, sizeof(float) * m->np, hipMemcpyHostToDevice, m->stream));
    m->wdirty = true;
  }
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
  MTRY(forward(m, (int)n, false));
  MTRY(backward(m, (int)n, 0, false));
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
  MTRY(forward(m, (int)n, false));
  MTRY(backward(m, (int)n, 0, true));
  MCHK(m, hipStreamSynchronize(m->stream));
  return FSNE_OK;
}

void fsne_mlp_destroy(fsne_mlp* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  void* bufs[] = {m->P, m->G, m->Mo, m->Vo, m->ymean, m->ystd, m->Xb, m->Tb, m->H1b, m->H2b,
                  m->Ob, m->dOb, m->dH1b, m->dH2, m->dH2b, m->W1b, m->W2b, m->lpart, m->ws,
                  m->ws2, m->part, m->part3, m->colpart, m->lchunk, m->xstage};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

const char* fsne_mlp_last_error(const fsne_mlp* m) { return m ? m->err.c_str() : "null network"; }

}  // extern "C"
