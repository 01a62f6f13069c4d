// Device-side building blocks of the FUnc-SNE step for gfx950 (wave64).
//
// Everything here runs inside one wavefront that owns one point: lanes hold
// list entries or candidates, cross-lane traffic goes through readlane,
// ds_bpermute shuffles and a per-wave LDS scratch area.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsne {

constexpr int kWave = 64;
constexpr int kCand = 32;          // candidate slots per point and refinement
constexpr int kSameNoN = 16;       // slots  0..15: neighbour of neighbour, own space
constexpr int kCrossDir = 20;      // slots 16..19: neighbour in the other space
constexpr int kCrossNoN = 28;      // slots 20..27: neighbour of neighbour, other space
                                   // slots 28..31: uniform random point
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kReduceBlocks = 1024; // partial sums of the Z / N_new reduction

// Third word of the Philox counter: which draw stream.
enum : uint32_t {
  kStreamHDC = 1, kStreamLDC = 2, kStreamNeg = 3, kStreamInitHD = 4, kStreamInitLD = 5,
  kStreamCoin = 7
};

// Scalars of the iteration, resident in device memory so that a whole
// iteration (and a captured graph of many) needs no host round trip.
struct Scalars {
  uint32_t t;          // iteration counter
  float E;             // smoothed fraction of points that gained HD neighbours
  int32_t fire;        // whether iteration t refines the HD lists
  int32_t hd_cur;      // which of the two HD buffers holds the lists of iteration t
  int32_t n_new;       // points whose HD list changed in the last refinement
  float Z;             // normaliser of the last iteration
  int32_t nonfinite;   // set when a NaN/inf reached the embedding
  int32_t last_fired;  // whether iteration t-1 refined the HD lists
};

// Hyperparameters in the form the kernels use.
struct Hyper {
  float alpha, inv_alpha, lr, momentum, attr, rep;
  float perplexity, ln_perp, e_smooth, p_min, margin;
  int32_t n_neg, hd_mode, dist_mode;
  uint32_t key0, key1;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of two 32x32->64-bit
// multiplies mixing the four counter words, the two key words advanced by
// the Weyl increments between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return make_uint4(c0, c1, c2, c3);
}

// floor(u * K / 2^32): index in [0, K).
__device__ __forceinline__ uint32_t draw_index(uint32_t u, uint32_t K) { return __umulhi(u, K); }

// A uniform point of {0..N-1} other than i.
__device__ __forceinline__ int32_t draw_other(uint32_t u, int32_t i, int32_t N) {
  const int32_t j = (int32_t)__umulhi(u, (uint32_t)(N - 1));
  return j + (j >= i ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Single-precision decisions that must match the stated operation sequence
// exactly (no contraction to FMA).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int coin_fires(float E, uint32_t t, const Hyper& h) {
#pragma clang fp contract(off)
  if (h.hd_mode == 1) return 1;
  if (h.hd_mode == 2) return 0;
  const float one_minus = 1.0f - h.p_min;
  const float prod = one_minus * E;
  const float p = h.p_min + prod;
  if (!(p < 1.0f)) return 1;
  if (!(p > 0.0f)) return 0;
  const uint32_t thr = (uint32_t)(p * 4294967296.0f);
  const uint4 u = philox(0xFFFFFFFFu, t, kStreamCoin, 0u, h.key0, h.key1);
  return u.x < thr ? 1 : 0;
}

__device__ __forceinline__ float E_next(float E, int32_t n_new, int32_t N, float lam) {
#pragma clang fp contract(off)
  const float frac = (float)n_new / (float)N;
  const float a = (1.0f - lam) * E;
  const float b = lam * frac;
  return a + b;
}

// ---------------------------------------------------------------------------
// Wave utilities.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float readlane_f(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Wave sum broadcast from lane 0.  Partner lanes of the butterfly can round
// differently once the compiler fuses a product into its first add, so a
// value that steers control flow is taken from one lane: every lane then
// branches alike and no lane drops out of a later cross-lane operation.
__device__ __forceinline__ float wave_sum_uniform(float v) {
  v = wave_sum(v);
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ int popc_below(uint64_t mask, int lane) {
  return __popcll(mask & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ bool key_less(float da, int ia, float db, int ib) {
  return da < db || (da == db && ia < ib);
}

// Rank of each lane's two entries (A: slot lane, B: slot 64+lane) among the
// nA + nB entries of the wave, ordered by (distance, index).  Invalid
// entries carry (+inf, INT_MAX) and rank after every valid one.
__device__ __forceinline__ void rank_two(float ka, int ia, float kb, int ib, int nA, int nB,
                                         float* skey, int* sid, int& ra, int& rb) {
  const int lane = lane_id();
  skey[lane] = ka;
  sid[lane] = ia;
  skey[kWave + lane] = kb;
  sid[kWave + lane] = ib;
  wave_lds_sync();
  int a = 0, b = 0;
  for (int k = 0; k < nA; ++k) {
    const float kk = skey[k];
    const int ii = sid[k];
    a += key_less(kk, ii, ka, ia);
    b += key_less(kk, ii, kb, ib);
  }
  for (int k = 0; k < nB; ++k) {
    const float kk = skey[kWave + k];
    const int ii = sid[kWave + k];
    a += key_less(kk, ii, ka, ia);
    b += key_less(kk, ii, kb, ib);
  }
  ra = a;
  rb = b;
  wave_lds_sync();
}

// True if v equals the value some lane k < n holds in x (n wave-uniform).
__device__ __forceinline__ bool in_lanes(int v, int x, int n) {
  bool hit = false;
  for (int k = 0; k < n; ++k) hit |= (v == __builtin_amdgcn_readlane(x, k));
  return hit;
}

// ---------------------------------------------------------------------------
// Perplexity calibration of one sorted HD row held one distance per lane
// (lanes < K).  Solves H(beta) = ln(perplexity) with
//   H = ln S + beta T / S,  S = sum e_k,  T = sum e_k D_k,  e_k = exp(-beta D_k),
// D_k = d2_k - m.  H falls strictly in beta, so the root is unique; Newton
// steps from the previous beta (warm restart), kept inside a bisection
// bracket, converge in a few iterations.  Returns {beta, m, r, invS}.
// ---------------------------------------------------------------------------
__device__ inline float4 calibrate_row(float d2, int K, const Hyper& h, float beta_prev) {
  const int lane = lane_id();
  const bool act = lane < K;
  const float m = readlane_f(d2, 0);
  const float r = readlane_f(d2, K - 1);
  const float D = act ? d2 - m : 0.0f;
  if (!(r > m)) return make_float4(0.0f, m, r, 1.0f / (float)K);
  const int ties = __popcll(__ballot(act && D == 0.0f));
  if ((float)ties >= h.perplexity) return make_float4(1e30f, m, r, 1.0f / (float)ties);

  const float target = h.ln_perp;
  float beta = readlane_f(beta_prev, 0);
  if (!(beta > 0.0f && beta < 1e29f)) beta = (float)K / wave_sum_uniform(D);
  float lo = 0.0f, hi = __int_as_float(0x7f800000);
  for (int it = 0; it < 48; ++it) {
    const float e = act ? expf(-beta * D) : 0.0f;
    const float S = wave_sum_uniform(e);
    const float T = wave_sum_uniform(e * D);
    const float U = wave_sum_uniform(e * D * D);
    const float mean = T / S;
    const float f = logf(S) + beta * mean - target;
    if (fabsf(f) <= 1e-6f) break;
    if (f > 0.0f)
      lo = beta;
    else
      hi = beta;
    if (hi < 3e38f && hi - lo <= 2e-7f * hi) break;
    const float var = U / S - mean * mean;
    float bn = beta + f / (beta * var);
    if (!(bn > lo && bn < hi)) bn = (hi < 3e38f) ? 0.5f * (lo + hi) : 2.0f * beta;
    beta = bn;
  }
  const float S = wave_sum_uniform(act ? expf(-beta * D) : 0.0f);
  return make_float4(beta, m, r, 1.0f / S);
}

}  // namespace fsne
