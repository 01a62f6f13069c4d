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
  kStreamCoin = 7, kStreamDelHD = 10, kStreamDelLD = 11, kStreamOrder = 12
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
  uint32_t hd_cand;    // distinct HD candidate rows loaded in the last iteration
  uint32_t ld_cand;    // distinct LD candidate rows loaded in the last iteration
  uint32_t refinements;  // iterations that refined the HD lists since init
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
    // each 32 x 32 -> 64-bit product in one multiply (v_mad_u64_u32) rather
    // than separate low and high halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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

// DPP moves (row = 16 lanes).  Lanes outside row_mask keep 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
constexpr int kDppSwap1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7-i within 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15-i within a row
constexpr int kDppBcast15 = 0x142;     // lane 15 of row r -> row r+1
constexpr int kDppBcast31 = 0x143;     // lane 31 -> rows 2, 3

// Sum over aligned groups of g lanes (g = 1, 2, ..., 64; g wave-uniform).
// For g <= 16 every lane of the group gets the sum; for g = 32 and 64 the
// last lane of the group holds it.  The sequence of additions depends only
// on lane positions.
__device__ __forceinline__ float group_sum_dpp(float v, int g) {
  if (g >= 2) v += dpp<kDppSwap1>(v);
  if (g >= 4) v += dpp<kDppSwap2>(v);
  if (g >= 8) v += dpp<kDppHalfMirror>(v);
  if (g >= 16) v += dpp<kDppMirror>(v);
  if (g >= 32) v += dpp<kDppBcast15, 0xA>(v);
  if (g >= 64) v += dpp<kDppBcast31, 0xC>(v);
  return v;
}

// A stored element as FP32 (BF16 bit patterns widened exactly).
__device__ __forceinline__ float to_unit_f32(float v) { return v; }
__device__ __forceinline__ float to_unit_f32(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}

// Wave sum, the same value in every lane (taken from lane 63 with readlane,
// so it is wave-uniform: control flow that depends on it cannot diverge and
// no lane drops out of a later cross-lane operation).
__device__ __forceinline__ float wave_sum_uniform(float v) {
  v = group_sum_dpp(v, kWave);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

__device__ __forceinline__ float wave_sum(float v) { return wave_sum_uniform(v); }

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
                                         int2* skey, int& ra, int& rb) {
  const int lane = lane_id();
  skey[lane] = make_int2(__float_as_int(ka), ia);
  skey[kWave + lane] = make_int2(__float_as_int(kb), ib);
  wave_lds_sync();
  int a = 0, b = 0;
  for (int k = 0; k < nA; ++k) {
    const int2 e = skey[k];
    const float kk = __int_as_float(e.x);
    a += key_less(kk, e.y, ka, ia);
    b += key_less(kk, e.y, kb, ib);
  }
  for (int k = 0; k < nB; ++k) {
    const int2 e = skey[kWave + k];
    const float kk = __int_as_float(e.x);
    a += key_less(kk, e.y, ka, ia);
    b += key_less(kk, e.y, kb, ib);
  }
  ra = a;
  rb = b;
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Sorting keys: (squared distance bits << 32) | index.  Distances are >= 0,
// so the unsigned order of the bits is the numeric order and ties between
// equal distances go to the smaller index; an empty slot is all ones.
// ---------------------------------------------------------------------------
constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ uint64_t pack_key(float d2, int id) {
  return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)id;
}
__device__ __forceinline__ int key_id(uint64_t k) { return (int)(uint32_t)k; }
__device__ __forceinline__ float key_d2(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }

template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppSwap1, 0xF, 0xF, false);
  else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppSwap2, 0xF, 0xF, false);
  else if constexpr (J < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);
  else return (uint32_t)__shfl_xor((int)v, J);
}

// One compare-exchange stage of a bitonic network: block size KB, distance J.
template <int KB, int J>
__device__ __forceinline__ void bitonic_stage(uint64_t& key, uint32_t& aux, int lane) {
  const uint32_t lo = xor_lane<J>((uint32_t)key);
  const uint32_t hi = xor_lane<J>((uint32_t)(key >> 32));
  const uint32_t pa = xor_lane<J>(aux);
  const uint64_t pk = ((uint64_t)hi << 32) | lo;
  const bool up = (lane & KB) == 0;            // this block sorts ascending
  const bool low = (lane & J) == 0;            // lower lane of the pair
  const bool take_min = (low == up);
  const bool mine = take_min ? (key <= pk) : (key >= pk);
  key = mine ? key : pk;
  aux = mine ? aux : pa;
}

// Ascending bitonic sort of one key (+ an attached word) per lane over
// aligned groups of NL lanes (NL = 32 or 64).
template <int NL>
__device__ __forceinline__ void bitonic_sort(uint64_t& key, uint32_t& aux) {
  const int lane = lane_id();
  bitonic_stage<2, 1>(key, aux, lane);
  bitonic_stage<4, 2>(key, aux, lane);
  bitonic_stage<4, 1>(key, aux, lane);
  bitonic_stage<8, 4>(key, aux, lane);
  bitonic_stage<8, 2>(key, aux, lane);
  bitonic_stage<8, 1>(key, aux, lane);
  bitonic_stage<16, 8>(key, aux, lane);
  bitonic_stage<16, 4>(key, aux, lane);
  bitonic_stage<16, 2>(key, aux, lane);
  bitonic_stage<16, 1>(key, aux, lane);
  bitonic_stage<NL == 32 ? 0 : 32, 16>(key, aux, lane);
  bitonic_stage<NL == 32 ? 0 : 32, 8>(key, aux, lane);
  bitonic_stage<NL == 32 ? 0 : 32, 4>(key, aux, lane);
  bitonic_stage<NL == 32 ? 0 : 32, 2>(key, aux, lane);
  bitonic_stage<NL == 32 ? 0 : 32, 1>(key, aux, lane);
  if constexpr (NL == 64) {
    bitonic_stage<0, 32>(key, aux, lane);
    bitonic_stage<0, 16>(key, aux, lane);
    bitonic_stage<0, 8>(key, aux, lane);
    bitonic_stage<0, 4>(key, aux, lane);
    bitonic_stage<0, 2>(key, aux, lane);
    bitonic_stage<0, 1>(key, aux, lane);
  }
}

// Number of keys of the ascending array a[0..n) below k (n <= MAXN, a power
// of two; keys past n are not read).
template <int MAXN = 64>
__device__ __forceinline__ int count_below(const uint64_t* a, int n, uint64_t k) {
  int pos = 0;
#pragma unroll
  for (int step = MAXN; step >= 1; step >>= 1) {
    const int probe = pos + step;
    if (probe <= n && a[probe - 1] < k) pos = probe;
  }
  return pos;
}

// ---------------------------------------------------------------------------
// Per-wave open-addressing set of point ids in LDS (kHashSlots entries,
// -1 = empty), filled with LDS compare-and-swap; tag bits ride along.
// ---------------------------------------------------------------------------
// SLOTS entries (a power of two, 256 by default; 512 where lists longer than
// a wave go in).
constexpr int kHashSlots = 256;

template <int SLOTS = kHashSlots>
__device__ __forceinline__ int hash_slot(int id) {
  constexpr int kBits = SLOTS == 256 ? 8 : SLOTS == 512 ? 9 : 10;
  static_assert(SLOTS == (1 << kBits), "256, 512 or 1024 slots");
  // multiplicative hash on a 24-bit multiply (full rate; a 32-bit multiply
  // is not), the id's bits above 24 folded into the low ones first; the
  // product is shifted as unsigned (__umul24 is declared to return int)
  const uint32_t v = (uint32_t)id ^ ((uint32_t)id >> 24);
  const uint32_t h = (uint32_t)__umul24(v, 0x9E3779u);
  return (int)(h >> (32 - kBits));
}

template <int SLOTS = kHashSlots>
__device__ __forceinline__ void hash_clear(int* tab, int* tag) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < SLOTS / kWave; ++k) {
    tab[k * kWave + lane] = -1;
    if (tag) tag[k * kWave + lane] = 0;
  }
  wave_lds_sync();
}

// Insert id (id >= 0); returns true if it was absent.  Lanes with id < 0 do
// nothing and return false.  tag_bits (if a tag array is given) are OR-ed
// into the slot's tag whether or not the id was new.
template <int SLOTS = kHashSlots>
__device__ __forceinline__ bool hash_insert(int* tab, int* tag, int id, int tag_bits) {
  bool fresh = false;
  if (id >= 0) {
    int slot = hash_slot<SLOTS>(id);
    for (int probe = 0; probe < SLOTS; ++probe) {
      const int old = atomicCAS(&tab[slot], -1, id);
      if (old == -1 || old == id) {
        fresh = old == -1;
        if (tag) atomicOr(&tag[slot], tag_bits);
        break;
      }
      slot = (slot + 1) & (SLOTS - 1);
    }
  }
  wave_lds_sync();
  return fresh;
}

// Tag of id in the set (0 if absent or id < 0).
template <int SLOTS = kHashSlots>
__device__ __forceinline__ int hash_find(const int* tab, const int* tag, int id) {
  if (id < 0) return 0;
  int slot = hash_slot<SLOTS>(id);
  for (int probe = 0; probe < SLOTS; ++probe) {
    const int v = tab[slot];
    if (v == id) return tag ? tag[slot] : 1;
    if (v == -1) return 0;
    slot = (slot + 1) & (SLOTS - 1);
  }
  return 0;
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
    const float bl = beta * 1.44269504f;   // exp(-beta D) = 2^(-beta log2(e) D)
    const float e = act ? exp2f(-bl * D) : 0.0f;
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

// ---------------------------------------------------------------------------
// The same calibration for a sorted row of K <= kMaxLong distances held in
// LDS (lists longer than a wave): lane l takes entries l, l + 64, ...; each
// sum adds a lane's entries in that order, then across the wave.
// ---------------------------------------------------------------------------
constexpr int kMaxLong = 256;   // longest HD list

__device__ inline float4 calibrate_row_lds(const float* d2, int K, const Hyper& h,
                                           float beta_prev) {
  constexpr int R = kMaxLong / kWave;
  const int lane = lane_id();
  const float m = d2[0];
  const float r = d2[K - 1];
  float D[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    D[q] = k < K ? d2[k] - m : 0.0f;
  }
  if (!(r > m)) return make_float4(0.0f, m, r, 1.0f / (float)K);
  int ties = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) ties += __popcll(__ballot(q * kWave + lane < K && D[q] == 0.0f));
  if ((float)ties >= h.perplexity) return make_float4(1e30f, m, r, 1.0f / (float)ties);
  auto lane_sum = [&](auto f) {
    float v = 0.0f;
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (q * kWave + lane < K) v += f(D[q]);
    return wave_sum_uniform(v);
  };
  const float target = h.ln_perp;
  float beta = beta_prev;
  if (!(beta > 0.0f && beta < 1e29f)) beta = (float)K / lane_sum([](float x) { return x; });
  float lo = 0.0f, hi = __int_as_float(0x7f800000);
  for (int it = 0; it < 48; ++it) {
    const float bl = beta * 1.44269504f;   // exp(-beta D) = 2^(-beta log2(e) D)
    const float S = lane_sum([&](float x) { return exp2f(-bl * x); });
    const float T = lane_sum([&](float x) { return exp2f(-bl * x) * x; });
    const float U = lane_sum([&](float x) { return exp2f(-bl * x) * x * x; });
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
  const float S = lane_sum([&](float x) { return expf(-beta * x); });
  return make_float4(beta, m, r, 1.0f / S);
}

// ---------------------------------------------------------------------------
// The same calibration for two rows at once, one per 32-lane half of the
// wave (lanes < K of each half; K <= 32).  Every quantity of a half is
// uniform within it; the sums over a half add the same values in the same
// order as the single-row version, so a row gets the same result bit for
// bit.  active: this half has a row to calibrate.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float half_sum_uniform(float v) {
  v = group_sum_dpp(v, 32);   // lane 31 of each half holds the half's sum
  return __shfl(v, (lane_id() & 32) + 31);
}

__device__ inline float4 calibrate_row_half(float d2, int K, const Hyper& h, float beta_prev,
                                            bool active) {
  const int lane = lane_id(), hbase = lane & 32, hl = lane & 31;
  const bool act = hl < K;
  const float m = __shfl(d2, hbase);
  const float r = __shfl(d2, hbase + K - 1);
  const float D = act ? d2 - m : 0.0f;
  const int ties = __popc((uint32_t)(__ballot(act && D == 0.0f) >> hbase));
  float4 special = make_float4(0.0f, m, r, 1.0f / (float)K);
  bool done = !active, fixed = false;
  if (!done && !(r > m)) {
    done = fixed = true;
  } else if (!done && (float)ties >= h.perplexity) {
    special = make_float4(1e30f, m, r, 1.0f / (float)ties);
    done = fixed = true;
  }
  const float target = h.ln_perp;
  float beta = __shfl(beta_prev, hbase);
  const float sD = half_sum_uniform(D);
  if (!(beta > 0.0f && beta < 1e29f)) beta = (float)K / sD;
  float lo = 0.0f, hi = __int_as_float(0x7f800000);
  for (int it = 0; it < 48; ++it) {
    if (__ballot(!done) == 0ull) break;
    const float bl = beta * 1.44269504f;   // exp(-beta D) = 2^(-beta log2(e) D)
    const float e = act ? exp2f(-bl * D) : 0.0f;
    const float S = half_sum_uniform(e);
    const float T = half_sum_uniform(e * D);
    const float U = half_sum_uniform(e * D * D);
    if (done) continue;
    const float mean = T / S;
    const float f = logf(S) + beta * mean - target;
    if (fabsf(f) <= 1e-6f) {
      done = true;
      continue;
    }
    if (f > 0.0f)
      lo = beta;
    else
      hi = beta;
    if (hi < 3e38f && hi - lo <= 2e-7f * hi) {
      done = true;
      continue;
    }
    const float var = U / S - mean * mean;
    float bn = beta + f / (beta * var);
    if (!(bn > lo && bn < hi)) bn = (hi < 3e38f) ? 0.5f * (lo + hi) : 2.0f * beta;
    beta = bn;
  }
  const float S = half_sum_uniform(act ? expf(-beta * D) : 0.0f);
  return fixed ? special : make_float4(beta, m, r, 1.0f / S);
}

}  // namespace fsne
