// HIP kernels of the FUnc-SNE iteration for gfx950.
//
// One wavefront owns one point (4 waves per 256-thread block).  Per
// iteration the host queues, on one stream:
//   hd_refine  (exits at once unless the coin of this iteration fired)
//   psym       (likewise)
//   ld_grad    LD refinement at the current Y plus gradient partials
//   reduce     fixed-order partial sums of Zh and of the HD flags
//   update     Z, momentum update, and the scalars of the next iteration
// Every phase reads the previous phase's buffers and writes its own
// (neighbour lists are double-buffered), so no kernel reads what another
// wave of the same kernel writes, and no float atomics are used.
#include "fsne_kernels.h"

#include <float.h>
#include <limits.h>

namespace fsne {

constexpr float kInf = __builtin_huge_valf();
constexpr int kNoId = INT_MAX;

// ---------------------------------------------------------------------------
// HD rows.  TX is float or uint16_t (bfloat16 bit patterns); VEC elements
// are loaded at once.  A sub-group of G lanes (G = 16, 32 or 64, chosen at
// run time from D) covers one row; 64/G rows are processed per pass.
// Each lane sums its elements in index order; the sub-group then reduces by
// an xor butterfly, so every HD distance in the library is computed with
// the same rounding sequence, whichever point of the pair owns the work.
// ---------------------------------------------------------------------------
template <typename TX>
__device__ __forceinline__ float to_f32(TX v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<uint16_t>(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}

template <typename TX, int VEC>
struct VecLoad;
template <>
struct VecLoad<float, 4> {
  static __device__ __forceinline__ void load(const float* p, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct VecLoad<float, 1> {
  static __device__ __forceinline__ void load(const float* p, float* o) { o[0] = *p; }
};
template <>
struct VecLoad<uint16_t, 8> {
  static __device__ __forceinline__ void load(const uint16_t* p, float* o) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      o[2 * k] = __uint_as_float(w[k] << 16);
      o[2 * k + 1] = __uint_as_float(w[k] & 0xFFFF0000u);
    }
  }
};
template <>
struct VecLoad<uint16_t, 1> {
  static __device__ __forceinline__ void load(const uint16_t* p, float* o) { o[0] = to_f32(*p); }
};

// A lane's chunk of a row kept as loaded (BF16 rows stay packed, two values
// per register) and widened to FP32 element by element where it is used.
template <typename TX, int VEC>
struct RawChunk;
template <>
struct RawChunk<float, 4> {
  float4 r;
  __device__ __forceinline__ void load(const float* p) { r = *reinterpret_cast<const float4*>(p); }
  __device__ __forceinline__ void zero() { r = make_float4(0.0f, 0.0f, 0.0f, 0.0f); }
  __device__ __forceinline__ float at(int v) const {
    return v == 0 ? r.x : v == 1 ? r.y : v == 2 ? r.z : r.w;
  }
};
template <>
struct RawChunk<float, 1> {
  float r;
  __device__ __forceinline__ void load(const float* p) { r = *p; }
  __device__ __forceinline__ void zero() { r = 0.0f; }
  __device__ __forceinline__ float at(int) const { return r; }
};
template <>
struct RawChunk<uint16_t, 8> {
  uint4 r;
  __device__ __forceinline__ void load(const uint16_t* p) { r = *reinterpret_cast<const uint4*>(p); }
  __device__ __forceinline__ void zero() { r = make_uint4(0u, 0u, 0u, 0u); }
  __device__ __forceinline__ float at(int v) const {
    const uint32_t w = (v >> 1) == 0 ? r.x : (v >> 1) == 1 ? r.y : (v >> 1) == 2 ? r.z : r.w;
    return __uint_as_float((v & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
};
template <>
struct RawChunk<uint16_t, 1> {
  uint16_t r;
  __device__ __forceinline__ void load(const uint16_t* p) { r = *p; }
  __device__ __forceinline__ void zero() { r = 0; }
  __device__ __forceinline__ float at(int) const { return __uint_as_float((uint32_t)r << 16); }
};

struct RowGeom {
  int G;       // lanes per row
  int lg;      // log2 G
  int chunks;  // vectors per lane
};

__device__ __forceinline__ RowGeom row_geom(int D, int VEC) {
  const int V = (D + VEC - 1) / VEC;
  RowGeom r;
  r.G = V <= 16 ? 16 : (V <= 32 ? 32 : 64);
  r.lg = V <= 16 ? 4 : (V <= 32 ? 5 : 6);
  r.chunks = (V + r.G - 1) / r.G;
  return r;
}

// Squared distances from x_i to the rows whose ids lanes 0..nrows-1 hold in
// cid (negative: skip).  Results go to sd2[0..nrows).  CH bounds the vectors
// per lane; x_i stays in registers and the loads of U passes are issued
// before their reductions.
template <typename TX, int VEC, int CH>
__device__ void hd_dist_rows(const TX* __restrict__ X, int D, int32_t i, int cid, int nrows,
                             float* sd2) {
  constexpr int U = CH >= 4 ? 1 : 4;
  const int lane = lane_id();
  const RowGeom geo = row_geom(D, VEC);
  const int g = lane >> geo.lg, sl = lane & (geo.G - 1);
  const int R = kWave >> geo.lg;
  // chunks stay as loaded (packed BF16: half the registers), widened at use
  RawChunk<TX, VEC> xi[CH];
  const TX* xr = X + (int64_t)i * D;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int e = (sl + k * geo.G) * VEC;
    if (k < geo.chunks && e < D)
      xi[k].load(xr + e);
    else
      xi[k].zero();
  }
  for (int p = 0; p < nrows; p += R * U) {
    float acc[U];
    RawChunk<TX, VEC> xc[U][CH];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int slot = p + u * R + g;
      const int c = __shfl(cid, slot & (kWave - 1));
      const bool ok = slot < nrows && c >= 0;
      const TX* cr = X + (int64_t)(ok ? c : i) * D;
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int e = (sl + k * geo.G) * VEC;
        if (k < geo.chunks && e < D)
          xc[u][k].load(cr + e);
        else
          xc[u][k] = xi[k];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < CH; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const float df = xi[k].at(v) - xc[u][k].at(v);
          s = fmaf(df, df, s);
        }
      acc[u] = group_sum_dpp(s, geo.G);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int slot = p + u * R + g;
      if (sl == geo.G - 1 && slot < nrows) sd2[slot] = acc[u];
    }
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Candidate generation (shared by the HD and the LD refinement).  Slot s of
// point i at iteration t draws Philox block (i, t, stream, s):
//   s  0..15  L[L[i][a]][b]     own-space neighbour of neighbour
//   s 16..19  Lx[i][a]          other-space neighbour
//   s 20..27  Lx[Lx[i][a]][b]   other-space neighbour of neighbour
//   s 28..31  uniform other point
// with a, b = floor(u * K / 2^32) from the block's first two words.  own /
// other hold i's rows of L and Lx, one entry per lane.  A slot is dropped
// if it gives i, an entry of i's own list, or the id of an earlier slot, and
// with MEMO also if it is one of the rejections i remembers (memo, one id
// per lane, -1 for none): those would lose the merge again.
// Returns the candidate id in lanes 0..31 (-1: dropped), -1 elsewhere.
// ---------------------------------------------------------------------------
// make_candidate_u takes the draw of its slot (lanes 0..31) from the caller;
// with OTHER_MEM, i's row of Lx is read from memory (lists longer than a
// wave) instead of from `other`.
template <bool MEMO = false, bool OTHER_MEM = false>
__device__ __forceinline__ int make_candidate_u(const uint4 u, int32_t i,
                                                const int32_t* __restrict__ L, int K, int own,
                                                const int32_t* __restrict__ Lx, int Kx, int other,
                                                int32_t N, int* tab, int memo = -1) {
  const int lane = lane_id();
  const int s = lane & (kCand - 1);
  const int a_own = (int)draw_index(u.x, (uint32_t)K);
  const int a_oth = (int)draw_index(u.x, (uint32_t)Kx);
  const int j_own = __shfl(own, a_own);
  int j_oth;
  if constexpr (OTHER_MEM)
    j_oth = Lx[(int64_t)i * Kx + a_oth];
  else
    j_oth = __shfl(other, a_oth);
  int c = -1;
  if (lane < kCand) {
    if (s < kSameNoN)
      c = L[(int64_t)j_own * K + draw_index(u.y, (uint32_t)K)];
    else if (s < kCrossDir)
      c = j_oth;
    else if (s < kCrossNoN)
      c = Lx[(int64_t)j_oth * Kx + draw_index(u.y, (uint32_t)Kx)];
    else
      c = draw_other(u.x, i, N);
  }
  // Duplicates go through a per-wave hash set: i's own list first, then the
  // candidates; of several equal candidates exactly one is inserted.  The
  // surviving set of ids is the one the earliest-slot rule keeps.
  hash_clear(tab, nullptr);
  hash_insert(tab, nullptr, lane < K ? own : -1, 0);
  if constexpr (MEMO) hash_insert(tab, nullptr, memo, 0);
  const bool fresh = hash_insert(tab, nullptr, (lane < kCand && c != i) ? c : -1, 0);
  return fresh ? c : -1;
}

template <bool MEMO = false>
__device__ __forceinline__ int make_candidate(int32_t i, uint32_t t, uint32_t stream,
                                              const Hyper& h, const int32_t* __restrict__ L,
                                              int K, int own, const int32_t* __restrict__ Lx,
                                              int Kx, int other, int32_t N, int* tab,
                                              int memo = -1) {
  const uint4 u =
      philox((uint32_t)i, t, stream, (uint32_t)(lane_id() & (kCand - 1)), h.key0, h.key1);
  return make_candidate_u<MEMO>(u, i, L, K, own, Lx, Kx, other, N, tab, memo);
}

// ---------------------------------------------------------------------------
// Random list completion: lst[0..n_have) holds ids already in the list; it
// is filled up to K distinct other points with the draws (i, t, stream, s),
// s = 0, 1, ... < 64K, completed if need be by i+1, i+2, ... (mod N).
// Draws are taken 64 at a time; a draw is a duplicate if it repeats an id of
// the list or an earlier draw of its round.  Initial lists are the case
// t = 0, n_have = 0.  The list goes to lst[0..K) (LDS).
// ---------------------------------------------------------------------------
__device__ void random_list(int32_t i, int32_t N, int K, uint32_t stream, uint32_t t,
                            const Hyper& h, int* lst, int n_have) {
  const int lane = lane_id();
  int n = n_have;
  for (int base = 0; n < K && base < kWave * K; base += kWave) {
    const uint4 u = philox((uint32_t)i, t, stream, (uint32_t)(base + lane), h.key0, h.key1);
    const int c = draw_other(u.x, i, N);
    bool dup = false;
    for (int k = 0; k < n; ++k) dup |= (lst[k] == c);
    for (int k = 0; k < kWave; ++k) dup |= (k < lane && c == __builtin_amdgcn_readlane(c, k));
    const uint64_t acc = __ballot(!dup);
    const int pos = n + popc_below(acc, lane);
    if (!dup && pos < K) lst[pos] = c;
    wave_lds_sync();
    n = min(K, n + (int)__popcll(acc));
  }
  if (n < K && lane == 0) {
    for (int32_t c = (i + 1) % N; n < K; c = (c + 1) % N) {
      bool dup = (c == i);
      for (int k = 0; k < n; ++k) dup |= (lst[k] == c);
      if (!dup) lst[n++] = c;
    }
  }
  wave_lds_sync();
}

struct WaveLds {
  int2 key[2 * kWave];
  float d2[kWave];
  float row[kWave];
  int lst[kWave];
  int tab[kHashSlots];
  uint64_t ck[kWave];
  uint64_t ok[kWave];
};

template <typename TX, int VEC, int CH>
__global__ __launch_bounds__(kBlock) void k_init_lists(const TX* __restrict__ X, int32_t N,
                                                       int32_t i0, int D, int Kh, int Kl,
                                                       Hyper h, int32_t* __restrict__ hd_idx,
                                                       float* __restrict__ hd_d2,
                                                       int32_t* __restrict__ ld_idx,
                                                       float4* __restrict__ rec,
                                                       uint8_t* __restrict__ flags) {
  __shared__ WaveLds lds_all[kWavesPerBlock];
  WaveLds& S = lds_all[threadIdx.x / kWave];
  const int32_t i = i0 + (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= N) return;
  const int lane = lane_id();
  random_list(i, N, Kl, kStreamInitLD, 0u, h, S.lst, 0);
  if (lane < Kl) ld_idx[(int64_t)i * Kl + lane] = S.lst[lane];
  wave_lds_sync();
  random_list(i, N, Kh, kStreamInitHD, 0u, h, S.lst, 0);
  const int id = lane < Kh ? S.lst[lane] : -1;
  hd_dist_rows<TX, VEC, CH>(X, D, i, id, Kh, S.d2);
  const float dd = lane < Kh ? S.d2[lane] : kInf;
  const int ii = lane < Kh ? id : kNoId;
  int ra, rb;
  rank_two(dd, ii, kInf, kNoId, Kh, 0, S.key, ra, rb);
  if (lane < Kh) {
    hd_idx[(int64_t)i * Kh + ra] = ii;
    hd_d2[(int64_t)i * Kh + ra] = dd;
    S.d2[ra] = dd;
  }
  wave_lds_sync();
  const float sorted = lane < Kh ? S.d2[lane] : 0.0f;
  const float4 r = calibrate_row(sorted, Kh, h, 0.0f);
  if (lane == 0) {
    rec[i] = r;
    flags[i] = 1;
  }
}

// Moves the non-negative ids of lanes 0..31 to lanes 0..n-1 (in lane order)
// and returns n; the other lanes get -1.
__device__ __forceinline__ int compact_ids(int& c, int* scratch) {
  const int lane = lane_id();
  const uint64_t m = __ballot(c >= 0);
  const int n = __popcll(m);
  if (c >= 0) scratch[popc_below(m, lane)] = c;
  wave_lds_sync();
  c = lane < n ? scratch[lane] : -1;
  wave_lds_sync();
  return n;
}

// ---------------------------------------------------------------------------
// BF16 screen of the candidates: dot products x_i . x_c on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  A pass takes 16 candidate
// rows as A (16 x 32 per instruction: lane l supplies row l mod 16 and the 8
// elements 8 (l / 16) .. +8 of each 32-wide step, so an instruction reads 64
// contiguous bytes of each of its 16 rows); every column of B holds x_i, so
// column 0 of C = A B holds the 16 dot products: lane 16 g, register r holds
// row 4 g + r.  The slots' products go to sdot; returns this lane's (lanes
// 0..31).
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

constexpr int kScreenRows = 16;   // candidate rows per matrix-core pass
constexpr int kScreenK = 32;      // elements of a row per instruction

__device__ __forceinline__ f32x4_t screen_pass(const uint16_t* __restrict__ ar, bool have_a,
                                               const uint16_t* __restrict__ br, int D, int kb) {
  constexpr int kSteps = 2;   // loads of two steps go out before the first product
  f32x4_t acc = {};
  for (int k0 = 0; k0 < D; k0 += kScreenK * kSteps) {
    uint4 av[kSteps], bv[kSteps];
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
      const int e = k0 + kScreenK * u + 8 * kb;   // this lane's 8 elements (D % 16 == 0)
      av[u] = make_uint4(0, 0, 0, 0);
      bv[u] = make_uint4(0, 0, 0, 0);
      if (e < D) {
        if (have_a) av[u] = *reinterpret_cast<const uint4*>(ar + e);
        bv[u] = *reinterpret_cast<const uint4*>(br + e);
      }
    }
#pragma unroll
    for (int u = 0; u < kSteps; ++u)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, av[u]),
                                                    __builtin_bit_cast(bf16x8_t, bv[u]), acc,
                                                    0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ float screen_dots(const uint16_t* __restrict__ X, int D, int32_t i,
                                             int c, float* sdot) {
  const int lane = lane_id(), row = lane & (kScreenRows - 1), kb = lane >> 4;
  const uint16_t* br = X + (int64_t)i * D;
  for (int p = 0; p < kCand; p += kScreenRows) {
    const int cr = __shfl(c, p + row);
    const f32x4_t acc = screen_pass(X + (int64_t)(cr >= 0 ? cr : i) * D, cr >= 0, br, D, kb);
    if (row == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) sdot[p + 4 * kb + r] = acc[r];
    }
  }
  wave_lds_sync();
  const float v = sdot[lane & (kCand - 1)];
  wave_lds_sync();
  return v;
}

// ---------------------------------------------------------------------------
// New memory of rejected candidates: this refinement's rejections first (the
// screened-out ids in lane order, then the re-ranked losers in key order),
// then the old entries, as many as the row's width (32 or 64) holds.  The
// new ids are never among the old ones (those were not evaluated), so the
// row stays duplicate-free.  One point per wave; old: entry `lane` of the row
// (lanes < width); lanes >= kCand pass -1 as rejections.
// ---------------------------------------------------------------------------
static_assert(kMemo == kWave && kCand <= 32, "one remembered entry per lane at the widest");

__device__ __forceinline__ void remember_rejections(int32_t* __restrict__ row, int width,
                                                    int old, int screened_out, int rejected,
                                                    int* lst) {
  const int lane = lane_id();
  const uint64_t ms = __ballot(screened_out >= 0);
  const uint64_t mr = __ballot(rejected >= 0);
  const int ns = __popcll(ms), nr = __popcll(mr);
  if (ns + nr == 0) return;
  if (screened_out >= 0) lst[popc_below(ms, lane)] = screened_out;
  if (rejected >= 0) lst[ns + popc_below(mr, lane)] = rejected;
  wave_lds_sync();
  const int nn = ns + nr;
  const int shifted = __shfl(old, lane >= nn ? lane - nn : 0);
  if (lane < width) row[lane] = lane < nn ? lst[lane] : shifted;
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// HD refinement of point i (runs when the coin fired): candidates from the
// HD lists and the LD lists of iteration t, their distances, merge into the
// sorted list, flag, and recalibration of beta_i when the list changed.
// ---------------------------------------------------------------------------
// What an HD refinement leaves for the affinity pass that follows it, 32
// bytes per point: the point's calibration record, then the distances at
// ranks Kh/2 - 1, Kh/4 - 1 and 3Kh/4 - 1 of its new list, where the
// membership scan halves its range (zero unless Kh is a multiple of 8).  The
// pass reads the record half for every entry it recomputes and the cut half
// only where it scans, from the line the first read brought in, so a
// neighbour's record and cuts cost one line where the record and two of its
// list's distances took two or three.
__device__ __forceinline__ void write_psym_head(float4* psh, int32_t i, const float4& rec,
                                                const float* row, int Kh) {
  float4 c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if ((Kh & 7) == 0) {
    c.x = row[Kh / 2 - 1];
    c.y = row[Kh / 4 - 1];
    c.z = row[3 * Kh / 4 - 1];
  }
  psh[2 * (int64_t)i] = rec;
  psh[2 * (int64_t)i + 1] = c;
}

template <typename TX, int VEC, int CH, bool SCREEN>
__global__ __launch_bounds__(kBlock) void k_hd_refine(StepArgs a) {
  const Scalars* sc = a.sc;
  if (!sc->fire) return;
  __shared__ WaveLds lds_all[kWavesPerBlock];
  WaveLds& S = lds_all[threadIdx.x / kWave];
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const int lane = lane_id();
  const uint32_t t = sc->t;
  const int cur = sc->hd_cur;
  const int Kh = a.Kh, Kl = a.Kl;
  const int32_t* hin = a.hd_idx[cur];
  const float* din = a.hd_d2[cur];
  const int32_t* lin = a.ld_idx[t & 1];
  const int own = lane < Kh ? hin[(int64_t)i * Kh + lane] : -1;
  const float od2 = lane < Kh ? din[(int64_t)i * Kh + lane] : kInf;
  const int oth = lane < Kl ? lin[(int64_t)i * Kl + lane] : -1;
  const int memo = (a.memo && lane < a.memo_w) ? a.memo[(int64_t)i * kMemo + lane] : -1;
  // candidates, compacted into lanes 0 .. n-1 so that only n rows are visited
  int c = make_candidate<true>(i, t, kStreamHDC, a.h, hin, Kh, own, lin, Kl, oth, a.N, S.tab,
                               memo);
  int n = compact_ids(c, S.lst);
  const int nload = n;   // candidate rows read from X
  int screened_out = -1;
  if constexpr (SCREEN) {
    // keep the candidates whose expanded-form distance
    // |x_i|^2 + |x_c|^2 - 2 x_i.x_c is within the current K-th distance (1 + margin)
    const float dot = screen_dots(static_cast<const uint16_t*>(a.X), a.D, i, c, S.d2);
    const float r_i = readlane_f(od2, Kh - 1);
    const float approx = a.xnorm[i] + (c >= 0 ? a.xnorm[c] : 0.0f) - 2.0f * dot;
    const bool keep = c >= 0 && approx <= r_i * (1.0f + a.h.margin);
    screened_out = keep ? -1 : c;
    c = keep ? c : -1;
    n = compact_ids(c, S.lst);
  }
  hd_dist_rows<TX, VEC, CH>(static_cast<const TX*>(a.X), a.D, i, c, n, S.d2);
  // sort the candidates by (distance, index), then rank old entries and
  // candidates against each other by binary search
  uint64_t ck = c >= 0 ? pack_key(S.d2[lane & (kCand - 1)], c) : kNoKey;
  uint32_t aux = 0;
  bitonic_sort<32>(ck, aux);
  const int ncand = n;
  const uint64_t ko = lane < Kh ? pack_key(od2, own) : kNoKey;
  S.ck[lane] = ck;
  S.ok[lane] = ko;
  wave_lds_sync();
  int32_t* hout = a.hd_idx[cur ^ 1];
  float* dout = a.hd_d2[cur ^ 1];
  // The stored list is ordered by this key, except after a state load whose
  // order came from other arithmetic (equal FP32 distances); then sort it.
  uint64_t ks = ko;
  uint32_t below = (uint32_t)lane;     // old entries before this one
  {
    const uint32_t nlo = (uint32_t)__shfl_down((int)(uint32_t)ko, 1);
    const uint32_t nhi = (uint32_t)__shfl_down((int)(uint32_t)(ko >> 32), 1);
    const uint64_t next = ((uint64_t)nhi << 32) | nlo;
    if (__ballot(lane + 1 < Kh && !(ko < next)) != 0ull) {
      bitonic_sort<kWave>(ks, below);   // below: original lane of the sorted key
      S.ok[lane] = ks;
      wave_lds_sync();
      const uint32_t src = below;
      below = (uint32_t)lane;
      // sorted position of this lane's own entry
      for (int k = 0; k < Kh; ++k)
        if (__builtin_amdgcn_readlane((int)src, k) == lane) below = (uint32_t)k;
    }
  }
  if (lane < Kh) {
    const int ro = (int)below + count_below(S.ck, ncand, ko);
    if (ro < Kh) {
      hout[(int64_t)i * Kh + ro] = own;
      dout[(int64_t)i * Kh + ro] = od2;
      S.row[ro] = od2;
    }
  }
  bool enter = false;
  if (lane < ncand) {
    const int rc = lane + count_below(S.ok, Kh, ck);
    enter = rc < Kh;
    if (enter) {
      hout[(int64_t)i * Kh + rc] = key_id(ck);
      dout[(int64_t)i * Kh + rc] = key_d2(ck);
      S.row[rc] = key_d2(ck);
    }
  }
  wave_lds_sync();
  const bool changed = __ballot(enter) != 0ull;
  // bit 0: list changed; bits 1..6: candidate rows loaded (for measurement)
  if (lane == 0) a.flags[i] = (uint8_t)((changed ? 1 : 0) | (nload << 1));
  if (a.memo) {
    const int rejected = (lane < ncand && !enter) ? key_id(ck) : -1;
    remember_rejections(a.memo + (int64_t)i * kMemo, a.memo_w, memo, screened_out, rejected,
                        S.lst);
  }
  float4 r = a.rec[i];
  if (changed) {
    const float sorted = lane < Kh ? S.row[lane] : 0.0f;
    r = calibrate_row(sorted, Kh, a.h, r.x);
    if (lane == 0) a.rec[i] = r;
  }
  if (lane == 0) write_psym_head(a.psh, i, r, S.row, Kh);
}

// ---------------------------------------------------------------------------
// The HD refinement for two points per wave (K_hd, K_ld <= 32; rows that fit
// one vector per lane).  Half h = lane / 32 handles point 2 w + h; every
// phase that needs at most 32 lanes per point (candidates, de-duplication,
// sorting, ranking, calibration) runs for both points in the same
// instructions, while the candidate rows of both points share the row
// groups of the distance pass.  Each point gets exactly what the one-point
// kernel computes: the same draws, the same per-row arithmetic and the same
// order of additions.
// ---------------------------------------------------------------------------
struct WaveLds2 {
  int tab[2 * kHashSlots];   // one hash set per half
  float d2[kWave];           // candidate distances, point 0's slots first
  float row[kWave];          // new list distances, 32 per half
  int lst[kWave];            // compaction scratch, 32 per half
  uint64_t ck[kWave];        // sorted candidate keys, 32 per half
  uint64_t ok[kWave];        // old list keys, 32 per half
};

// remember_rejections for the two points of a wave, each half on its own row
// of MW entries; old[r] holds entry 32 r + hl of the half's row.
template <int MW>
__device__ __forceinline__ void remember_rejections2(int32_t* __restrict__ memo, int32_t i,
                                                     bool live, const int* old,
                                                     int screened_out, int rejected, int* lst) {
  constexpr int R = MW / 32;
  const int lane = lane_id(), hl = lane & 31, hb = lane & 32;
  const uint32_t ms = (uint32_t)(__ballot(screened_out >= 0) >> hb);
  const uint32_t mr = (uint32_t)(__ballot(rejected >= 0) >> hb);
  const int ns = __popc(ms), nn = ns + __popc(mr);
  const uint32_t below = (1u << hl) - 1u;
  if (screened_out >= 0) lst[hb + __popc(ms & below)] = screened_out;
  if (rejected >= 0) lst[hb + ns + __popc(mr & below)] = rejected;
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = 32 * r + hl;            // position in the new row
    const int q = p - nn;                 // position in the old row (p >= nn)
    const int src = hb + (q & 31);
    int shifted = -1;
#pragma unroll
    for (int r2 = 0; r2 < R; ++r2) {
      const int v = __shfl(old[r2], src);
      if (q >= 0 && (q >> 5) == r2) shifted = v;
    }
    if (live && nn > 0) memo[(int64_t)i * kMemo + p] = p < nn ? lst[hb + p] : shifted;
  }
  wave_lds_sync();
}

// Squared distances for the candidates of both points: slots 0..n0-1 are the
// ids in lanes 0..n0-1 (point i0), slots n0..n0+n1-1 those in lanes
// 32..32+n1-1 (point i1).  Results go to sd2[slot].
template <typename TX, int VEC>
__device__ void hd_dist_rows2(const TX* __restrict__ X, int D, int32_t i0, int32_t i1, int cid,
                              int n0, int n1, float* sd2) {
  constexpr int U = VEC >= 8 ? 2 : 4;   // loads in flight per lane, within the register budget
  const int lane = lane_id();
  const RowGeom geo = row_geom(D, VEC);
  const int g = lane >> geo.lg, sl = lane & (geo.G - 1);
  const int R = kWave >> geo.lg;
  const int e = sl * VEC;
  const bool in_row = e < D;
  // the two points' chunks stay as loaded: packed BF16 needs half the registers
  RawChunk<TX, VEC> xa, xb;
  if (in_row) {
    xa.load(X + (int64_t)i0 * D + e);
    xb.load(X + (int64_t)i1 * D + e);
  } else {
    xa.zero();
    xb.zero();
  }
  const int nrows = n0 + n1;
  for (int p = 0; p < nrows; p += R * U) {
    RawChunk<TX, VEC> xc[U];
    bool second[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int slot = p + u * R + g;
      second[u] = slot >= n0;
      const int src = second[u] ? 32 + slot - n0 : slot;
      const int c = __shfl(cid, src & (kWave - 1));
      const bool ok = slot < nrows && c >= 0;
      if (in_row)
        xc[u].load(X + (int64_t)(ok ? c : i0) * D + e);
      else
        xc[u].zero();
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float s = 0.0f;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const float df = (second[u] ? xb.at(v) : xa.at(v)) - xc[u].at(v);
        s = fmaf(df, df, s);
      }
      const float acc = group_sum_dpp(s, geo.G);
      const int slot = p + u * R + g;
      if (sl == geo.G - 1 && slot < nrows) sd2[slot] = acc;
    }
  }
  wave_lds_sync();
}

// The BF16 screen for two points at once.  Slots 0..n0-1 are the ids in
// lanes 0..n0-1 (candidates of point i0), slots n0..n0+n1-1 those in lanes
// 32..32+n1-1 (point i1).  Each pass takes 16 slots as the rows of A; the
// columns of B hold x_i0 (0..7) and x_i1 (8..15), so the product of slot s
// with its own point is column 0 or 8 of its row.  sdot[slot] gets it.
__device__ void screen_dots2(const uint16_t* __restrict__ X, int D, int32_t i0, int32_t i1,
                             int cid, int n0, int n1, float* sdot) {
  const int lane = lane_id(), row = lane & (kScreenRows - 1), kb = lane >> 4;
  const uint16_t* br = X + (int64_t)(row < 8 ? i0 : i1) * D;
  const int nrows = n0 + n1;
  for (int p = 0; p < nrows; p += kScreenRows) {
    const int slot = p + row;
    const int src = slot >= n0 ? 32 + slot - n0 : slot;
    const int cs = __shfl(cid, src & (kWave - 1));
    const int cr = slot < nrows ? cs : -1;
    const f32x4_t acc = screen_pass(X + (int64_t)(cr >= 0 ? cr : i0) * D, cr >= 0, br, D, kb);
    // lanes 16 g (column 0) and 16 g + 8 (column 8) hold rows 4 g .. 4 g + 3
    if (row == 0 || row == 8) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = p + 4 * kb + r;
        if (s < nrows && ((s < n0) == (row == 0))) sdot[s] = acc[r];
      }
    }
  }
  wave_lds_sync();
}

template <typename TX, int VEC, bool SCREEN, int MW>
__global__ __launch_bounds__(kBlock) void k_hd_refine2(StepArgs a) {
  static_assert(MW % 32 == 0 && MW <= kMemo, "whole rows of 32 per half");
  const Scalars* sc = a.sc;
  if (!sc->fire) return;
  __shared__ WaveLds2 lds_all[kWavesPerBlock];
  WaveLds2& S = lds_all[threadIdx.x / kWave];
  const int32_t w = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (2 * w >= a.N) return;
  const int lane = lane_id(), h = lane >> 5, hl = lane & 31, hb = h * 32;
  const int32_t i = 2 * w + h;
  const bool live = i < a.N;                 // the last wave may hold one point
  const int32_t i0 = 2 * w, i1 = i0 + 1 < a.N ? i0 + 1 : i0;   // wave-uniform
  const uint32_t t = sc->t;
  const int cur = sc->hd_cur;
  const int Kh = a.Kh, Kl = a.Kl;
  const int32_t* hin = a.hd_idx[cur];
  const float* din = a.hd_d2[cur];
  const int32_t* lin = a.ld_idx[t & 1];
  const int own = (live && hl < Kh) ? hin[(int64_t)i * Kh + hl] : -1;
  const float od2 = (live && hl < Kh) ? din[(int64_t)i * Kh + hl] : kInf;
  const int oth = (live && hl < Kl) ? lin[(int64_t)i * Kl + hl] : -1;
  int memo[MW / 32];        // entries hl, hl + 32, ... of i's row
#pragma unroll
  for (int r = 0; r < MW / 32; ++r)
    memo[r] = (a.memo && live) ? a.memo[(int64_t)i * kMemo + 32 * r + hl] : -1;

  // candidates (the one-point rule, per half)
  int c = -1;
  {
    const uint4 u = philox((uint32_t)i, t, kStreamHDC, (uint32_t)hl, a.h.key0, a.h.key1);
    const int a_own = (int)draw_index(u.x, (uint32_t)Kh);
    const int a_oth = (int)draw_index(u.x, (uint32_t)Kl);
    const int j_own = __shfl(own, hb + a_own);
    const int j_oth = __shfl(oth, hb + a_oth);
    if (live) {
      if (hl < kSameNoN)
        c = hin[(int64_t)j_own * Kh + draw_index(u.y, (uint32_t)Kh)];
      else if (hl < kCrossDir)
        c = j_oth;
      else if (hl < kCrossNoN)
        c = lin[(int64_t)j_oth * Kl + draw_index(u.y, (uint32_t)Kl)];
      else
        c = draw_other(u.x, i, a.N);
    }
    int* tab = S.tab + h * kHashSlots;
#pragma unroll
    for (int k = 0; k < kHashSlots / 32; ++k) tab[k * 32 + hl] = -1;
    wave_lds_sync();
    hash_insert(tab, nullptr, hl < Kh ? own : -1, 0);
#pragma unroll
    for (int r = 0; r < MW / 32; ++r) hash_insert(tab, nullptr, memo[r], 0);
    const bool fresh = hash_insert(tab, nullptr, c != i ? c : -1, 0);
    c = fresh ? c : -1;
  }
  // compact each half's candidates to its first lanes
  int n;
  {
    const uint32_t m = (uint32_t)(__ballot(c >= 0) >> hb);
    n = __popc(m);
    if (c >= 0) S.lst[hb + __popc(m & ((1u << hl) - 1u))] = c;
    wave_lds_sync();
    c = hl < n ? S.lst[hb + hl] : -1;
    wave_lds_sync();
  }
  const int nload = n;
  int n0 = __shfl(n, 0), n1 = __shfl(n, 32);
  int screened_out = -1;
  if constexpr (SCREEN) {
    // keep the candidates whose expanded-form distance
    // |x_i|^2 + |x_c|^2 - 2 x_i.x_c is within the current K-th distance (1 + margin)
    screen_dots2(static_cast<const uint16_t*>(a.X), a.D, i0, i1, c, n0, n1, S.d2);
    const float r_i = __shfl(od2, hb + Kh - 1);
    const float dot = hl < n ? S.d2[(h ? n0 : 0) + hl] : 0.0f;
    const float approx = (live ? a.xnorm[i] : 0.0f) + (c >= 0 ? a.xnorm[c] : 0.0f) - 2.0f * dot;
    const bool keep = c >= 0 && approx <= r_i * (1.0f + a.h.margin);
    screened_out = keep ? -1 : c;
    c = keep ? c : -1;
    wave_lds_sync();
    const uint32_t m = (uint32_t)(__ballot(c >= 0) >> hb);
    n = __popc(m);
    if (c >= 0) S.lst[hb + __popc(m & ((1u << hl) - 1u))] = c;
    wave_lds_sync();
    c = hl < n ? S.lst[hb + hl] : -1;
    wave_lds_sync();
    n0 = __shfl(n, 0);
    n1 = __shfl(n, 32);
  }
  hd_dist_rows2<TX, VEC>(static_cast<const TX*>(a.X), a.D, i0, i1, c, n0, n1, S.d2);
  uint64_t ck = c >= 0 ? pack_key(S.d2[(h ? n0 : 0) + hl], c) : kNoKey;
  uint32_t aux = 0;
  bitonic_sort<32>(ck, aux);
  const int ncand = n;
  const uint64_t ko = (live && hl < Kh) ? pack_key(od2, own) : kNoKey;
  S.ck[lane] = ck;
  S.ok[lane] = ko;
  wave_lds_sync();
  int32_t* hout = a.hd_idx[cur ^ 1];
  float* dout = a.hd_d2[cur ^ 1];
  // a stored list that is not in key order (after a state load) is sorted first
  uint32_t below = (uint32_t)hl;
  {
    const uint32_t nlo = (uint32_t)__shfl_down((int)(uint32_t)ko, 1);
    const uint32_t nhi = (uint32_t)__shfl_down((int)(uint32_t)(ko >> 32), 1);
    const uint64_t next = ((uint64_t)nhi << 32) | nlo;
    const uint64_t bad = __ballot(hl + 1 < Kh && !(ko < next));
    if (bad != 0ull) {
      const bool mine = ((uint32_t)(bad >> hb)) != 0u;
      uint64_t sk = ko;
      uint32_t src = (uint32_t)hl;
      bitonic_sort<32>(sk, src);
      if (mine) S.ok[lane] = sk;
      wave_lds_sync();
      uint32_t pos = (uint32_t)hl;
      for (int k = 0; k < Kh; ++k)
        if ((uint32_t)__shfl((int)src, hb + k) == (uint32_t)hl) pos = (uint32_t)k;
      if (mine) below = pos;
    }
  }
  if (live && hl < Kh) {
    const int ro = (int)below + count_below(S.ck + hb, ncand, ko);
    if (ro < Kh) {
      hout[(int64_t)i * Kh + ro] = own;
      dout[(int64_t)i * Kh + ro] = od2;
      S.row[hb + ro] = od2;
    }
  }
  bool enter = false;
  if (live && hl < ncand) {
    const int rc = hl + count_below(S.ok + hb, Kh, ck);
    enter = rc < Kh;
    if (enter) {
      hout[(int64_t)i * Kh + rc] = key_id(ck);
      dout[(int64_t)i * Kh + rc] = key_d2(ck);
      S.row[hb + rc] = key_d2(ck);
    }
  }
  wave_lds_sync();
  const bool changed = ((uint32_t)(__ballot(enter) >> hb)) != 0u;
  if (live && hl == 0) a.flags[i] = (uint8_t)((changed ? 1 : 0) | (nload << 1));
  if (a.memo) {
    const int rejected = (live && hl < ncand && !enter) ? key_id(ck) : -1;
    remember_rejections2<MW>(a.memo, i, live, memo, screened_out, rejected, S.lst);
  }
  float4 r = live ? a.rec[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (__ballot(changed) != 0ull) {
    const float sorted = hl < Kh ? S.row[hb + hl] : 0.0f;
    const float4 rn = calibrate_row_half(sorted, Kh, a.h, r.x, changed);
    if (changed) r = rn;
    if (changed && hl == 0) a.rec[i] = r;
  }
  if (live && hl == 0) write_psym_head(a.psh, i, r, S.row + hb, Kh);
}

// ---------------------------------------------------------------------------
// HD lists longer than a wave (64 < K_hd <= kMaxLong, K_ld <= 64): one point
// per wave, its list in LDS with entry k handled by lane k mod 64.  The same
// candidates, merge rule, flags, remembered rejections and calibration as
// k_hd_refine; the merge ranks the old entries against the sorted candidates
// and the candidates against the old list by binary search.
// ---------------------------------------------------------------------------
constexpr int kLongSlots = 2 * kHashSlots;   // ids of the list, memory and candidates

struct WaveLdsLong {
  uint64_t ok[kMaxLong];    // list keys (d2 bits << 32 | id), ascending
  float row[kMaxLong];      // distances of the new (or initial) list
  int lst[kMaxLong];        // ids of the initial list; compaction scratch
  uint64_t ck[kCand];       // sorted candidate keys
  float d2[kWave];          // candidate distances
  int tab[kLongSlots];
};

// Sorts the n <= kMaxLong distinct keys of a[] ascending in place: each lane
// ranks its entries against all n, then writes them to their ranks.
__device__ void rank_sort_lds(uint64_t* a, int n) {
  constexpr int R = kMaxLong / kWave;
  const int lane = lane_id();
  uint64_t mine[R];
  int rank[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    mine[q] = k < n ? a[k] : kNoKey;
    rank[q] = 0;
  }
  for (int m = 0; m < n; ++m) {
    const uint64_t v = a[m];
#pragma unroll
    for (int q = 0; q < R; ++q) rank[q] += v < mine[q] ? 1 : 0;
  }
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (q * kWave + lane < n) a[rank[q]] = mine[q];
  wave_lds_sync();
}

template <typename TX, int VEC, int CH>
__global__ __launch_bounds__(kBlock) void k_hd_refine_long(StepArgs a) {
  constexpr int R = kMaxLong / kWave;
  const Scalars* sc = a.sc;
  if (!sc->fire) return;
  __shared__ WaveLdsLong lds_all[kWavesPerBlock];
  WaveLdsLong& S = lds_all[threadIdx.x / kWave];
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const int lane = lane_id();
  const uint32_t t = sc->t;
  const int cur = sc->hd_cur;
  const int Kh = a.Kh, Kl = a.Kl;
  const int32_t* hin = a.hd_idx[cur];
  const float* din = a.hd_d2[cur];
  const int32_t* lin = a.ld_idx[t & 1];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    if (k < Kh) S.ok[k] = pack_key(din[(int64_t)i * Kh + k], hin[(int64_t)i * Kh + k]);
  }
  const int oth = lane < Kl ? lin[(int64_t)i * Kl + lane] : -1;
  const int memo = (a.memo && lane < a.memo_w) ? a.memo[(int64_t)i * kMemo + lane] : -1;
  wave_lds_sync();
  // candidates, as make_candidate with i's own list read from LDS (in its
  // stored order: the draws index it)
  const uint4 u =
      philox((uint32_t)i, t, kStreamHDC, (uint32_t)(lane & (kCand - 1)), a.h.key0, a.h.key1);
  const int j_oth = __shfl(oth, (int)draw_index(u.x, (uint32_t)Kl));
  int c = -1;
  if (lane < kCand) {
    if (lane < kSameNoN) {
      const int j = key_id(S.ok[draw_index(u.x, (uint32_t)Kh)]);
      c = hin[(int64_t)j * Kh + draw_index(u.y, (uint32_t)Kh)];
    } else if (lane < kCrossDir) {
      c = j_oth;
    } else if (lane < kCrossNoN) {
      c = lin[(int64_t)j_oth * Kl + draw_index(u.y, (uint32_t)Kl)];
    } else {
      c = draw_other(u.x, i, a.N);
    }
  }
  // the stored list is in key order except after a state load whose order
  // came from other arithmetic: then sort it for the merge
  bool unsorted = false;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    if (k + 1 < Kh) unsorted |= !(S.ok[k] < S.ok[k + 1]);
  }
  if (__ballot(unsorted) != 0ull) rank_sort_lds(S.ok, Kh);
  hash_clear<kLongSlots>(S.tab, nullptr);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    hash_insert<kLongSlots>(S.tab, nullptr, k < Kh ? key_id(S.ok[k]) : -1, 0);
  }
  hash_insert<kLongSlots>(S.tab, nullptr, memo, 0);
  const bool fresh =
      hash_insert<kLongSlots>(S.tab, nullptr, (lane < kCand && c != i) ? c : -1, 0);
  c = fresh ? c : -1;
  const int n = compact_ids(c, S.lst);
  hd_dist_rows<TX, VEC, CH>(static_cast<const TX*>(a.X), a.D, i, c, n, S.d2);
  uint64_t ck = c >= 0 ? pack_key(S.d2[lane & (kCand - 1)], c) : kNoKey;
  uint32_t aux = 0;
  bitonic_sort<32>(ck, aux);
  if (lane < kCand) S.ck[lane] = ck;
  wave_lds_sync();
  int32_t* hout = a.hd_idx[cur ^ 1];
  float* dout = a.hd_d2[cur ^ 1];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    if (k < Kh) {
      const uint64_t ko = S.ok[k];
      const int ro = k + count_below<kCand>(S.ck, n, ko);
      if (ro < Kh) {
        hout[(int64_t)i * Kh + ro] = key_id(ko);
        dout[(int64_t)i * Kh + ro] = key_d2(ko);
        S.row[ro] = key_d2(ko);
      }
    }
  }
  bool enter = false;
  if (lane < n) {
    const int rc = lane + count_below<kMaxLong>(S.ok, Kh, ck);
    enter = rc < Kh;
    if (enter) {
      hout[(int64_t)i * Kh + rc] = key_id(ck);
      dout[(int64_t)i * Kh + rc] = key_d2(ck);
      S.row[rc] = key_d2(ck);
    }
  }
  wave_lds_sync();
  const bool changed = __ballot(enter) != 0ull;
  if (lane == 0) a.flags[i] = (uint8_t)((changed ? 1 : 0) | (n << 1));
  if (a.memo) {
    const int rejected = (lane < n && !enter) ? key_id(ck) : -1;
    remember_rejections(a.memo + (int64_t)i * kMemo, a.memo_w, memo, -1, rejected, S.lst);
  }
  float4 r = a.rec[i];
  if (changed) {
    r = calibrate_row_lds(S.row, Kh, a.h, r.x);
    if (lane == 0) a.rec[i] = r;
  }
  if (lane == 0) write_psym_head(a.psh, i, r, S.row, Kh);
}

// Initial lists for K_hd > 64: the rule of k_init_lists, the HD list sorted
// in LDS.
template <typename TX, int VEC, int CH>
__global__ __launch_bounds__(kBlock) void k_init_lists_long(const TX* __restrict__ X, int32_t N,
                                                            int32_t i0, int D, int Kh, int Kl,
                                                            Hyper h, int32_t* __restrict__ hd_idx,
                                                            float* __restrict__ hd_d2,
                                                            int32_t* __restrict__ ld_idx,
                                                            float4* __restrict__ rec,
                                                            uint8_t* __restrict__ flags) {
  constexpr int R = kMaxLong / kWave;
  __shared__ WaveLdsLong lds_all[kWavesPerBlock];
  WaveLdsLong& S = lds_all[threadIdx.x / kWave];
  const int32_t i = i0 + (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= N) return;
  const int lane = lane_id();
  random_list(i, N, Kl, kStreamInitLD, 0u, h, S.lst, 0);
  if (lane < Kl) ld_idx[(int64_t)i * Kl + lane] = S.lst[lane];
  wave_lds_sync();
  random_list(i, N, Kh, kStreamInitHD, 0u, h, S.lst, 0);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int base = q * kWave;
    if (base < Kh) {
      const int k = base + lane;
      hd_dist_rows<TX, VEC, CH>(X, D, i, k < Kh ? S.lst[k] : -1, min(kWave, Kh - base),
                                S.row + base);
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    if (k < Kh) S.ok[k] = pack_key(S.row[k], S.lst[k]);
  }
  wave_lds_sync();
  rank_sort_lds(S.ok, Kh);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = q * kWave + lane;
    if (k < Kh) {
      hd_idx[(int64_t)i * Kh + k] = key_id(S.ok[k]);
      hd_d2[(int64_t)i * Kh + k] = key_d2(S.ok[k]);
      S.row[k] = key_d2(S.ok[k]);
    }
  }
  wave_lds_sync();
  const float4 r = calibrate_row_lds(S.row, Kh, h, 0.0f);
  if (lane == 0) {
    rec[i] = r;
    flags[i] = 1;
  }
}

// ---------------------------------------------------------------------------
// Symmetrised affinities of point i (eq. (1)) over its HD list:
//   P_ik = (p_{j|i} + p_{i|j}) / (2N), j = HD[i][k],
//   p_{j|i} = exp(-beta_i (d2 - m_i)) invS_i,
//   p_{i|j} = exp(-beta_j (d2 - m_j)) invS_j if i is in j's HD list, else 0.
// standalone = 1: run regardless of the coin, on the current lists.
// ---------------------------------------------------------------------------
constexpr int kPsymHalvings = 2;   // range halvings of the membership scan
static_assert(kPsymHalvings == 2, "the list cuts a refinement leaves cover two halvings");

__global__ __launch_bounds__(kBlock) void k_psym(StepArgs a, int standalone) {
  const Scalars* sc = a.sc;
  const int fire = standalone ? 0 : sc->fire;
  if (!standalone && !fire) return;
  // one thread per list entry, so that no lane idles whatever K_hd is
  const int Kh = a.Kh;
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q >= (int64_t)a.N * Kh) return;
  const int32_t i = (int32_t)(q / Kh);
  const int buf = sc->hd_cur ^ fire;
  const int32_t* hl = a.hd_idx[buf];
  const float* hd = a.hd_d2[buf];
  const int32_t j = hl[q];
  // After a refinement an entry's value can only change if point i or point j
  // changed its list, and so its record (the flag bit 0 of this refinement):
  // other entries keep the value they hold.  A standalone pass recomputes all.
  // (j's flag is read only when i's is clear: early on nearly every point changes)
  if (!standalone && !(a.flags[i] & 1u) && !(a.flags[j] & 1u)) return;
  const float d2 = hd[q];
  const float4 ri = a.rec[i];
  // after a refinement j's record comes from the line that also holds its
  // list cuts (the same values as rec[j])
  const float4 rj = standalone ? a.rec[j] : a.psh[2 * (int64_t)j];
  const float pji = expf(-ri.x * (d2 - ri.y)) * ri.w;
  // Every stored HD distance comes from the same symmetric FP32 computation,
  // so i can only be in j's sorted list if d2 <= r_j (j's largest distance);
  // the list itself is scanned only then, 16 bytes per load.
  bool member = false;
  if (d2 <= rj.z * (1.0f + 1e-6f)) {
    const int32_t* row = hl + (int64_t)j * Kh;
    if ((Kh & 7) == 0) {
      int lo = 0, hi = Kh;   // entries that can hold i
      if (!standalone) {
        // A refinement leaves every list sorted by (distance, index), and
        // both lists of a pair hold the same distance (up to the rounding of
        // an injected state, hence the band): i can only be in the part of
        // j's list its distance falls in, found by halving the range while
        // the parts stay whole 4-entry groups; near a cut both are kept.
        // (the cuts come from the refinement: Kh/2, then Kh/4 or 3Kh/4)
        const float4 cj = a.psh[2 * (int64_t)j + 1];
        for (int h = 0; h < kPsymHalvings && ((hi - lo) & 7) == 0; ++h) {
          const int m = (lo + hi) >> 1;
          const float cut = h == 0 ? cj.x : lo == 0 ? cj.y : cj.z;
          if (d2 < cut * (1.0f - 1e-5f))
            hi = m;
          else if (d2 > cut * (1.0f + 1e-5f))
            lo = m;
          else
            break;
        }
      }
      const int k0 = lo >> 2, k1 = hi >> 2;   // in 4-entry groups
      const int4* r4 = reinterpret_cast<const int4*>(row);
      for (int k = k0; k < k1; ++k) {
        const int4 v = r4[k];
        member |= (v.x == i) | (v.y == i) | (v.z == i) | (v.w == i);
      }
    } else if ((Kh & 3) == 0) {
      const int4* r4 = reinterpret_cast<const int4*>(row);
      for (int k = 0; k < (Kh >> 2); ++k) {
        const int4 v = r4[k];
        member |= (v.x == i) | (v.y == i) | (v.z == i) | (v.w == i);
      }
    } else {
      for (int k = 0; k < Kh; ++k) member |= (row[k] == i);
    }
  }
  const float pij = member ? expf(-rj.x * (d2 - rj.y)) * rj.w : 0.0f;
  a.P[q] = (pji + pij) / (2.0f * (float)a.N);
}

// ---------------------------------------------------------------------------
// LD refinement of point i at Y_t and its gradient partials (eqs. (4)-(6),
// attraction and repulsion kept apart):
//   A_i  = sum_k P_ik w^(1/a) (y_i - y_j)         over the HD list
//   R_i  = sum_{j in U} w^(1+1/a) (y_i - y_j) + (N-1)/n_neg sum_s [j_s not in U] ...
//   Zh_i = sum_{j in U} w + (N-1)/n_neg sum_s [j_s not in U] w
// with w = (1 + d^2/alpha)^(-alpha), U = HD list union new LD list.  Rows
// of Y are stored with a padded stride DP (zeros beyond d).
// ---------------------------------------------------------------------------
// Row-group layout: a row of DP floats is spread over G lanes, VEC floats
// each, so one load instruction fetches RPI whole rows (coalesced per row).
template <int DP, int KLM = kWave>
struct LdGeom {
  static constexpr int VEC = DP >= 4 ? 4 : DP;
  static constexpr int G = DP / VEC;
  static constexpr int LG = G == 1 ? 0 : G == 2 ? 1 : G == 4 ? 2 : G == 8 ? 3 : 4;
  static constexpr int RPI = kWave / G;
  static constexpr int MAXE = KLM + kCand;                  // LD entries: old list + slots
  static constexpr int MAXP = (MAXE + RPI - 1) / RPI;         // passes over the entries
  // keep entry rows in registers only while they are few: at wider rows the
  // registers cost more occupancy than the second read of the kept entries
  static constexpr bool CACHE = MAXP * VEC <= 24;
};

template <int VEC>
__device__ __forceinline__ void load_chunk(const float* __restrict__ p, float* r) {
  if constexpr (VEC == 4) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
  } else {
    const float2 v = *reinterpret_cast<const float2*>(p);
    r[0] = v.x; r[1] = v.y;
  }
}

// The LD distance that decides list membership: the squares, each rounded,
// summed pairwise as a balanced binary tree with the components in index
// order at the leaves (padding components are zero and change nothing).  A
// lane holds VEC consecutive components, the row's G lanes hold the row in
// order, so the lane's pairs come first, then neighbouring lanes, quads,
// 8-lane and 16-lane groups are added by DPP exchanges inside the row
// (x + y = y + x exactly, so both sides of a pair get the same node); every
// lane of the group ends with the total.  G <= 16, so no exchange leaves a
// row and none goes through LDS.
template <int DP>
__device__ __forceinline__ float ld_decision_d2(const float* yi, const float* yj, int q) {
#pragma clang fp contract(off)
  using Geo = LdGeom<DP>;
  float sq[Geo::VEC];
#pragma unroll
  for (int v = 0; v < Geo::VEC; ++v) {
    const float df = yj[v] - yi[v];
    sq[v] = df * df;
  }
  float s;
  if constexpr (Geo::VEC == 4)
    s = (sq[0] + sq[1]) + (sq[2] + sq[3]);
  else
    s = sq[0] + sq[1];
  static_assert(Geo::G <= 16, "a row group stays within a DPP row");
  s = group_sum_dpp(s, Geo::G);
  (void)q;
  return s;
}

// Sum over the G lanes of a row group (G <= 16: every lane gets it).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  return group_sum_dpp(v, G);
}

// Sum over the lanes holding the same chunk (lane mod G): row rotations by
// G, 2G, ... < 16 within each row, then the four rows.
template <int G>
__device__ __forceinline__ float strided_sum(float v) {
  if constexpr (G <= 1) v += dpp<0x121>(v);   // row_ror:1
  if constexpr (G <= 2) v += dpp<0x122>(v);   // row_ror:2
  if constexpr (G <= 4) v += dpp<0x124>(v);   // row_ror:4
  if constexpr (G <= 8) v += dpp<0x128>(v);   // row_ror:8
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

template <int HS = kHashSlots>
struct LdLds {
  int ent[2 * kWave];     // LD entries: candidate slots, then the old list (-1: none)
  float dd[2 * kWave];    // their decision distances
  int2 key[2 * kWave];    // rank scratch
  int newl[kWave];        // new LD list
  int kind[2 * kWave];    // 1: entry kept and not an HD neighbour
  int neg[kWave];         // negative samples outside U (-1: none)
  int tab[HS];            // hash set of ids (candidate dedupe, then U)
  int tag[HS];            // 1: HD neighbour, 2: new LD neighbour
};

// Adds one neighbour's contribution to this lane's components:
//   A += patt w^(1/a) (y_i - y_j),  R += scale w^(1+1/a) (y_i - y_j);
// returns scale * w (the Zh term), with w = (1 + q2/alpha)^(-alpha).
template <int VEC>
__device__ __forceinline__ float pair_terms(const float* yi, const float* yj, float q2,
                                            const Hyper& h, float patt, float scale, float* A,
                                            float* R) {
  // the base is at least 1, so the hardware reciprocal (within 1 ulp) is
  // well conditioned here and costs one instruction instead of a division
  const float wa = __builtin_amdgcn_rcpf(fmaf(q2, h.inv_alpha, 1.0f));
  float w;
  if (h.alpha == 1.0f)
    w = wa;
  else if (h.alpha == 0.5f)
    w = sqrtf(wa);
  else
    w = exp2f(h.alpha * log2f(wa));
  const float fa = patt * wa, fr = scale * w * wa;
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const float dy = yi[v] - yj[v];
    A[v] = fmaf(fa, dy, A[v]);
    R[v] = fmaf(fr, dy, R[v]);
  }
  return scale * w;
}

// KLM bounds the LD list length (32 or 64), which sizes the entry passes; HL
// bounds the HD list length: 64 (held one entry per lane) or kMaxLong (read
// from memory where it is used; the set U then needs a larger hash table).
template <int DP, int KLM, int HL = kWave>
__global__ __launch_bounds__(kBlock) void k_ld_grad(StepArgs a) {
  using Geo = LdGeom<DP, KLM>;
  constexpr int VEC = Geo::VEC, G = Geo::G, RPI = Geo::RPI;
  constexpr bool LONG_H = HL > kWave;
  constexpr int HS = LONG_H ? 2 * kHashSlots : kHashSlots;
  constexpr int LP = (HL + RPI - 1) / RPI;      // passes over the HD list
  constexpr bool PRE_H = !LONG_H && LP * VEC <= 8;   // HD rows kept in registers
  constexpr bool PRE_E = Geo::CACHE;            // entry rows kept in registers
  // negative samples' rows loaded with the first loads only for narrow rows:
  // at d = 16 their registers cost the kernel its eighth wave per SIMD
  // (70 against 64 VGPRs), which was worth more than the early load
  constexpr bool PRE_N = DP <= 8;
  __shared__ LdLds<HS> lds_all[kWavesPerBlock];
  LdLds<HS>& S = lds_all[threadIdx.x / kWave];
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const Scalars* sc = a.sc;
  const int lane = lane_id();
  const int q = lane & (G - 1);          // chunk of a row this lane holds
  const int rg = lane >> Geo::LG;        // row slot within a pass
  const uint32_t t = sc->t;
  const int hb = sc->hd_cur ^ sc->fire;  // HD lists after this iteration's HD phase
  const int Kh = a.Kh, Kl = a.Kl, nneg = a.h.n_neg;
  const int ne = kCand + Kl;             // entries: candidate slots [0,32), old LD list after
  const int32_t* hl = a.hd_idx[hb];
  const int32_t* lin = a.ld_idx[t & 1];
  int32_t* lout = a.ld_idx[(t & 1) ^ 1];
  const float* yrow = a.Y + q * VEC;     // chunk q of row j: yrow + j * DP

  // Loads that do not depend on the candidates go out first: own row, lists,
  // HD neighbour rows, old LD neighbour rows, negative sample rows.
  float yi[VEC];
  load_chunk<VEC>(yrow + (int64_t)i * DP, yi);
  const int hid = (!LONG_H && lane < Kh) ? hl[(int64_t)i * Kh + lane] : -1;
  const float pk = (!LONG_H && lane < Kh) ? a.P[(int64_t)i * Kh + lane] : 0.0f;
  const int lid = lane < Kl ? lin[(int64_t)i * Kl + lane] : -1;
  // One Philox pass draws the candidate slots (lanes 0..31) and negative
  // samples 0..31 (lanes 32..63); negative s ends in lane s.
  const uint4 ud = philox((uint32_t)i, t, lane < kCand ? kStreamLDC : kStreamNeg,
                          (uint32_t)(lane & (kCand - 1)), a.h.key0, a.h.key1);
  int jn = __shfl(draw_other(ud.x, i, a.N), (lane + kCand) & (kWave - 1));
  if (nneg > kCand) {   // negatives 32..63
    const uint4 u2 = philox((uint32_t)i, t, kStreamNeg, (uint32_t)lane, a.h.key0, a.h.key1);
    if (lane >= kCand) jn = draw_other(u2.x, i, a.N);
  }
  if (lane >= nneg) jn = -1;
  float yh[PRE_H ? LP : 1][VEC];
  float er[PRE_E ? Geo::MAXP : 1][VEC];
  if constexpr (PRE_H) {
#pragma unroll
    for (int p = 0; p < LP; ++p) {
      const int r = p * RPI + rg;
      const int id = __shfl(hid, r & (kWave - 1));
      if (p * RPI < Kh && r < Kh) load_chunk<VEC>(yrow + (int64_t)id * DP, yh[p]);
    }
  }
  if constexpr (PRE_E) {
#pragma unroll
    for (int p = 0; p < Geo::MAXP; ++p) {
      const int e = p * RPI + rg;
      const int id = __shfl(lid, (e - kCand) & (kWave - 1));
      if (p * RPI + RPI > kCand && e >= kCand && e < ne)
        load_chunk<VEC>(yrow + (int64_t)id * DP, er[p]);
    }
  }
  float yn[PRE_N ? VEC : 1];
  if constexpr (PRE_N) {
    const int id = __shfl(jn, rg & (kWave - 1));
    if (nneg <= RPI && rg < nneg) load_chunk<VEC>(yrow + (int64_t)id * DP, yn);
  }

  const int c = make_candidate_u<false, LONG_H>(ud, i, lin, Kl, lid, hl, Kh, hid, a.N, S.tab);
  if (lane < kCand) S.ent[lane] = c;
  if (lane < Kl) S.ent[kCand + lane] = lid;
  {
    const int nc = __popcll(__ballot(c >= 0));
    if (lane == 0) a.ldc[i] = (uint8_t)nc;
  }
  if constexpr (PRE_E) {
#pragma unroll
    for (int p = 0; p < Geo::MAXP; ++p) {
      const int e = p * RPI + rg;
      const int id = __shfl(c, e & (kWave - 1));
      if (p * RPI < kCand && e < kCand && id >= 0)
        load_chunk<VEC>(yrow + (int64_t)id * DP, er[p]);
    }
  }
  wave_lds_sync();

  // decision distances of all entries
#pragma unroll
  for (int p = 0; p < Geo::MAXP; ++p) {
    if (p * RPI < ne) {
      const int e = p * RPI + rg;
      const int id = e < ne ? S.ent[e] : -1;
      float yj[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) yj[v] = yi[v];
      if (id >= 0) {
        if constexpr (PRE_E) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) yj[v] = er[p][v];
        } else {
          load_chunk<VEC>(yrow + (int64_t)id * DP, yj);
        }
      }
      const float dist = ld_decision_d2<DP>(yi, yj, q);
      if (q == G - 1 && e < ne) S.dd[e] = id >= 0 ? dist : kInf;
    }
  }
  wave_lds_sync();

  // merge: order the entries by (distance, index) and keep the first Kl
  bool keep = false;
  int kid = -1;
  if (Geo::MAXE <= kWave || ne <= kWave) {
    // each entry's rank among all entries by (distance, index): the valid
    // keys are distinct (the candidates differ from the list and from one
    // another), so the kept entries take the ranks 0 .. Kl-1.  The rank is
    // counted within the entry's half (candidate slots in lanes 0..31, the
    // old list in 32..63), each half is laid out in that order, and the
    // other half's keys below are found by binary search.
    const int e = lane;
    const int id = e < ne ? S.ent[e] : -1;
    const uint64_t key = id >= 0 ? pack_key(S.dd[e], id) : kNoKey;
    uint64_t* keys = reinterpret_cast<uint64_t*>(S.key);   // [0, 64): by lane
    uint64_t* sorted = keys + kWave;                        // [64, 128): halves sorted
    const int half = lane & kCand;
    keys[lane] = key;
    sorted[lane] = kNoKey;
    wave_lds_sync();
    int rank = 0;
#pragma unroll
    for (int m = 0; m < kCand; ++m) rank += keys[half + m] < key ? 1 : 0;
    if (key != kNoKey) sorted[half + rank] = key;
    wave_lds_sync();
    rank += count_below<kCand>(sorted + (half ^ kCand), kCand, key);
    const bool kept = key != kNoKey && rank < Kl;
    S.kind[lane] = kept ? 2 : 0;   // kept; refined below
    S.kind[kWave + lane] = 0;
    if (kept) {
      lout[(int64_t)i * Kl + rank] = id;
      S.newl[rank] = id;
    }
    wave_lds_sync();
    keep = lane < Kl;
    kid = keep ? S.newl[lane] : -1;
  } else {
    const int eA = lane, eB = kWave + lane;
    const int idA = eA < ne ? S.ent[eA] : -1;
    const int idB = eB < ne ? S.ent[eB] : -1;
    const float dA = idA >= 0 ? S.dd[eA] : kInf;
    const float dB = idB >= 0 ? S.dd[eB] : kInf;
    int rA, rB;
    rank_two(dA, idA >= 0 ? idA : kNoId, dB, idB >= 0 ? idB : kNoId, min(ne, kWave),
             max(ne - kWave, 0), S.key, rA, rB);
    const bool keepA = idA >= 0 && rA < Kl, keepB = idB >= 0 && rB < Kl;
    S.kind[eA] = keepA ? 2 : 0;
    S.kind[eB] = keepB ? 2 : 0;
    if (keepA) {
      lout[(int64_t)i * Kl + rA] = idA;
      S.newl[rA] = idA;
    }
    if (keepB) {
      lout[(int64_t)i * Kl + rB] = idB;
      S.newl[rB] = idB;
    }
    wave_lds_sync();
    keep = lane < Kl;
    kid = keep ? S.newl[lane] : -1;
  }
  wave_lds_sync();
  // U = HD list + new LD list as a tagged hash set: LD entries that are HD
  // neighbours too act once, as HD neighbours; negatives in U act not at all
  hash_clear<HS>(S.tab, S.tag);
  if constexpr (LONG_H) {
    for (int b = 0; b < Kh; b += kWave)
      hash_insert<HS>(S.tab, S.tag, b + lane < Kh ? hl[(int64_t)i * Kh + b + lane] : -1, 1);
  } else {
    hash_insert<HS>(S.tab, S.tag, lane < Kh ? hid : -1, 1);
  }
  hash_insert<HS>(S.tab, S.tag, kid, 2);
  for (int e = lane; e < ne; e += kWave) {
    if (S.kind[e] == 2) S.kind[e] = (hash_find<HS>(S.tab, S.tag, S.ent[e]) & 1) ? 0 : 1;
  }
  const bool n_in = hash_find<HS>(S.tab, S.tag, jn) != 0;
  S.neg[lane] = (lane < nneg && !n_in) ? jn : -1;
  wave_lds_sync();

  float A[VEC], R[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) A[v] = R[v] = 0.0f;
  float zh = 0.0f;
  // HD neighbours: attraction and repulsion
#pragma unroll
  for (int p = 0; p < LP; ++p) {
    if (p * RPI < Kh) {
      const int r = p * RPI + rg;
      float pr;
      float yj[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) yj[v] = yi[v];
      if constexpr (LONG_H) {
        pr = r < Kh ? a.P[(int64_t)i * Kh + r] : 0.0f;
        if (r < Kh) load_chunk<VEC>(yrow + (int64_t)hl[(int64_t)i * Kh + r] * DP, yj);
      } else if constexpr (PRE_H) {
        pr = __shfl(pk, r & (kWave - 1));
        if (r < Kh) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) yj[v] = yh[p][v];
        }
      } else {
        pr = __shfl(pk, r & (kWave - 1));
        const int id = __shfl(hid, r & (kWave - 1));
        if (r < Kh) load_chunk<VEC>(yrow + (int64_t)id * DP, yj);
      }
      float part = 0.0f;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const float dy = yi[v] - yj[v];
        part = fmaf(dy, dy, part);
      }
      const float q2 = group_sum<G>(part);
      if (r < Kh) {
        const float z = pair_terms<VEC>(yi, yj, q2, a.h, pr, 1.0f, A, R);
        if (q == 0) zh += z;
      }
    }
  }
  // LD neighbours that are not HD neighbours: repulsion
#pragma unroll
  for (int p = 0; p < Geo::MAXP; ++p) {
    if (p * RPI < ne) {
      const int e = p * RPI + rg;
      if (e < ne && S.kind[e]) {
        float yj[VEC];
        if constexpr (PRE_E) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) yj[v] = er[p][v];
        } else {
          load_chunk<VEC>(yrow + (int64_t)S.ent[e] * DP, yj);
        }
        const float z = pair_terms<VEC>(yi, yj, S.dd[e], a.h, 0.0f, 1.0f, A, R);
        if (q == 0) zh += z;
      }
    }
  }
  // negative samples outside U, weighted (N-1)/n_neg
  for (int b = 0; b < nneg; b += RPI) {
    const int r = b + rg;
    const int id = r < nneg ? S.neg[r] : -1;
    float yj[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) yj[v] = yi[v];
    if (id >= 0) {
      if (PRE_N && nneg <= RPI) {
#pragma unroll
        for (int v = 0; v < (PRE_N ? VEC : 1); ++v) yj[v] = yn[v];
      } else {
        load_chunk<VEC>(yrow + (int64_t)id * DP, yj);
      }
    }
    float part = 0.0f;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const float dy = yi[v] - yj[v];
      part = fmaf(dy, dy, part);
    }
    const float q2 = group_sum<G>(part);
    if (id >= 0) {
      const float z = pair_terms<VEC>(yi, yj, q2, a.h, 0.0f, a.neg_scale, A, R);
      if (q == 0) zh += z;
    }
  }
  // sum over the row slots (lanes holding the same chunk), then store
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    A[v] = strided_sum<G>(A[v]);
    R[v] = strided_sum<G>(R[v]);
  }
  zh = wave_sum_uniform(zh);
  if (lane < G) {
    float* ao = a.A + (int64_t)i * DP + lane * VEC;
    float* ro = a.R + (int64_t)i * DP + lane * VEC;
    if constexpr (VEC == 4) {
      *reinterpret_cast<float4*>(ao) = make_float4(A[0], A[1], A[2], A[3]);
      *reinterpret_cast<float4*>(ro) = make_float4(R[0], R[1], R[2], R[3]);
    } else {
      *reinterpret_cast<float2*>(ao) = make_float2(A[0], A[1]);
      *reinterpret_cast<float2*>(ro) = make_float2(R[0], R[1]);
    }
  }
  if (lane == 0) a.Zh[i] = zh;
}

// ---------------------------------------------------------------------------
// Fixed-order partial sums: block b sums Zh (and, when the coin fired, the
// flags) over its contiguous chunk of points.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(StepArgs a) {
  __shared__ float sz[256];
  __shared__ int sf[256];
  __shared__ uint32_t sh[256], sl[256];
  const int fire = a.sc->fire;
  const int64_t N = a.N;
  const int64_t chunk = (N + kReduceBlocks - 1) / kReduceBlocks;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < N ? lo + chunk : N;
  float z = 0.0f;
  int f = 0;
  uint32_t ch = 0, cl = 0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) {
    z += a.Zh[k];
    if (fire) {
      const uint32_t fl = a.flags[k];
      f += (int)(fl & 1u);
      ch += fl >> 1;
    }
    cl += a.ldc[k];
  }
  sz[threadIdx.x] = z;
  sf[threadIdx.x] = f;
  sh[threadIdx.x] = ch;
  sl[threadIdx.x] = cl;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sz[threadIdx.x] += sz[threadIdx.x + o];
      sf[threadIdx.x] += sf[threadIdx.x + o];
      sh[threadIdx.x] += sh[threadIdx.x + o];
      sl[threadIdx.x] += sl[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.zpart[blockIdx.x] = sz[0];
    a.fpart[blockIdx.x] = sf[0];
    a.cpart[blockIdx.x] = sh[0];
    a.cpart[kReduceBlocks + blockIdx.x] = sl[0];
  }
}

// Sum of the kReduceBlocks partials in a fixed order, by one 256-thread block.
__device__ float block_sum_partials(const float* part, float* s) {
  float v = 0.0f;
  for (int k = threadIdx.x; k < kReduceBlocks; k += 256) v += part[k];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  const float r = s[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Momentum update g = 4 (attr A - rep R / Z); V <- mu V - lr g; Y <- Y + V.
// Block 0 then advances the scalars: N_new, E (after an HD refinement), the
// HD buffer, t, and the coin of the next iteration.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_update(StepArgs a) {
  __shared__ float s[256];
  Scalars* sc = a.sc;
  const float Z = block_sum_partials(a.zpart, s);
  const float rz = a.h.rep / Z;
  const int64_t total = (int64_t)a.N * a.DP;
  bool bad = false;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * 256) {
    const float g = 4.0f * (a.h.attr * a.A[k] - rz * a.R[k]);
    const float v = a.h.momentum * a.V[k] - a.h.lr * g;
    const float y = a.Y[k] + v;
    a.V[k] = v;
    a.Y[k] = y;
    bad |= !isfinite(y);
  }
  if (bad) sc->nonfinite = 1;
  if (blockIdx.x == 0) {
    __shared__ int sf[256];
    __shared__ uint32_t sh[256], sl[256];
    const int fire = sc->fire;
    int f = 0;
    uint32_t ch = 0, cl = 0;
    for (int k = threadIdx.x; k < kReduceBlocks; k += 256) {
      if (fire) {
        f += a.fpart[k];
        ch += a.cpart[k];
      }
      cl += a.cpart[kReduceBlocks + k];
    }
    sf[threadIdx.x] = f;
    sh[threadIdx.x] = ch;
    sl[threadIdx.x] = cl;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
      if ((int)threadIdx.x < o) {
        sf[threadIdx.x] += sf[threadIdx.x + o];
        sh[threadIdx.x] += sh[threadIdx.x + o];
        sl[threadIdx.x] += sl[threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      sc->hd_cand = sh[0];
      sc->ld_cand = sl[0];
      const uint32_t t1 = sc->t + 1u;
      float E = sc->E;
      if (fire) {
        sc->n_new = sf[0];
        E = E_next(E, sf[0], a.N, a.h.e_smooth);
        sc->hd_cur ^= 1;
        sc->refinements += 1u;
      }
      sc->E = E;
      sc->Z = Z;
      sc->last_fired = fire;
      sc->t = t1;
      sc->fire = coin_fires(E, t1, a.h);
    }
  }
}

// Coin of the current iteration from (E, t), after init or a state load.
__global__ void k_set_fire(Scalars* sc, Hyper h) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc->fire = coin_fires(sc->E, sc->t, h);
}

// Y, V <- Y / f, V / f.
__global__ void k_scale(float* Y, float* V, int64_t n, float inv) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    Y[k] *= inv;
    V[k] *= inv;
  }
}

// ---------------------------------------------------------------------------
// Recalibration of every point (perplexity change) on the current lists.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_calibrate_all(StepArgs a) {
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const int lane = lane_id();
  const float* hd = a.hd_d2[a.sc->hd_cur];
  const float d2 = lane < a.Kh ? hd[(int64_t)i * a.Kh + lane] : 0.0f;
  const float4 r = calibrate_row(d2, a.Kh, a.h, a.rec[i].x);
  if (lane == 0) a.rec[i] = r;
}

// The same for lists longer than a wave (rows staged in LDS).
__global__ __launch_bounds__(kBlock) void k_calibrate_all_long(StepArgs a) {
  __shared__ float rows[kWavesPerBlock][kMaxLong];
  const int w = threadIdx.x / kWave;
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + w);
  if (i >= a.N) return;
  const int lane = lane_id();
  const float* hd = a.hd_d2[a.sc->hd_cur];
  for (int k = lane; k < a.Kh; k += kWave) rows[w][k] = hd[(int64_t)i * a.Kh + k];
  wave_lds_sync();
  const float4 r = calibrate_row_lds(rows[w], a.Kh, a.h, a.rec[i].x);
  if (lane == 0) a.rec[i] = r;
}

// ---------------------------------------------------------------------------
// Drift: recompute every HD entry that pairs with a moved point (moved[] is
// a per-point byte map), re-sort those rows, flag and recalibrate them.
// ---------------------------------------------------------------------------
template <typename TX, int VEC, int CH>
__global__ __launch_bounds__(kBlock) void k_drift_rows(StepArgs a, const uint8_t* moved) {
  __shared__ WaveLds lds_all[kWavesPerBlock];
  WaveLds& S = lds_all[threadIdx.x / kWave];
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const int lane = lane_id();
  const int Kh = a.Kh;
  const int cur = a.sc->hd_cur;
  int32_t* hl = a.hd_idx[cur];
  float* hd = a.hd_d2[cur];
  const int id = lane < Kh ? hl[(int64_t)i * Kh + lane] : -1;
  const float old = lane < Kh ? hd[(int64_t)i * Kh + lane] : kInf;
  const bool mi = moved[i] != 0;
  const bool redo = lane < Kh && (mi || moved[id] != 0);
  if (__ballot(redo) == 0ull) {
    if (lane == 0) a.flags[i] = 0;
    return;
  }
  hd_dist_rows<TX, VEC, CH>(static_cast<const TX*>(a.X), a.D, i, redo ? id : -1, Kh, S.d2);
  const float dd = lane < Kh ? (redo ? S.d2[lane] : old) : kInf;
  int ra, rb;
  rank_two(dd, lane < Kh ? id : kNoId, kInf, kNoId, Kh, 0, S.key, ra, rb);
  if (lane < Kh) {
    hl[(int64_t)i * Kh + ra] = id;
    hd[(int64_t)i * Kh + ra] = dd;
    S.d2[ra] = dd;
  }
  wave_lds_sync();
  const float sorted = lane < Kh ? S.d2[lane] : 0.0f;
  const float4 r = calibrate_row(sorted, Kh, a.h, a.rec[i].x);
  if (lane == 0) {
    a.rec[i] = r;
    a.flags[i] = 1;
  }
}

// ---------------------------------------------------------------------------
// Point deletion.  Rows moved by the compaction (see fsne_delete_points) are
// copied first; then every surviving point i < N' has its lists rewritten:
// ids pass through newid (deleted points map to -1).  HD: deleted entries
// are dropped and the row is refilled with random points (draws (i, t, 10,
// s)), whose distances are computed; the row is re-sorted by (d2, id) when
// anything in it changed, and recalibrated (flag set) when an entry was
// dropped.  LD: surviving entries keep their order, refills (draws
// (i, t, 11, s)) follow.
// ---------------------------------------------------------------------------
__global__ void k_move_rows(uint8_t* base, const int32_t* src, const int32_t* dst, int32_t m,
                            int32_t rowbytes) {
  const int64_t total = (int64_t)m * rowbytes;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = q / rowbytes, b = q % rowbytes;
    base[(int64_t)dst[k] * rowbytes + b] = base[(int64_t)src[k] * rowbytes + b];
  }
}

template <typename TX, int VEC, int CH>
__global__ __launch_bounds__(kBlock) void k_delete_fix(StepArgs a, const int32_t* newid) {
  __shared__ WaveLds lds_all[kWavesPerBlock];
  WaveLds& S = lds_all[threadIdx.x / kWave];
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const int lane = lane_id();
  const int Kh = a.Kh, Kl = a.Kl;
  const uint32_t t = a.sc->t;
  int32_t* hl = a.hd_idx[a.sc->hd_cur];
  float* hd = a.hd_d2[a.sc->hd_cur];
  int32_t* ll = a.ld_idx[t & 1u];
  // LD list: survivors in order, then refills
  {
    const int id = lane < Kl ? ll[(int64_t)i * Kl + lane] : -1;
    const int nid = id >= 0 ? newid[id] : -1;
    const uint64_t keep = __ballot(nid >= 0);
    const int nk = __popcll(keep);
    if (nid >= 0) S.lst[popc_below(keep, lane)] = nid;
    wave_lds_sync();
    if (nk < Kl) random_list(i, a.N, Kl, kStreamDelLD, t, a.h, S.lst, nk);
    if (lane < Kl) ll[(int64_t)i * Kl + lane] = S.lst[lane];
    wave_lds_sync();
  }
  // HD list
  const int id = lane < Kh ? hl[(int64_t)i * Kh + lane] : -1;
  const int nid = id >= 0 ? newid[id] : -1;
  const float od2 = lane < Kh ? hd[(int64_t)i * Kh + lane] : kInf;
  const uint64_t keep = __ballot(nid >= 0);
  const int nk = __popcll(keep);
  const bool remapped = __ballot(lane < Kh && nid != id) != 0ull;
  if (!remapped) return;
  if (nid >= 0) {
    S.lst[popc_below(keep, lane)] = nid;
    S.row[popc_below(keep, lane)] = od2;
  }
  wave_lds_sync();
  if (nk < Kh) random_list(i, a.N, Kh, kStreamDelHD, t, a.h, S.lst, nk);
  const int e = lane < Kh ? S.lst[lane] : -1;
  const float keptd = lane < nk ? S.row[lane] : kInf;
  wave_lds_sync();
  // distances of the refills (lanes nk .. Kh-1), packed to lanes 0 .. Kh-nk-1
  const int fresh = (lane >= nk && lane < Kh) ? e : -1;
  int cid = __shfl(fresh, (lane + nk) & (kWave - 1));
  if (lane >= Kh - nk) cid = -1;
  hd_dist_rows<TX, VEC, CH>(static_cast<const TX*>(a.X), a.D, i, cid, Kh - nk, S.d2);
  const float dd = lane < nk ? keptd : (lane < Kh ? S.d2[(lane - nk) & (kWave - 1)] : kInf);
  int ra, rb;
  rank_two(dd, lane < Kh ? e : kNoId, kInf, kNoId, Kh, 0, S.key, ra, rb);
  if (lane < Kh) {
    hl[(int64_t)i * Kh + ra] = e;
    hd[(int64_t)i * Kh + ra] = dd;
    S.d2[ra] = dd;
  }
  wave_lds_sync();
  if (nk < Kh) {
    const float sorted = lane < Kh ? S.d2[lane] : 0.0f;
    const float4 r = calibrate_row(sorted, Kh, a.h, a.rec[i].x);
    if (lane == 0) {
      a.rec[i] = r;
      a.flags[i] = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static inline unsigned wave_blocks(int64_t n) {
  return (unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock);
}

// Vector width: 16-byte loads when every row starts 16-byte aligned; CH
// bounds the vectors each lane holds (chunks = ceil(D / VEC / 64) when a row
// takes the whole wave).
template <template <typename, int, int> class F, typename TX, int VEC, typename... Args>
static hipError_t dispatch_ch(int D, Args&&... args) {
  const int V = (D + VEC - 1) / VEC;
  const int chunks = V <= 64 ? 1 : (V + 63) / 64;
  if (chunks <= 1) return F<TX, VEC, 1>::run(args...);
  if (chunks <= 4) return F<TX, VEC, 4>::run(args...);
  // 16 chunks: single elements, or FP32 rows up to 4096 wide (BF16 rows stop
  // at 4 chunks of 8, the widest the MFMA screen takes)
  if constexpr (VEC * sizeof(TX) <= 4 || std::is_same<TX, float>::value) {
    if (chunks <= 16) return F<TX, VEC, 16>::run(args...);
  }
  return hipErrorInvalidValue;
}

template <template <typename, int, int> class F, typename... Args>
static hipError_t dispatch_x(const StepArgs& a, Args&&... args) {
  if (a.xdtype == 0) {
    if (a.xvec_ok && a.D % 4 == 0) return dispatch_ch<F, float, 4>(a.D, a, args...);
    return dispatch_ch<F, float, 1>(a.D, a, args...);
  }
  if (a.xvec_ok && a.D % 8 == 0) return dispatch_ch<F, uint16_t, 8>(a.D, a, args...);
  return dispatch_ch<F, uint16_t, 1>(a.D, a, args...);
}

template <typename TX, int VEC, int CH>
struct InitLaunch {
  static hipError_t run(const StepArgs& a, int32_t i0, int32_t n, hipStream_t s) {
    if (a.Kh > kWave)
      hipLaunchKernelGGL((k_init_lists_long<TX, VEC, CH>), dim3(wave_blocks(n)), dim3(kBlock), 0,
                         s, static_cast<const TX*>(a.X), i0 + n, i0, a.D, a.Kh, a.Kl, a.h,
                         a.hd_idx[a.hd_buf_host], a.hd_d2[a.hd_buf_host],
                         a.ld_idx[a.ld_buf_host], a.rec, a.flags);
    else
    hipLaunchKernelGGL((k_init_lists<TX, VEC, CH>), dim3(wave_blocks(n)), dim3(kBlock), 0, s,
                       static_cast<const TX*>(a.X), i0 + n, i0, a.D, a.Kh, a.Kl, a.h,
                       a.hd_idx[a.hd_buf_host], a.hd_d2[a.hd_buf_host], a.ld_idx[a.ld_buf_host],
                       a.rec, a.flags);
    return hipGetLastError();
  }
};

template <typename TX, int VEC, int CH>
struct RefineLaunch {
  static hipError_t run(const StepArgs& a, hipStream_t s) {
    if (a.Kh > kWave)
      hipLaunchKernelGGL((k_hd_refine_long<TX, VEC, CH>), dim3(wave_blocks(a.N)), dim3(kBlock),
                         0, s, a);
    else if (CH == 1 && a.Kh <= 32 && a.Kl <= 32 && a.memo_w == 64)
      hipLaunchKernelGGL((k_hd_refine2<TX, VEC, false, 64>), dim3(wave_blocks((a.N + 1) / 2)),
                         dim3(kBlock), 0, s, a);
    else if (CH == 1 && a.Kh <= 32 && a.Kl <= 32)
      hipLaunchKernelGGL((k_hd_refine2<TX, VEC, false, 32>), dim3(wave_blocks((a.N + 1) / 2)),
                         dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_hd_refine<TX, VEC, CH, false>), dim3(wave_blocks(a.N)),
                         dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
};

// BF16 rows, D % 16 == 0 (checked by the host), 16-byte aligned.
hipError_t launch_hd_refine_bf16(const StepArgs& a, hipStream_t s) {
  if (a.xdtype != 1 || a.D % 16 != 0 || !a.xvec_ok || a.Kh > kWave) return hipErrorInvalidValue;
  const int chunks = (a.D / 8 + 63) / 64;
  if (chunks <= 1 && a.Kh <= 32 && a.Kl <= 32)
    hipLaunchKernelGGL((k_hd_refine2<uint16_t, 8, true, 32>), dim3(wave_blocks((a.N + 1) / 2)),
                       dim3(kBlock), 0, s, a);
  else if (chunks <= 1)
    hipLaunchKernelGGL((k_hd_refine<uint16_t, 8, 1, true>), dim3(wave_blocks(a.N)), dim3(kBlock),
                       0, s, a);
  else if (chunks <= 4)
    hipLaunchKernelGGL((k_hd_refine<uint16_t, 8, 4, true>), dim3(wave_blocks(a.N)), dim3(kBlock),
                       0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename TX, int VEC, int CH>
struct DriftLaunch {
  static hipError_t run(const StepArgs& a, const uint8_t* moved, hipStream_t s) {
    hipLaunchKernelGGL((k_drift_rows<TX, VEC, CH>), dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a,
                       moved);
    return hipGetLastError();
  }
};

template <typename TX, int VEC, int CH>
struct DeleteLaunch {
  static hipError_t run(const StepArgs& a, const int32_t* newid, hipStream_t s) {
    hipLaunchKernelGGL((k_delete_fix<TX, VEC, CH>), dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a,
                       newid);
    return hipGetLastError();
  }
};

hipError_t launch_delete_fix(const StepArgs& a, const int32_t* newid, hipStream_t s) {
  return dispatch_x<DeleteLaunch>(a, newid, s);
}

hipError_t launch_move_rows(void* base, const int32_t* src, const int32_t* dst, int32_t m,
                            int32_t row_bytes, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_move_rows, dim3(1024), dim3(256), 0, s, static_cast<uint8_t*>(base), src,
                     dst, m, row_bytes);
  return hipGetLastError();
}

hipError_t launch_init_lists(const StepArgs& a, int32_t i0, int32_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return dispatch_x<InitLaunch>(a, i0, n, s);
}

hipError_t launch_hd_refine(const StepArgs& a, hipStream_t s) {
  if (a.h.dist_mode == 1) return launch_hd_refine_bf16(a, s);
  return dispatch_x<RefineLaunch>(a, s);
}

hipError_t launch_drift_rows(const StepArgs& a, const uint8_t* moved, hipStream_t s) {
  return dispatch_x<DriftLaunch>(a, moved, s);
}

hipError_t launch_psym(const StepArgs& a, int standalone, hipStream_t s) {
  const int64_t entries = (int64_t)a.N * a.Kh;
  hipLaunchKernelGGL(k_psym, dim3((unsigned)((entries + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, a, standalone);
  return hipGetLastError();
}

hipError_t launch_calibrate_all(const StepArgs& a, hipStream_t s) {
  if (a.Kh > kWave)
    hipLaunchKernelGGL(k_calibrate_all_long, dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_calibrate_all, dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ld_grad(const StepArgs& a, hipStream_t s) {
  const dim3 g(wave_blocks(a.N)), b(kBlock);
  const bool short_list = a.Kl <= 32, long_hd = a.Kh > kWave;
#define FSNE_LD_CASE(DPV)                                                        \
  case DPV:                                                                      \
    if (long_hd)                                                                 \
      hipLaunchKernelGGL((k_ld_grad<DPV, kWave, kMaxLong>), g, b, 0, s, a);      \
    else if (short_list)                                                         \
      hipLaunchKernelGGL((k_ld_grad<DPV, 32>), g, b, 0, s, a);                   \
    else                                                                         \
      hipLaunchKernelGGL((k_ld_grad<DPV, kWave>), g, b, 0, s, a);                \
    break;
  switch (a.DP) {
    FSNE_LD_CASE(2)
    FSNE_LD_CASE(4)
    FSNE_LD_CASE(8)
    FSNE_LD_CASE(16)
    FSNE_LD_CASE(32)
    FSNE_LD_CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef FSNE_LD_CASE
  return hipGetLastError();
}

hipError_t launch_reduce(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_update(const StepArgs& a, hipStream_t s) {
  const int64_t total = (int64_t)a.N * a.DP;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_update, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_set_fire(Scalars* sc, const Hyper& h, hipStream_t s) {
  hipLaunchKernelGGL(k_set_fire, dim3(1), dim3(64), 0, s, sc, h);
  return hipGetLastError();
}

hipError_t launch_scale(float* Y, float* V, int64_t n, float inv, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(1024), dim3(256), 0, s, Y, V, n, inv);
  return hipGetLastError();
}

// Row scatter for drift: dst[ids[k]] <- src[k] (row_bytes each), byte-wise.
__global__ void k_scatter_rows(uint8_t* dst, const uint8_t* src, const int32_t* ids, int32_t n,
                               int32_t row_bytes) {
  const int64_t total = (int64_t)n * row_bytes;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = q / row_bytes, b = q % row_bytes;
    dst[(int64_t)ids[k] * row_bytes + b] = src[q];
  }
}

// Mark moved points and reset their velocity.
__global__ void k_mark_moved(uint8_t* moved, float* V, int32_t DP, const int32_t* ids,
                             int32_t n) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < (int64_t)n * DP;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = q / DP, c = q % DP;
    V[(int64_t)ids[k] * DP + c] = 0.0f;
    if (c == 0) moved[ids[k]] = 1;
  }
}

hipError_t launch_scatter_rows(void* dst, const void* src, const int32_t* ids, int32_t n,
                               int32_t row_bytes, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_rows, dim3(1024), dim3(256), 0, s, static_cast<uint8_t*>(dst),
                     static_cast<const uint8_t*>(src), ids, n, row_bytes);
  return hipGetLastError();
}

hipError_t launch_mark_moved(uint8_t* moved, float* V, int32_t DP, const int32_t* ids, int32_t n,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_moved, dim3(256), dim3(256), 0, s, moved, V, DP, ids, n);
  return hipGetLastError();
}

// Row re-striding between the caller's n x d layout and the padded n x DP one
// (padding written as zero).
__global__ void k_restride(float* dst, int dst_stride, const float* src, int src_stride,
                           int64_t n, int width, int zero_to) {
  const int64_t total = n * (int64_t)zero_to;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q / zero_to;
    const int c = (int)(q % zero_to);
    dst[r * dst_stride + c] = c < width ? src[r * src_stride + c] : 0.0f;
  }
}

hipError_t launch_restride(float* dst, int dst_stride, const float* src, int src_stride,
                           int64_t n, int width, int zero_to, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_restride, dim3(2048), dim3(256), 0, s, dst, dst_stride, src, src_stride,
                     n, width, zero_to);
  return hipGetLastError();
}

}  // namespace fsne
