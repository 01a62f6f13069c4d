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
// cid (negative: skip).  Results go to sd2[0..nrows).
template <typename TX, int VEC>
__device__ void hd_dist_rows(const TX* __restrict__ X, int D, int32_t i, int cid, int nrows,
                             float* sd2) {
  const int lane = lane_id();
  const RowGeom geo = row_geom(D, VEC);
  const int g = lane >> geo.lg, sl = lane & (geo.G - 1);
  const int R = kWave >> geo.lg;
  const TX* xi = X + (int64_t)i * D;
  for (int p = 0; p < nrows; p += R) {
    const int slot = p + g;
    const int c = __shfl(cid, slot & (kWave - 1));
    float acc = 0.0f;
    if (slot < nrows && c >= 0) {
      const TX* xc = X + (int64_t)c * D;
      for (int k = 0; k < geo.chunks; ++k) {
        const int e = (sl + k * geo.G) * VEC;
        if (e < D) {
          float a[VEC], b[VEC];
          VecLoad<TX, VEC>::load(xi + e, a);
          VecLoad<TX, VEC>::load(xc + e, b);
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const float df = a[v] - b[v];
            acc = fmaf(df, df, acc);
          }
        }
      }
    }
    for (int o = geo.G >> 1; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    if (sl == 0 && slot < nrows) sd2[slot] = acc;
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
// if it gives i, an entry of i's own list, or the id of an earlier slot.
// Returns the candidate id in lanes 0..31 (-1: dropped), -1 elsewhere.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int make_candidate(int32_t i, uint32_t t, uint32_t stream,
                                              const Hyper& h, const int32_t* __restrict__ L,
                                              int K, int own, const int32_t* __restrict__ Lx,
                                              int Kx, int other, int32_t N) {
  const int lane = lane_id();
  const int s = lane & (kCand - 1);
  const uint4 u = philox((uint32_t)i, t, stream, (uint32_t)s, h.key0, h.key1);
  const int a_own = (int)draw_index(u.x, (uint32_t)K);
  const int a_oth = (int)draw_index(u.x, (uint32_t)Kx);
  const int j_own = __shfl(own, a_own);
  const int j_oth = __shfl(other, a_oth);
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
  bool ok = lane < kCand && c != i && !in_lanes(c, own, K);
  for (int k = 0; k < kCand; ++k) ok &= !(k < s && c == __builtin_amdgcn_readlane(c, k));
  return ok ? c : -1;
}

// ---------------------------------------------------------------------------
// Initial lists: for point i, the first K distinct other points among the
// draws (i, 0, stream, s), s = 0, 1, ... < 64K, completed if need be by
// i+1, i+2, ... (mod N).  Draws are taken 64 at a time; a draw is a
// duplicate if it repeats an accepted id or an earlier draw of its round.
// The list goes to lst[0..K) (LDS).
// ---------------------------------------------------------------------------
__device__ void random_list(int32_t i, int32_t N, int K, uint32_t stream, const Hyper& h,
                            int* lst) {
  const int lane = lane_id();
  int n = 0;
  for (int base = 0; n < K && base < kWave * K; base += kWave) {
    const uint4 u = philox((uint32_t)i, 0u, stream, (uint32_t)(base + lane), h.key0, h.key1);
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
  float key[2 * kWave];
  int id[2 * kWave];
  float d2[kWave];
  int lst[kWave];
};

template <typename TX, int VEC>
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
  random_list(i, N, Kl, kStreamInitLD, h, S.lst);
  if (lane < Kl) ld_idx[(int64_t)i * Kl + lane] = S.lst[lane];
  wave_lds_sync();
  random_list(i, N, Kh, kStreamInitHD, h, S.lst);
  const int id = lane < Kh ? S.lst[lane] : -1;
  hd_dist_rows<TX, VEC>(X, D, i, id, Kh, S.d2);
  const float dd = lane < Kh ? S.d2[lane] : kInf;
  const int ii = lane < Kh ? id : kNoId;
  int ra, rb;
  rank_two(dd, ii, kInf, kNoId, Kh, 0, S.key, S.id, ra, rb);
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

// ---------------------------------------------------------------------------
// HD refinement of point i (runs when the coin fired): candidates from the
// HD lists and the LD lists of iteration t, their distances, merge into the
// sorted list, flag, and recalibration of beta_i when the list changed.
// ---------------------------------------------------------------------------
template <typename TX, int VEC>
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
  const int c = make_candidate(i, t, kStreamHDC, a.h, hin, Kh, own, lin, Kl, oth, a.N);
  hd_dist_rows<TX, VEC>(static_cast<const TX*>(a.X), a.D, i, c, kCand, S.d2);
  const float cd2 = c >= 0 ? S.d2[lane & (kCand - 1)] : kInf;
  int ro, rc;
  rank_two(lane < Kh ? od2 : kInf, lane < Kh ? own : kNoId, cd2, c >= 0 ? c : kNoId, Kh,
           kCand, S.key, S.id, ro, rc);
  int32_t* hout = a.hd_idx[cur ^ 1];
  float* dout = a.hd_d2[cur ^ 1];
  if (lane < Kh && ro < Kh) {
    hout[(int64_t)i * Kh + ro] = own;
    dout[(int64_t)i * Kh + ro] = od2;
    S.d2[ro] = od2;
  }
  const bool enter = c >= 0 && rc < Kh;
  if (enter) {
    hout[(int64_t)i * Kh + rc] = c;
    dout[(int64_t)i * Kh + rc] = cd2;
    S.d2[rc] = cd2;
  }
  wave_lds_sync();
  const bool changed = __ballot(enter) != 0ull;
  if (lane == 0) a.flags[i] = changed ? 1 : 0;
  if (changed) {
    const float sorted = lane < Kh ? S.d2[lane] : 0.0f;
    const float4 r = calibrate_row(sorted, Kh, a.h, a.rec[i].x);
    if (lane == 0) a.rec[i] = r;
  }
}

// ---------------------------------------------------------------------------
// Symmetrised affinities of point i (eq. (1)) over its HD list:
//   P_ik = (p_{j|i} + p_{i|j}) / (2N), j = HD[i][k],
//   p_{j|i} = exp(-beta_i (d2 - m_i)) invS_i,
//   p_{i|j} = exp(-beta_j (d2 - m_j)) invS_j if i is in j's HD list, else 0.
// standalone = 1: run regardless of the coin, on the current lists.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_psym(StepArgs a, int standalone) {
  const Scalars* sc = a.sc;
  const int fire = standalone ? 0 : sc->fire;
  if (!standalone && !fire) return;
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const int lane = lane_id();
  const int Kh = a.Kh;
  const int buf = sc->hd_cur ^ fire;
  const int32_t* hl = a.hd_idx[buf];
  const float* hd = a.hd_d2[buf];
  if (lane >= Kh) return;
  const int32_t j = hl[(int64_t)i * Kh + lane];
  const float d2 = hd[(int64_t)i * Kh + lane];
  const float4 ri = a.rec[i];
  const float4 rj = a.rec[j];
  const float pji = expf(-ri.x * (d2 - ri.y)) * ri.w;
  // Every stored HD distance comes from the same symmetric FP32 computation,
  // so i can only be in j's sorted list if d2 <= r_j (j's largest distance);
  // the list itself is scanned only then, 16 bytes per load.
  bool member = false;
  if (d2 <= rj.z * (1.0f + 1e-6f)) {
    const int32_t* row = hl + (int64_t)j * Kh;
    if ((Kh & 3) == 0) {
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
  a.P[(int64_t)i * Kh + lane] = (pji + pij) / (2.0f * (float)a.N);
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
template <int DP>
struct LdGeom {
  static constexpr int VEC = DP >= 4 ? 4 : DP;
  static constexpr int G = DP / VEC;
  static constexpr int LG = G == 1 ? 0 : G == 2 ? 1 : G == 4 ? 2 : G == 8 ? 3 : 4;
  static constexpr int RPI = kWave / G;
  static constexpr int MAXE = kWave + kCand;                 // LD entries: old list + slots
  static constexpr int MAXP = (MAXE + RPI - 1) / RPI;         // passes over the entries
  static constexpr bool CACHE = MAXP * VEC <= 48;             // keep entry rows in registers
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

// The LD distance that decides list membership: components summed in index
// order, each square and each sum rounded separately.  The row is split over
// G lanes, so the running sum is handed from lane to lane in component order;
// the last lane of the group ends with the total.
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
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < Geo::G; ++k) {
    const float prev = Geo::G > 1 ? __shfl_up(acc, 1) : 0.0f;
    if (q == k) {
      float s = k == 0 ? 0.0f : prev;
#pragma unroll
      for (int v = 0; v < Geo::VEC; ++v) s = s + sq[v];
      acc = s;
    }
  }
  return acc;
}

// Sum over the G lanes of a row group (every lane of the group gets it).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

struct LdLds {
  int ent[2 * kWave];     // LD entries: old list, then candidate slots (-1: none)
  float dd[2 * kWave];    // their decision distances
  float key[2 * kWave];   // rank scratch
  int id[2 * kWave];
  int newl[kWave];        // new LD list
  int kind[2 * kWave];    // 1: entry kept and not an HD neighbour
  int neg[kWave];         // negative samples outside U (-1: none)
};

// Adds one neighbour's contribution to this lane's components:
//   A += patt w^(1/a) (y_i - y_j),  R += scale w^(1+1/a) (y_i - y_j);
// returns scale * w (the Zh term), with w = (1 + q2/alpha)^(-alpha).
template <int VEC>
__device__ __forceinline__ float pair_terms(const float* yi, const float* yj, float q2,
                                            const Hyper& h, float patt, float scale, float* A,
                                            float* R) {
  const float wa = 1.0f / fmaf(q2, h.inv_alpha, 1.0f);
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

template <int DP>
__global__ __launch_bounds__(kBlock) void k_ld_grad(StepArgs a) {
  using Geo = LdGeom<DP>;
  constexpr int VEC = Geo::VEC, G = Geo::G, RPI = Geo::RPI;
  __shared__ LdLds lds_all[kWavesPerBlock];
  LdLds& S = lds_all[threadIdx.x / kWave];
  const int32_t i = (int32_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave);
  if (i >= a.N) return;
  const Scalars* sc = a.sc;
  const int lane = lane_id();
  const int q = lane & (G - 1);          // chunk of the row this lane holds
  const int rg = lane >> Geo::LG;        // row slot within a pass
  const uint32_t t = sc->t;
  const int hb = sc->hd_cur ^ sc->fire;  // HD lists after this iteration's HD phase
  const int Kh = a.Kh, Kl = a.Kl;
  const int32_t* hl = a.hd_idx[hb];
  const int32_t* lin = a.ld_idx[t & 1];
  int32_t* lout = a.ld_idx[(t & 1) ^ 1];
  const float* Y = a.Y;

  float yi[VEC];
  load_chunk<VEC>(Y + (int64_t)i * DP + q * VEC, yi);
  const int hid = lane < Kh ? hl[(int64_t)i * Kh + lane] : -1;
  const float pk = lane < Kh ? a.P[(int64_t)i * Kh + lane] : 0.0f;
  const int lid = lane < Kl ? lin[(int64_t)i * Kl + lane] : -1;
  const int c = make_candidate(i, t, kStreamLDC, a.h, lin, Kl, lid, hl, Kh, hid, a.N);

  // entry table: old LD list at [0, Kl), candidate slot s at Kl + s
  const int ne = Kl + kCand;
  if (lane < Kl) S.ent[lane] = lid;
  if (lane < kCand) S.ent[Kl + lane] = c;
  wave_lds_sync();

  // decision distances of the entries, rows kept in registers when they fit
  float rows[Geo::CACHE ? Geo::MAXP : 1][VEC];
#pragma unroll
  for (int p = 0; p < Geo::MAXP; ++p) {
    if (p * RPI < ne) {
      const int e = p * RPI + rg;
      const int id = e < ne ? S.ent[e] : -1;
      float yj[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) yj[v] = yi[v];
      if (id >= 0) load_chunk<VEC>(Y + (int64_t)id * DP + q * VEC, yj);
      const float dist = ld_decision_d2<DP>(yi, yj, q);
      if (q == G - 1 && e < ne) S.dd[e] = id >= 0 ? dist : kInf;
      if constexpr (Geo::CACHE) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) rows[p][v] = yj[v];
      }
    }
  }
  wave_lds_sync();

  // merge: rank of every entry by (distance, index); keep the first Kl
  const int eA = lane, eB = kWave + lane;
  const int idA = eA < ne ? S.ent[eA] : -1;
  const int idB = eB < ne ? S.ent[eB] : -1;
  const float dA = idA >= 0 ? S.dd[eA] : kInf;
  const float dB = idB >= 0 ? S.dd[eB] : kInf;
  int rA, rB;
  rank_two(dA, idA >= 0 ? idA : kNoId, dB, idB >= 0 ? idB : kNoId, min(ne, kWave),
           max(ne - kWave, 0), S.key, S.id, rA, rB);
  const bool keepA = idA >= 0 && rA < Kl, keepB = idB >= 0 && rB < Kl;
  if (keepA) {
    lout[(int64_t)i * Kl + rA] = idA;
    S.newl[rA] = idA;
  }
  if (keepB) {
    lout[(int64_t)i * Kl + rB] = idB;
    S.newl[rB] = idB;
  }

  // negatives: uniform other points, one per lane
  const bool has_neg = lane < a.h.n_neg;
  int jn = -1;
  if (has_neg) {
    const uint4 u = philox((uint32_t)i, t, kStreamNeg, (uint32_t)lane, a.h.key0, a.h.key1);
    jn = draw_other(u.x, i, a.N);
  }
  bool a_hd = false, b_hd = false, n_in = false;
  for (int k = 0; k < Kh; ++k) {
    const int v = __builtin_amdgcn_readlane(hid, k);
    a_hd |= (idA == v);
    b_hd |= (idB == v);
    n_in |= (jn == v);
  }
  wave_lds_sync();
  for (int k = 0; k < Kl; ++k) n_in |= (jn == S.newl[k]);
  if (eA < ne) S.kind[eA] = (keepA && !a_hd) ? 1 : 0;
  if (eB < ne) S.kind[eB] = (keepB && !b_hd) ? 1 : 0;
  S.neg[lane] = (has_neg && !n_in) ? jn : -1;
  wave_lds_sync();

  float A[VEC], R[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) A[v] = R[v] = 0.0f;
  float zh = 0.0f;
  // HD neighbours: attraction and repulsion
  for (int b = 0; b < Kh; b += RPI) {
    const int r = b + rg;
    const int id = __shfl(hid, r & (kWave - 1));
    const float pr = __shfl(pk, r & (kWave - 1));
    float yj[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) yj[v] = yi[v];
    if (r < Kh) load_chunk<VEC>(Y + (int64_t)id * DP + q * VEC, yj);
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
  // LD neighbours that are not HD neighbours: repulsion
#pragma unroll
  for (int p = 0; p < Geo::MAXP; ++p) {
    if (p * RPI < ne) {
      const int e = p * RPI + rg;
      if (e < ne && S.kind[e]) {
        float yj[VEC];
        if constexpr (Geo::CACHE) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) yj[v] = rows[p][v];
        } else {
          load_chunk<VEC>(Y + (int64_t)S.ent[e] * DP + q * VEC, yj);
        }
        const float z = pair_terms<VEC>(yi, yj, S.dd[e], a.h, 0.0f, 1.0f, A, R);
        if (q == 0) zh += z;
      }
    }
  }
  // negative samples outside U, weighted (N-1)/n_neg
  for (int b = 0; b < a.h.n_neg; b += RPI) {
    const int r = b + rg;
    const int id = r < a.h.n_neg ? S.neg[r] : -1;
    float yj[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) yj[v] = yi[v];
    if (id >= 0) load_chunk<VEC>(Y + (int64_t)id * DP + q * VEC, yj);
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
  for (int o = G; o < kWave; o <<= 1) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      A[v] += __shfl_xor(A[v], o);
      R[v] += __shfl_xor(R[v], o);
    }
  }
  zh = wave_sum(zh);
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
  const int fire = a.sc->fire;
  const int64_t N = a.N;
  const int64_t chunk = (N + kReduceBlocks - 1) / kReduceBlocks;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < N ? lo + chunk : N;
  float z = 0.0f;
  int f = 0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) {
    z += a.Zh[k];
    if (fire) f += a.flags[k];
  }
  sz[threadIdx.x] = z;
  sf[threadIdx.x] = f;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sz[threadIdx.x] += sz[threadIdx.x + o];
      sf[threadIdx.x] += sf[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.zpart[blockIdx.x] = sz[0];
    a.fpart[blockIdx.x] = sf[0];
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
    const int fire = sc->fire;
    int f = 0;
    if (fire)
      for (int k = threadIdx.x; k < kReduceBlocks; k += 256) f += a.fpart[k];
    sf[threadIdx.x] = f;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
      if ((int)threadIdx.x < o) sf[threadIdx.x] += sf[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const uint32_t t1 = sc->t + 1u;
      float E = sc->E;
      if (fire) {
        sc->n_new = sf[0];
        E = E_next(E, sf[0], a.N, a.h.e_smooth);
        sc->hd_cur ^= 1;
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

// ---------------------------------------------------------------------------
// Drift: recompute every HD entry that pairs with a moved point (moved[] is
// a per-point byte map), re-sort those rows, flag and recalibrate them.
// ---------------------------------------------------------------------------
template <typename TX, int VEC>
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
  hd_dist_rows<TX, VEC>(static_cast<const TX*>(a.X), a.D, i, redo ? id : -1, Kh, S.d2);
  const float dd = lane < Kh ? (redo ? S.d2[lane] : old) : kInf;
  int ra, rb;
  rank_two(dd, lane < Kh ? id : kNoId, kInf, kNoId, Kh, 0, S.key, S.id, ra, rb);
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
// Launchers.
// ---------------------------------------------------------------------------
static inline unsigned wave_blocks(int64_t n) {
  return (unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock);
}

// Vector width: 16-byte loads when every row starts 16-byte aligned.
template <template <typename, int> class F, typename... Args>
static hipError_t dispatch_x(const StepArgs& a, Args&&... args) {
  if (a.xdtype == 0) {
    if (a.xvec_ok && a.D % 4 == 0) return F<float, 4>::run(a, args...);
    return F<float, 1>::run(a, args...);
  }
  if (a.xvec_ok && a.D % 8 == 0) return F<uint16_t, 8>::run(a, args...);
  return F<uint16_t, 1>::run(a, args...);
}

template <typename TX, int VEC>
struct InitLaunch {
  static hipError_t run(const StepArgs& a, int32_t i0, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_init_lists<TX, VEC>), dim3(wave_blocks(n)), dim3(kBlock), 0, s,
                       static_cast<const TX*>(a.X), i0 + n, i0, a.D, a.Kh, a.Kl, a.h,
                       a.hd_idx[a.hd_buf_host], a.hd_d2[a.hd_buf_host], a.ld_idx[a.ld_buf_host],
                       a.rec, a.flags);
    return hipGetLastError();
  }
};

template <typename TX, int VEC>
struct RefineLaunch {
  static hipError_t run(const StepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_hd_refine<TX, VEC>), dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
};

template <typename TX, int VEC>
struct DriftLaunch {
  static hipError_t run(const StepArgs& a, const uint8_t* moved, hipStream_t s) {
    hipLaunchKernelGGL((k_drift_rows<TX, VEC>), dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a,
                       moved);
    return hipGetLastError();
  }
};

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
  hipLaunchKernelGGL(k_psym, dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a, standalone);
  return hipGetLastError();
}

hipError_t launch_calibrate_all(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_calibrate_all, dim3(wave_blocks(a.N)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ld_grad(const StepArgs& a, hipStream_t s) {
  const dim3 g(wave_blocks(a.N)), b(kBlock);
  switch (a.DP) {
    case 2: hipLaunchKernelGGL((k_ld_grad<2>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_ld_grad<4>), g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_ld_grad<8>), g, b, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_ld_grad<16>), g, b, 0, s, a); break;
    case 32: hipLaunchKernelGGL((k_ld_grad<32>), g, b, 0, s, a); break;
    case 64: hipLaunchKernelGGL((k_ld_grad<64>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
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
