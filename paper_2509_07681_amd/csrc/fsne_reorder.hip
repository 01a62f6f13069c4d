// Renumbering of the points for memory locality.  Every candidate, neighbour
// and negative row the step reads is a gather at a random position; when the
// points that are near one another in the data also have nearby ids, the
// rows a block gathers come from a small region and hit in the caches.
//
// fsne_renumber applies a caller's permutation: every per-point row moves to
// its new id and every list entry is mapped.  fsne_reorder picks the
// permutation itself, as the Morton (Z-order) curve over a projection of the
// embedding onto at most three axes: points close in the embedding, which
// the method makes close in the data, get nearby ids (a stable sort of the
// Morton keys: equal keys keep the order of the current ids).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fsne_context.h"

namespace {

// dst row new_of_old[i] = src row i, i < n (4-byte words when the row allows).
__global__ void k_permute_rows(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src,
                               const int32_t* __restrict__ new_of_old, int32_t n,
                               int32_t row_bytes) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if ((row_bytes & 3) == 0) {
    const int32_t w = row_bytes >> 2;
    const int64_t total = (int64_t)n * w;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
      const int64_t i = q / w, k = q - i * w;
      reinterpret_cast<uint32_t*>(dst)[(int64_t)new_of_old[i] * w + k] =
          reinterpret_cast<const uint32_t*>(src)[q];
    }
  } else {
    const int64_t total = (int64_t)n * row_bytes;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
      const int64_t i = q / row_bytes, k = q - i * row_bytes;
      dst[(int64_t)new_of_old[i] * row_bytes + k] = src[q];
    }
  }
}

// ids[e] = new_of_old[ids[e]], e < count (every entry is a live id).
__global__ void k_map_ids(int32_t* __restrict__ ids, const int32_t* __restrict__ new_of_old,
                          int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    ids[e] = new_of_old[ids[e]];
}

constexpr int kMaxAxes = 3;
constexpr int kRedBlocks = 1024;

// Coordinate a (< axes) of the projection of y: y itself when d <= 3,
// otherwise the coordinates c = a, a + 3, a + 6, ... summed with alternating
// signs (a fixed +-1 projection onto three axes).
struct Projection {
  int d, axes;
  __device__ float operator()(const float* y, int a) const {
    if (d <= kMaxAxes) return y[a];
    float s = 0.0f;
    for (int c = a, k = 0; c < d; c += kMaxAxes, ++k) s += (k & 1) ? -y[c] : y[c];
    return s;
  }
};

// Per-block minimum and maximum of each projected axis.
__global__ void k_proj_range(const float* __restrict__ Y, int32_t n, int DP, Projection pr,
                             float* __restrict__ part) {
  __shared__ float lo[kMaxAxes][256], hi[kMaxAxes][256];
  float l[kMaxAxes], h[kMaxAxes];
  for (int a = 0; a < kMaxAxes; ++a) {
    l[a] = INFINITY;
    h[a] = -INFINITY;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int a = 0; a < pr.axes; ++a) {
      const float v = pr(Y + i * DP, a);
      l[a] = fminf(l[a], v);
      h[a] = fmaxf(h[a], v);
    }
  }
  for (int a = 0; a < kMaxAxes; ++a) {
    lo[a][threadIdx.x] = l[a];
    hi[a][threadIdx.x] = h[a];
  }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < kMaxAxes; ++a) {
        lo[a][threadIdx.x] = fminf(lo[a][threadIdx.x], lo[a][threadIdx.x + s]);
        hi[a][threadIdx.x] = fmaxf(hi[a][threadIdx.x], hi[a][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < kMaxAxes; ++a) {
      part[blockIdx.x * 2 * kMaxAxes + 2 * a] = lo[a][0];
      part[blockIdx.x * 2 * kMaxAxes + 2 * a + 1] = hi[a][0];
    }
}

// Spread the low 10 (3 axes), 15 (2 axes) or 30 (1 axis) bits of v so that
// the axes interleave.
__device__ __forceinline__ uint32_t spread(uint32_t v, int axes) {
  if (axes == 1) return v;
  uint32_t r = 0;
  const int bits = 30 / axes;
  for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1u) << (b * axes);
  return r;
}

// Morton key of point i from its projected coordinates scaled to the range.
__global__ void k_morton(const float* __restrict__ Y, int32_t n, int DP, Projection pr,
                         const float* __restrict__ range, uint32_t* __restrict__ keys,
                         int32_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bits = 30 / pr.axes;
  const float top = (float)((1u << bits) - 1u);
  uint32_t key = 0;
  for (int a = 0; a < pr.axes; ++a) {
    const float lo = range[2 * a], hi = range[2 * a + 1];
    const float t = hi > lo ? (pr(Y + i * DP, a) - lo) / (hi - lo) : 0.0f;
    const uint32_t q = (uint32_t)fminf(fmaxf(t * top, 0.0f), top);
    key |= spread(q, pr.axes) << a;
  }
  keys[i] = key;
  ids[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// Stable least-significant-digit radix sort of (key, id) pairs by 8-bit
// digits (four passes cover the 30-bit keys).  A block owns a tile of
// kSortItems rounds of 256 consecutive elements.  Per pass: every block counts
// its digits into a digit-major table; one block per digit turns its row
// into exclusive offsets and sums the digit's total; every block scatters
// its tile in element order (digit d of block b starts after every smaller
// digit, from a scan of the totals, and after digit d of the blocks before
// b), each element at its digit's offset plus the number of equal digits
// before it in the tile (found with ballots within a wave, per-wave counts
// across the waves of a round, running counts across rounds).  Equal keys
// keep their order, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;   // = number of digit values
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortWaves = kSortThreads / 64;

__global__ __launch_bounds__(kSortThreads) void k_digit_count(const uint32_t* __restrict__ keys,
                                                              int32_t n, int shift,
                                                              uint32_t* __restrict__ count) {
  __shared__ uint32_t c[kSortThreads];
  c[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&c[(keys[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  count[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = c[threadIdx.x];
}

// Inclusive prefix sum of part[0..kSortThreads) in LDS by the whole block
// (log2 steps, each read, barrier, add, barrier).
__device__ __forceinline__ void block_inclusive_scan(uint32_t* part) {
  const int tid = threadIdx.x;
  for (int off = 1; off < kSortThreads; off <<= 1) {
    const uint32_t u = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += u;
    __syncthreads();
  }
}

// One block per digit d: row d of the count table (the nb per-block counts
// of digit d) becomes its exclusive prefix sums, and total[d] its sum.  Rows
// are contiguous, so every load and store is coalesced.
__global__ __launch_bounds__(kSortThreads) void k_digit_row_scan(uint32_t* __restrict__ count,
                                                                 int32_t nb,
                                                                 uint32_t* __restrict__ total) {
  __shared__ uint32_t part[kSortThreads];
  uint32_t* row = count + (int64_t)blockIdx.x * nb;
  const int tid = threadIdx.x;
  uint32_t carry = 0u;
  for (int32_t t0 = 0; t0 < nb; t0 += kSortThreads) {
    const int32_t k = t0 + tid;
    const uint32_t v = k < nb ? row[k] : 0u;
    part[tid] = v;
    __syncthreads();
    block_inclusive_scan(part);
    if (k < nb) row[k] = carry + part[tid] - v;
    carry += part[kSortThreads - 1];
    __syncthreads();
  }
  if (tid == 0) total[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(
    const uint32_t* __restrict__ keys, const int32_t* __restrict__ ids, int32_t n, int shift,
    const uint32_t* __restrict__ offset, const uint32_t* __restrict__ total,
    uint32_t* __restrict__ keys_out, int32_t* __restrict__ ids_out) {
  __shared__ uint32_t run[kSortThreads];             // next position of each digit
  __shared__ uint32_t wcount[kSortWaves][kSortThreads];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  // digit tid starts after every smaller digit (exclusive scan of the
  // totals) and after digit tid of the blocks before this one
  const uint32_t own = total[tid];
  run[tid] = own;
  __syncthreads();
  block_inclusive_scan(run);
  run[tid] = run[tid] - own + offset[(int64_t)tid * gridDim.x + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    const bool ok = i < n;
    const uint32_t k = ok ? keys[i] : 0u;
    const int32_t v = ok ? ids[i] : 0;
    const uint32_t dg = (k >> shift) & 0xFFu;
    // lanes of this wave whose element has the same digit
    uint64_t same = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = ((dg >> b) & 1u) != 0u;
      const uint64_t m = __ballot(ok && bit);
      same &= bit ? m : ~m;
    }
    const uint32_t below = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    for (int q = 0; q < kSortWaves; ++q) wcount[q][tid] = 0u;
    __syncthreads();
    if (ok && below == 0u) wcount[w][dg] = (uint32_t)__popcll(same);
    __syncthreads();
    uint32_t pos = 0u;
    if (ok) {
      pos = run[dg] + below;
      for (int q = 0; q < w; ++q) pos += wcount[q][dg];
    }
    __syncthreads();
    uint32_t add = 0u;
    for (int q = 0; q < kSortWaves; ++q) add += wcount[q][tid];
    run[tid] += add;
    if (ok) {
      keys_out[pos] = k;
      ids_out[pos] = v;
    }
    __syncthreads();
  }
}

// Words of the count table and digit totals for n elements.
size_t sort_count_words(int32_t n) {
  return (size_t)kSortThreads * (size_t)((n + kSortTile - 1) / kSortTile) + kSortThreads;
}

// Sorts (keys, ids) by the low `bits` bits of the keys (bits <= 32, even
// number of passes: the result ends in keys / ids; tmp_* are the other
// buffers of the ping-pong, count holds sort_count_words(n) words).
hipError_t radix_sort_pairs(uint32_t* keys, int32_t* ids, uint32_t* tmp_keys, int32_t* tmp_ids,
                            uint32_t* count, int32_t n, int bits, hipStream_t s) {
  const unsigned nb = (unsigned)((n + kSortTile - 1) / kSortTile);
  uint32_t* total = count + (size_t)kSortThreads * nb;
  int passes = (bits + 7) / 8;
  passes += passes & 1;
  uint32_t *ka = keys, *kb = tmp_keys;
  int32_t *ia = ids, *ib = tmp_ids;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_digit_count, dim3(nb), dim3(kSortThreads), 0, s, ka, n, shift, count);
    hipLaunchKernelGGL(k_digit_row_scan, dim3(kSortThreads), dim3(kSortThreads), 0, s, count,
                       (int32_t)nb, total);
    hipLaunchKernelGGL(k_digit_scatter, dim3(nb), dim3(kSortThreads), 0, s, ka, ia, n, shift,
                       count, total, kb, ib);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(ka, kb);
    std::swap(ia, ib);
  }
  return hipSuccess;
}

// new_of_old[old_of_new[k]] = k.
__global__ void k_invert(const int32_t* __restrict__ old_of_new, int32_t n,
                         int32_t* __restrict__ new_of_old) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) new_of_old[old_of_new[k]] = (int32_t)k;
}

unsigned grid_for(int64_t work) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 65536));
}

// The renumbering's device workspace, kept by the context between calls (a
// call that needs more replaces it) and freed with the context, so that a
// renumbering allocates nothing once the first one has run.
hipError_t workspace(fsne_ctx* c, size_t bytes, uint8_t** out) {
  if (c->rwork_bytes < bytes) {
    if (c->rwork) {
      const auto it = std::find(c->owned.begin(), c->owned.end(), (void*)c->rwork);
      if (it != c->owned.end()) c->owned.erase(it);
      (void)hipFree(c->rwork);
      c->rwork = nullptr;
      c->rwork_bytes = 0;
    }
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return e;
    c->owned.push_back(q);
    c->rwork = static_cast<uint8_t*>(q);
    c->rwork_bytes = bytes;
  }
  *out = c->rwork;
  return hipSuccess;
}

constexpr size_t align_up(size_t b) { return (b + 255) & ~(size_t)255; }

struct RowArray {
  void* base;
  size_t bytes;
};

// Per-point arrays a renumbering moves (null ones are skipped), and the
// largest of them in bytes for N points.
std::vector<RowArray> row_arrays(fsne_ctx* c, const fsne::Scalars& sc, size_t* most) {
  const size_t xb = c->xdtype == FSNE_F32 ? 4 : 2;
  std::vector<RowArray> rows = {
      {c->X, (size_t)c->D * xb},
      {c->Xu, sizeof(float) * c->D},
      {c->xnorm, sizeof(float)},
      {c->Y, sizeof(float) * c->DP},
      {c->V, sizeof(float) * c->DP},
      {c->A, sizeof(float) * c->DP},
      {c->R, sizeof(float) * c->DP},
      {c->Zh, sizeof(float)},
      {c->rec, sizeof(float4)},
      {c->P, sizeof(float) * c->Kh},
      {c->flags, 1},
      {c->ldc, 1},
      {c->hd_idx[sc.hd_cur], sizeof(int32_t) * c->Kh},
      {c->hd_d2[sc.hd_cur], sizeof(float) * c->Kh},
      {c->ld_idx[sc.t & 1u], sizeof(int32_t) * c->Kl},
  };
  *most = 0;
  for (const RowArray& r : rows)
    if (r.base) *most = std::max(*most, r.bytes * (size_t)c->N);
  return rows;
}

fsne_status read_scalars(fsne_ctx* c, fsne::Scalars* sc) {
  hipError_t e = hipMemcpyAsync(sc, c->sc, sizeof(*sc), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("fsne_renumber: scalars: ") + hipGetErrorString(e);
    return FSNE_EHIP;
  }
  return FSNE_OK;
}

fsne_status hip_error(fsne_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? FSNE_ENOMEM : FSNE_EHIP;
}

// Move every per-point row to its new id and map the list entries; d_new is
// a device permutation of 0..N-1 and buf a staging area of the size
// row_arrays reports.  The remembered rejections are cleared.
fsne_status apply_permutation(fsne_ctx* c, const fsne::Scalars& sc, const int32_t* d_new,
                              uint8_t* buf) {
  hipStream_t s = c->stream;
  const int32_t N = (int32_t)c->N;
  size_t most = 0;
  const std::vector<RowArray> rows = row_arrays(c, sc, &most);
  hipError_t e;
  for (const RowArray& r : rows) {
    if (!r.base) continue;
    hipLaunchKernelGGL(k_permute_rows, dim3(grid_for((int64_t)N * r.bytes / 4 + 1)), dim3(256),
                       0, s, buf, static_cast<const uint8_t*>(r.base), d_new, N,
                       (int32_t)r.bytes);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(r.base, buf, r.bytes * (size_t)N, hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
      return hip_error(c, e, "fsne_renumber: rows");
  }
  for (int32_t* ids : {c->hd_idx[sc.hd_cur], c->ld_idx[sc.t & 1u]}) {
    const int64_t count = (int64_t)N * (ids == c->hd_idx[sc.hd_cur] ? c->Kh : c->Kl);
    hipLaunchKernelGGL(k_map_ids, dim3(grid_for(count)), dim3(256), 0, s, ids, d_new, count);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(c, e, "fsne_renumber: lists");
  }
  if ((e = hipMemsetAsync(c->memo, 0xFF, sizeof(int32_t) * (size_t)c->cap * fsne::kMemo, s)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_error(c, e, "fsne_renumber");
  return FSNE_OK;
}

}  // namespace

extern "C" fsne_status fsne_renumber(fsne_ctx* c, const int32_t* new_of_old) {
  if (!c) return FSNE_EINVAL;
  if (!new_of_old) {
    c->err = "fsne_renumber: new_of_old is NULL";
    return FSNE_EINVAL;
  }
  if (!c->own_X) {
    c->err = "fsne_renumber: X is borrowed; create the context with capacity";
    return FSNE_ESTATE;
  }
  const int32_t N = (int32_t)c->N;
  std::vector<uint8_t> seen((size_t)N, 0);
  for (int32_t i = 0; i < N; ++i) {
    const int32_t v = new_of_old[i];
    if (v < 0 || v >= N || seen[(size_t)v]) {
      c->err = "fsne_renumber: new_of_old is not a permutation of 0..N-1";
      return FSNE_EINVAL;
    }
    seen[(size_t)v] = 1;
  }
  fsne::Scalars sc;
  fsne_status st = read_scalars(c, &sc);
  if (st != FSNE_OK) return st;
  size_t most = 0;
  (void)row_arrays(c, sc, &most);
  const size_t o_new = 0, o_buf = align_up(sizeof(int32_t) * (size_t)N);
  uint8_t* w = nullptr;
  hipError_t e;
  if ((e = workspace(c, o_buf + most, &w)) != hipSuccess)
    return hip_error(c, e, "fsne_renumber: workspace");
  int32_t* d_new = reinterpret_cast<int32_t*>(w + o_new);
  if ((e = hipMemcpyAsync(d_new, new_of_old, sizeof(int32_t) * (size_t)N,
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return hip_error(c, e, "fsne_renumber: upload");
  return apply_permutation(c, sc, d_new, w + o_buf);
}

namespace {

// Signs r_ka = +-1 of the fixed projection of the data rows: bit 0 of the
// first word of Philox block (k, a, 12, 0) under the context's seed.
__global__ void k_projection_signs(float* __restrict__ sign, int D, uint32_t key0,
                                   uint32_t key1) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= D * kMaxAxes) return;
  const uint4 u = fsne::philox((uint32_t)(q / kMaxAxes), (uint32_t)(q % kMaxAxes),
                               fsne::kStreamOrder, 0u, key0, key1);
  sign[q] = (u.x & 1u) ? -1.0f : 1.0f;
}

// coords[i] = (sum_k x_ik r_k0, sum_k x_ik r_k1, sum_k x_ik r_k2, 0): one wave
// per row, lanes along the row.
template <typename TX>
__global__ __launch_bounds__(256) void k_project_rows(const TX* __restrict__ X, int D, int32_t n,
                                                      const float* __restrict__ sign,
                                                      float4* __restrict__ coords) {
  const int32_t i = (int32_t)(blockIdx.x * 4 + threadIdx.x / 64);
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  float p[kMaxAxes] = {0.0f, 0.0f, 0.0f};
  const TX* row = X + (int64_t)i * D;
  for (int k = lane; k < D; k += 64) {
    const float x = fsne::to_unit_f32(row[k]);
#pragma unroll
    for (int a = 0; a < kMaxAxes; ++a) p[a] = fmaf(x, sign[k * kMaxAxes + a], p[a]);
  }
#pragma unroll
  for (int a = 0; a < kMaxAxes; ++a) p[a] = fsne::wave_sum_uniform(p[a]);
  if (lane == 0) coords[i] = make_float4(p[0], p[1], p[2], 0.0f);
}

// Renumber along the Morton curve of `coords` (row stride `stride` floats)
// projected by pr; the workspace holds `extra` bytes at its start for the
// caller (the coordinates, when they are not the embedding).
fsne_status reorder_along(fsne_ctx* c, const fsne::Scalars& sc, const float* coords, int stride,
                          Projection pr, uint8_t* w, size_t o_base, int32_t* new_of_old,
                          const char* who) {
  const int32_t N = (int32_t)c->N;
  hipStream_t s = c->stream;
  size_t most = 0;
  (void)row_arrays(c, sc, &most);
  hipError_t e;
  const size_t sort_bytes = sizeof(uint32_t) * sort_count_words(N);
  const size_t n4 = align_up(sizeof(int32_t) * (size_t)N);
  const size_t o_part = o_base, o_range = o_part + align_up(sizeof(float) * kRedBlocks * 2 * kMaxAxes);
  const size_t o_keys = o_range + align_up(sizeof(float) * 2 * kMaxAxes);
  const size_t o_keys2 = o_keys + n4, o_ids = o_keys2 + n4, o_ids2 = o_ids + n4;
  const size_t o_new = o_ids2 + n4, o_sort = o_new + n4;
  const size_t o_buf = o_sort + align_up(sort_bytes);
  float* part = reinterpret_cast<float*>(w + o_part);
  float* range = reinterpret_cast<float*>(w + o_range);
  uint32_t* keys = reinterpret_cast<uint32_t*>(w + o_keys);
  uint32_t* keys2 = reinterpret_cast<uint32_t*>(w + o_keys2);
  int32_t* ids = reinterpret_cast<int32_t*>(w + o_ids);
  int32_t* ids2 = reinterpret_cast<int32_t*>(w + o_ids2);
  int32_t* d_new = reinterpret_cast<int32_t*>(w + o_new);
  uint32_t* sort_count = reinterpret_cast<uint32_t*>(w + o_sort);
  (void)most;
  hipLaunchKernelGGL(k_proj_range, dim3(kRedBlocks), dim3(256), 0, s, coords, N, stride, pr, part);
  std::vector<float> hp((size_t)kRedBlocks * 2 * kMaxAxes);
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = hipMemcpyAsync(hp.data(), part, sizeof(float) * hp.size(), hipMemcpyDeviceToHost,
                          s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_error(c, e, who);
  float rg[2 * kMaxAxes] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int a = 0; a < pr.axes; ++a) {
    rg[2 * a] = INFINITY;
    rg[2 * a + 1] = -INFINITY;
    for (int b = 0; b < kRedBlocks; ++b) {
      rg[2 * a] = std::min(rg[2 * a], hp[(size_t)b * 2 * kMaxAxes + 2 * a]);
      rg[2 * a + 1] = std::max(rg[2 * a + 1], hp[(size_t)b * 2 * kMaxAxes + 2 * a + 1]);
    }
    if (!std::isfinite(rg[2 * a]) || !std::isfinite(rg[2 * a + 1])) {
      c->err = std::string(who) + ": the coordinates hold a NaN or infinity";
      return FSNE_ENONFINITE;
    }
  }
  const unsigned gn = (unsigned)((N + 255) / 256);
  if ((e = hipMemcpyAsync(range, rg, sizeof(rg), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(c, e, who);
  hipLaunchKernelGGL(k_morton, dim3(gn), dim3(256), 0, s, coords, N, stride, pr, range, keys, ids);
  if ((e = hipGetLastError()) != hipSuccess ||
      (e = radix_sort_pairs(keys, ids, keys2, ids2, sort_count, N, 30, s)) != hipSuccess)
    return hip_error(c, e, who);
  hipLaunchKernelGGL(k_invert, dim3(gn), dim3(256), 0, s, ids, N, d_new);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(c, e, who);
  fsne_status st = apply_permutation(c, sc, d_new, w + o_buf);
  if (st != FSNE_OK) return st;
  if (new_of_old &&
      ((e = hipMemcpy(new_of_old, d_new, sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToHost)) !=
       hipSuccess))
    return hip_error(c, e, who);
  return FSNE_OK;
}

// Workspace bytes reorder_along needs after its first `o_base` bytes.
size_t reorder_bytes(fsne_ctx* c, const fsne::Scalars& sc) {
  const int32_t N = (int32_t)c->N;
  size_t most = 0;
  (void)row_arrays(c, sc, &most);
  const size_t n4 = align_up(sizeof(int32_t) * (size_t)N);
  return align_up(sizeof(float) * kRedBlocks * 2 * kMaxAxes) +
         align_up(sizeof(float) * 2 * kMaxAxes) + 5 * n4 +
         align_up(sizeof(uint32_t) * sort_count_words(N)) +
         most;
}

}  // namespace

extern "C" fsne_status fsne_reorder(fsne_ctx* c, int32_t* new_of_old) {
  if (!c) return FSNE_EINVAL;
  if (!c->own_X) {
    c->err = "fsne_reorder: X is borrowed; create the context with capacity";
    return FSNE_ESTATE;
  }
  fsne::Scalars sc;
  fsne_status st = read_scalars(c, &sc);
  if (st != FSNE_OK) return st;
  uint8_t* w = nullptr;
  hipError_t e;
  if ((e = workspace(c, reorder_bytes(c, sc), &w)) != hipSuccess)
    return hip_error(c, e, "fsne_reorder: workspace");
  return reorder_along(c, sc, c->Y, c->DP, Projection{c->d, std::min(c->d, kMaxAxes)}, w, 0,
                       new_of_old, "fsne_reorder");
}

extern "C" fsne_status fsne_reorder_data(fsne_ctx* c, int32_t* new_of_old) {
  if (!c) return FSNE_EINVAL;
  if (!c->own_X) {
    c->err = "fsne_reorder_data: X is borrowed; create the context with capacity";
    return FSNE_ESTATE;
  }
  fsne::Scalars sc;
  fsne_status st = read_scalars(c, &sc);
  if (st != FSNE_OK) return st;
  const int32_t N = (int32_t)c->N;
  hipStream_t s = c->stream;
  const size_t o_sign = 0, o_coords = align_up(sizeof(float) * (size_t)c->D * kMaxAxes);
  const size_t o_base = o_coords + align_up(sizeof(float4) * (size_t)N);
  uint8_t* w = nullptr;
  hipError_t e;
  if ((e = workspace(c, o_base + reorder_bytes(c, sc), &w)) != hipSuccess)
    return hip_error(c, e, "fsne_reorder_data: workspace");
  float* sign = reinterpret_cast<float*>(w + o_sign);
  float4* coords = reinterpret_cast<float4*>(w + o_coords);
  hipLaunchKernelGGL(k_projection_signs, dim3((unsigned)((c->D * kMaxAxes + 255) / 256)),
                     dim3(256), 0, s, sign, c->D, (uint32_t)c->seed, (uint32_t)(c->seed >> 32));
  const dim3 g((unsigned)((N + 3) / 4));
  // under the angular metric the rows scaled to unit length are the data
  if (c->hp.metric == 1 && c->Xu)
    hipLaunchKernelGGL(k_project_rows<float>, g, dim3(256), 0, s, c->Xu, c->D, N, sign, coords);
  else if (c->xdtype == FSNE_F32)
    hipLaunchKernelGGL(k_project_rows<float>, g, dim3(256), 0, s,
                       static_cast<const float*>(c->X), c->D, N, sign, coords);
  else
    hipLaunchKernelGGL(k_project_rows<uint16_t>, g, dim3(256), 0, s,
                       static_cast<const uint16_t*>(c->X), c->D, N, sign, coords);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(c, e, "fsne_reorder_data: project");
  return reorder_along(c, sc, reinterpret_cast<const float*>(coords), 4,
                       Projection{kMaxAxes, kMaxAxes}, w, o_base, new_of_old, "fsne_reorder_data");
}
