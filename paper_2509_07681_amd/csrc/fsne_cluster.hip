// Clustering of the embedding for the hierarchy graph of Sec. 4.2: DBSCAN
// (Ester, Kriegel, Sander, Xu 1996) with each point's eps-neighbourhood
// taken from its LD neighbour list, which the iteration keeps up to date:
//   N(i)  = {i} + {j in LD list of i : |y_i - y_j|^2 <= eps^2}
//   core  : |N(i)| >= min_pts
//   clusters: connected components of the core points, two core points
//             being linked when either lies in the other's N;
//   border: a non-core point within eps of a core point (in either list)
//           joins the cluster of the nearest such core point (ties: the
//           smaller cluster label); every other point is noise (-1).
// Squared distances are summed over the components in index order in FP32
// without fused multiply-add.  Components are found by min-label hooking
// with pointer jumping (atomicMin), so the result does not depend on
// scheduling; clusters are numbered by the smallest index among their core
// points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>

#include "fsne_context.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float pair_d2(const float* Y, int DP, int d, int32_t i, int32_t j) {
#pragma clang fp contract(off)
  float s = 0.0f;
  for (int c = 0; c < d; ++c) {
    const float df = Y[(int64_t)j * DP + c] - Y[(int64_t)i * DP + c];
    s = s + df * df;
  }
  return s;
}

__global__ void k_cl_core(const float* Y, int DP, int d, const int32_t* ld, int K, int32_t N,
                          float eps2, int min_pts, uint8_t* core, int32_t* label) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= N) return;
  int cnt = 1;
  for (int k = 0; k < K; ++k) cnt += pair_d2(Y, DP, d, i, ld[(int64_t)i * K + k]) <= eps2;
  const bool c = cnt >= min_pts;
  core[i] = c ? 1 : 0;
  label[i] = c ? i : INT_MAX;
}

// One round of hooking: linked core points lower each other's label.
__global__ void k_cl_hook(const float* Y, int DP, int d, const int32_t* ld, int K, int32_t N,
                          float eps2, const uint8_t* core, int32_t* label, int32_t* changed) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= N || !core[i]) return;
  for (int k = 0; k < K; ++k) {
    const int32_t j = ld[(int64_t)i * K + k];
    if (!core[j] || pair_d2(Y, DP, d, i, j) > eps2) continue;
    const int32_t a = label[i], b = label[j];
    if (a < b) {
      atomicMin(&label[j], a);
      *changed = 1;
    } else if (b < a) {
      atomicMin(&label[i], b);
      *changed = 1;
    }
  }
}

// Pointer jumping: a label is a core point of the same component with a
// label no larger, so label <- label[label] only shortens the chains.
__global__ void k_cl_jump(const uint8_t* core, int32_t* label, int32_t N, int32_t* changed) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= N || !core[i]) return;
  const int32_t l = label[i];
  const int32_t ll = label[l];
  if (ll < l) {
    atomicMin(&label[i], ll);
    *changed = 1;
  }
}

// Border points: the nearest core point within eps in either list, packed
// as (d2 bits, component) so that atomicMin keeps the nearest (then the
// smaller component).
__global__ void k_cl_border(const float* Y, int DP, int d, const int32_t* ld, int K, int32_t N,
                            float eps2, const uint8_t* core, const int32_t* label,
                            unsigned long long* best) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= N) return;
  for (int k = 0; k < K; ++k) {
    const int32_t j = ld[(int64_t)i * K + k];
    if (core[i] == core[j]) continue;
    const float q = pair_d2(Y, DP, d, i, j);
    if (q > eps2) continue;
    const int32_t border = core[i] ? j : i, owner = core[i] ? i : j;
    const unsigned long long key =
        ((unsigned long long)__float_as_uint(q) << 32) | (uint32_t)label[owner];
    atomicMin(&best[border], key);
  }
}

__global__ void k_cl_final(const uint8_t* core, const int32_t* label,
                           const unsigned long long* best, int32_t N, int32_t* out) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= N) return;
  if (core[i])
    out[i] = label[i];
  else
    out[i] = best[i] == ~0ull ? -1 : (int32_t)(uint32_t)(best[i] & 0xffffffffull);
}

__global__ void k_fill_u64(unsigned long long* p, int32_t n, unsigned long long v) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

extern "C" {

fsne_status fsne_cluster(fsne_ctx* c, float eps, int32_t min_pts, int32_t* labels,
                         int32_t* n_clusters) {
  if (!c) return FSNE_EINVAL;
  if (!labels || !(eps > 0.0f) || min_pts < 1 || min_pts > c->Kl + 1) {
    c->err = "fsne_cluster: need labels, eps > 0 and 1 <= min_pts <= K_ld + 1";
    return FSNE_EINVAL;
  }
  const int32_t N = (int32_t)c->N;
  uint8_t* core = nullptr;
  int32_t *label = nullptr, *out = nullptr, *changed = nullptr;
  unsigned long long* best = nullptr;
  fsne_status st = FSNE_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == FSNE_OK) {
      c->err = std::string("fsne_cluster: ") + what + ": " + hipGetErrorString(e);
      st = FSNE_EHIP;
    }
    return st == FSNE_OK;
  };
  fsne::Scalars s;
  const dim3 g((unsigned)((N + kThreads - 1) / kThreads)), b(kThreads);
  const float eps2 = eps * eps;
  if (chk(hipMemcpyAsync(&s, c->sc, sizeof s, hipMemcpyDeviceToHost, c->stream), "scalars") &&
      chk(hipStreamSynchronize(c->stream), "sync") &&
      chk(hipMalloc(&core, (size_t)N), "hipMalloc") &&
      chk(hipMalloc(&label, sizeof(int32_t) * N), "hipMalloc") &&
      chk(hipMalloc(&out, sizeof(int32_t) * N), "hipMalloc") &&
      chk(hipMalloc(&changed, sizeof(int32_t)), "hipMalloc") &&
      chk(hipMalloc(&best, sizeof(unsigned long long) * N), "hipMalloc")) {
    const int32_t* ld = c->ld_idx[s.t & 1u];
    hipLaunchKernelGGL(k_cl_core, g, b, 0, c->stream, c->Y, c->DP, c->d, ld, c->Kl, N, eps2,
                       min_pts, core, label);
    chk(hipGetLastError(), "core");
    int32_t h = 1;
    for (int round = 0; h && st == FSNE_OK; ++round) {
      if (round == 100000) {
        c->err = "fsne_cluster: components did not converge";
        st = FSNE_EHIP;
        break;
      }
      h = 0;
      chk(hipMemcpyAsync(changed, &h, sizeof h, hipMemcpyHostToDevice, c->stream), "flag");
      hipLaunchKernelGGL(k_cl_hook, g, b, 0, c->stream, c->Y, c->DP, c->d, ld, c->Kl, N, eps2,
                         core, label, changed);
      for (int j = 0; j < 4; ++j)
        hipLaunchKernelGGL(k_cl_jump, g, b, 0, c->stream, core, label, N, changed);
      chk(hipGetLastError(), "components");
      chk(hipMemcpyAsync(&h, changed, sizeof h, hipMemcpyDeviceToHost, c->stream), "flag");
      chk(hipStreamSynchronize(c->stream), "sync");
    }
    hipLaunchKernelGGL(k_fill_u64, g, b, 0, c->stream, best, N, ~0ull);
    hipLaunchKernelGGL(k_cl_border, g, b, 0, c->stream, c->Y, c->DP, c->d, ld, c->Kl, N, eps2,
                       core, label, best);
    hipLaunchKernelGGL(k_cl_final, g, b, 0, c->stream, core, label, best, N, out);
    chk(hipGetLastError(), "border");
    chk(hipMemcpyAsync(labels, out, sizeof(int32_t) * N, hipMemcpyDeviceToHost, c->stream),
        "labels");
    chk(hipStreamSynchronize(c->stream), "sync");
  }
  for (void* p : {(void*)core, (void*)label, (void*)out, (void*)changed, (void*)best})
    if (p) (void)hipFree(p);
  if (st != FSNE_OK) return st;
  // number the clusters 0, 1, ... by their roots (smallest core point index)
  std::vector<int32_t> dense((size_t)N, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < N; ++i)
    if (labels[i] == i) dense[(size_t)i] = nc++;
  for (int32_t i = 0; i < N; ++i) labels[i] = labels[i] >= 0 ? dense[(size_t)labels[i]] : -1;
  if (n_clusters) *n_clusters = nc;
  return FSNE_OK;
}

fsne_status fsne_hierarchy_edges(const int32_t* la, int32_t ca, const int32_t* lb, int32_t cb,
                                 int64_t n, float* E) {
  if (!la || !lb || !E || ca < 0 || cb < 0 || n < 0) return FSNE_EINVAL;
  std::vector<int64_t> na((size_t)ca, 0), nb((size_t)cb, 0), both((size_t)ca * cb, 0);
  for (int64_t k = 0; k < n; ++k) {
    if (la[k] >= ca || lb[k] >= cb) return FSNE_EINVAL;
    if (la[k] >= 0) ++na[(size_t)la[k]];
    if (lb[k] >= 0) ++nb[(size_t)lb[k]];
    if (la[k] >= 0 && lb[k] >= 0) ++both[(size_t)la[k] * cb + lb[k]];
  }
  for (int32_t i = 0; i < ca; ++i)
    for (int32_t j = 0; j < cb; ++j) {
      const int64_t m = std::min(na[(size_t)i], nb[(size_t)j]);
      E[(size_t)i * cb + j] = m > 0 ? (float)((double)both[(size_t)i * cb + j] / (double)m) : 0.0f;
    }
  return FSNE_OK;
}

}  // extern "C"
