// C ABI of libfsne.so (declared in include/fsne.h): context, device state,
// argument checks, and the launch sequence of one FUnc-SNE iteration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fsne.h"
#include "fsne_kernels.h"

using fsne::Hyper;
using fsne::Scalars;
using fsne::StepArgs;

#include "fsne_context.h"

// Device staging of fsne_drift_points_noalloc (the ids, X rows and Y rows of
// one call): a fixed 16 MiB per device, held until the process ends.  Host
// code never passes `scratch` itself to a kernel or a copy; it uses the
// device address bind_scratch looks up.
static constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
constexpr int32_t kGraphIters = 25;   // iterations per captured graph
std::mutex g_scratch_mu;
void* g_scratch[kMaxScratchDevices] = {};

const char* kNoCtx = "null context";

fsne_status fail(fsne_ctx* c, fsne_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

fsne_status hip_fail(fsne_ctx* c, hipError_t e, const char* where) {
  return fail(c, FSNE_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                  \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

int pad_dim(int d) {
  int p = 2;
  while (p < d) p <<= 1;
  return p;
}

Hyper make_hyper(const fsne_ctx* c) {
  Hyper h{};
  const fsne_hparams& p = c->hp;
  h.alpha = p.alpha;
  h.inv_alpha = 1.0f / p.alpha;
  h.lr = p.lr;
  h.momentum = p.momentum;
  h.attr = p.attr;
  h.rep = p.rep;
  h.perplexity = p.perplexity;
  h.ln_perp = logf(p.perplexity);
  h.e_smooth = p.e_smooth;
  h.p_min = p.p_min;
  h.margin = p.rerank_margin;
  h.n_neg = p.n_neg;
  h.hd_mode = p.hd_mode;
  h.dist_mode = p.dist_mode;
  h.key0 = (uint32_t)c->seed;
  h.key1 = (uint32_t)(c->seed >> 32);
  return h;
}

StepArgs make_args(const fsne_ctx* c) {
  StepArgs a;
  std::memset(&a, 0, sizeof a);   // padding too: the graph cache compares whole structs
  a.X = c->X;
  a.xnorm = c->xnorm;
  a.xdtype = c->xdtype;
  a.xvec_ok = (((uintptr_t)c->X) & 15u) == 0;
  a.N = (int32_t)c->N;
  a.D = c->D;
  a.d = c->d;
  a.DP = c->DP;
  a.Kh = c->Kh;
  a.Kl = c->Kl;
  a.h = make_hyper(c);
  a.sc = c->sc;
  for (int b = 0; b < 2; ++b) {
    a.hd_idx[b] = c->hd_idx[b];
    a.hd_d2[b] = c->hd_d2[b];
    a.ld_idx[b] = c->ld_idx[b];
  }
  a.rec = c->rec;
  a.psh = c->psh;
  a.P = c->P;
  a.flags = c->flags;
  a.Y = c->Y;
  a.V = c->V;
  a.A = c->A;
  a.R = c->R;
  a.Zh = c->Zh;
  a.zpart = c->zpart;
  a.fpart = c->fpart;
  a.cpart = c->cpart;
  a.ldc = c->ldc;
  a.memo = c->hp.reject_memo ? c->memo : nullptr;
  // angular metric: the HD kernels take the Euclidean distances of the rows
  // scaled to unit length
  if (c->hp.metric == 1 && c->Xu) {
    a.X = c->Xu;
    a.xdtype = FSNE_F32;
    a.xvec_ok = 1;
  }
  // 64 remembered rejections pay where a saved row is large (direct distances
  // on rows of 512 bytes or more); elsewhere the extra 256 bytes of memory
  // traffic per point, or the screen kernel's registers, cost more than they save
  const int64_t row_bytes = (int64_t)c->D * (a.xdtype == FSNE_F32 ? 4 : 2);
  a.memo_w = (c->hp.dist_mode == 0 && row_bytes >= 512) ? 64 : 32;
  a.neg_scale = c->hp.n_neg > 0 ? (float)(c->N - 1) / (float)c->hp.n_neg : 0.0f;
  return a;
}

// The same with the stored rows themselves (for the BF16 row norms).
StepArgs raw_args(const fsne_ctx* c) {
  StepArgs a = make_args(c);
  a.X = c->X;
  a.xdtype = c->xdtype;
  a.xvec_ok = (((uintptr_t)c->X) & 15u) == 0;
  return a;
}

fsne_status check_hparams(fsne_ctx* c, const fsne_hparams* hp, int32_t Kh, int32_t xdtype,
                          int32_t D) {
  if (!hp) return fail(c, FSNE_EINVAL, "hparams is NULL");
  if (!(hp->alpha > 0.0f) || !std::isfinite(hp->alpha))
    return fail(c, FSNE_EINVAL, "alpha must be > 0");
  if (!(hp->perplexity > 1.0f) || !(hp->perplexity < (float)Kh))
    return fail(c, FSNE_EINVAL, "perplexity must satisfy 1 < perplexity < K_hd");
  if (!(hp->lr >= 0.0f) || !std::isfinite(hp->lr)) return fail(c, FSNE_EINVAL, "lr must be >= 0");
  if (!(hp->momentum >= 0.0f && hp->momentum < 1.0f))
    return fail(c, FSNE_EINVAL, "momentum must be in [0, 1)");
  if (!(hp->attr >= 0.0f) || !(hp->rep >= 0.0f) || !std::isfinite(hp->attr) ||
      !std::isfinite(hp->rep))
    return fail(c, FSNE_EINVAL, "attr and rep must be >= 0");
  if (hp->n_neg < 0 || hp->n_neg > 64) return fail(c, FSNE_EINVAL, "n_neg must be in 0..64");
  if (hp->hd_mode < 0 || hp->hd_mode > 2) return fail(c, FSNE_EINVAL, "hd_mode must be 0, 1, 2");
  if (hp->dist_mode < 0 || hp->dist_mode > 1)
    return fail(c, FSNE_EINVAL, "dist_mode must be 0 or 1");
  if (hp->dist_mode == 1 && (xdtype != FSNE_BF16 || D % 16 != 0))
    return fail(c, FSNE_EINVAL, "dist_mode 1 needs BF16 X with D % 16 == 0");
  if (!(hp->e_smooth > 0.0f && hp->e_smooth <= 1.0f))
    return fail(c, FSNE_EINVAL, "e_smooth must be in (0, 1]");
  if (!(hp->p_min >= 0.0f && hp->p_min <= 1.0f))
    return fail(c, FSNE_EINVAL, "p_min must be in [0, 1]");
  if (!(hp->rerank_margin >= 0.0f) || !std::isfinite(hp->rerank_margin))
    return fail(c, FSNE_EINVAL, "rerank_margin must be >= 0");
  if (hp->reject_memo < 0 || hp->reject_memo > 1)
    return fail(c, FSNE_EINVAL, "reject_memo must be 0 or 1");
  if (hp->metric < 0 || hp->metric > 1) return fail(c, FSNE_EINVAL, "metric must be 0 or 1");
  if (hp->metric == 1 && hp->dist_mode == 1)
    return fail(c, FSNE_EINVAL, "the BF16 screen needs metric 0 (it works on the raw rows)");
  if (Kh > fsne::kWave && hp->dist_mode == 1)
    return fail(c, FSNE_EINVAL, "the BF16 screen takes HD lists of at most 64");
  return FSNE_OK;
}

template <typename T>
fsne_status dalloc(fsne_ctx* c, T** p, size_t n) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 1);
  if (e != hipSuccess) return fail(c, FSNE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->owned.push_back(q);
  *p = static_cast<T*>(q);
  return FSNE_OK;
}

#define TRY(expr)                    \
  do {                               \
    fsne_status s_ = (expr);         \
    if (s_ != FSNE_OK) return s_;    \
  } while (0)

size_t xbytes(const fsne_ctx* c) { return c->xdtype == FSNE_F32 ? 4 : 2; }

// Host rows (n x d) -> device rows (n x DP, padding zero) at row offset r0.
// The host block goes over in one contiguous copy; a kernel re-strides it.
fsne_status put_Y(fsne_ctx* c, float* dst, const float* src, int64_t r0, int64_t n) {
  if (n <= 0) return FSNE_OK;
  if (!src) {
    HIPCHK(c, hipMemsetAsync(dst + r0 * c->DP, 0, sizeof(float) * n * c->DP, c->stream));
    return FSNE_OK;
  }
  if (c->d == c->DP) {
    HIPCHK(c, hipMemcpyAsync(dst + r0 * c->DP, src, sizeof(float) * n * c->d,
                             hipMemcpyHostToDevice, c->stream));
    return FSNE_OK;
  }
  float* tmp = nullptr;
  HIPCHK(c, hipMallocAsync(reinterpret_cast<void**>(&tmp), sizeof(float) * n * c->d, c->stream));
  HIPCHK(c, hipMemcpyAsync(tmp, src, sizeof(float) * n * c->d, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, fsne::launch_restride(dst + r0 * c->DP, c->DP, tmp, c->d, n, c->d, c->DP, c->stream));
  HIPCHK(c, hipFreeAsync(tmp, c->stream));
  return FSNE_OK;
}

// Device rows (N x DP) -> caller rows (N x d), host or device.
fsne_status get_rows(fsne_ctx* c, float* dst, const float* src, bool dst_dev) {
  const int64_t n = c->N;
  if (c->d == c->DP) {
    HIPCHK(c, hipMemcpyAsync(dst, src, sizeof(float) * n * c->d,
                             dst_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    return FSNE_OK;
  }
  if (dst_dev) {
    HIPCHK(c, fsne::launch_restride(dst, c->d, src, c->DP, n, c->d, c->d, c->stream));
    return FSNE_OK;
  }
  float* tmp = nullptr;
  HIPCHK(c, hipMallocAsync(reinterpret_cast<void**>(&tmp), sizeof(float) * n * c->d, c->stream));
  HIPCHK(c, fsne::launch_restride(tmp, c->d, src, c->DP, n, c->d, c->d, c->stream));
  HIPCHK(c, hipMemcpyAsync(dst, tmp, sizeof(float) * n * c->d, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipFreeAsync(tmp, c->stream));
  return FSNE_OK;
}

fsne_status read_scalars(fsne_ctx* c, Scalars* s) {
  HIPCHK(c, hipMemcpyAsync(s, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

fsne_status write_scalars(fsne_ctx* c, const Scalars& s) {
  HIPCHK(c, hipMemcpyAsync(c->sc, &s, sizeof(Scalars), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

fsne_status refresh_affinities(fsne_ctx* c, bool recalibrate) {
  StepArgs a = make_args(c);
  if (recalibrate) HIPCHK(c, fsne::launch_calibrate_all(a, c->stream));
  HIPCHK(c, fsne::launch_psym(a, 1, c->stream));
  HIPCHK(c, fsne::launch_set_fire(c->sc, a.h, c->stream));
  return FSNE_OK;
}

// Under the angular metric the HD kernels read Xu, the rows of X scaled to
// unit length: allocated on first use and recomputed for every row whenever
// X changes while that metric is in use (and when it is switched on).
fsne_status refresh_unit_rows(fsne_ctx* c) {
  if (c->hp.metric != 1) return FSNE_OK;
  if (!c->Xu) TRY(dalloc(c, &c->Xu, (size_t)c->cap * c->D));
  HIPCHK(c, fsne::launch_unit_rows(c->X, c->xdtype, c->Xu, c->D, 0, (int32_t)c->N, c->stream));
  return FSNE_OK;
}

// The HD metric changed (c->hp holds the new one): every list keeps its
// members, every stored distance is recomputed in the new metric, each row is
// re-sorted by (d2, id), flagged and recalibrated (the drift kernel with every
// point marked), P is recomputed, and E restarts at 1 so that the coin
// refines at once: the lists are not yet the new metric's neighbours.
fsne_status switch_metric(fsne_ctx* c) {
  TRY(refresh_unit_rows(c));
  HIPCHK(c, hipMemsetAsync(c->moved, 1, (size_t)c->N, c->stream));
  HIPCHK(c, fsne::launch_drift_rows(make_args(c), c->moved, c->stream));
  Scalars s;
  TRY(read_scalars(c, &s));
  s.E = 1.0f;
  TRY(write_scalars(c, s));
  return refresh_affinities(c, false);
}

// Forget the rejected HD candidates of rows [r0, r0 + n).
fsne_status clear_memo(fsne_ctx* c, int64_t r0, int64_t n) {
  if (n > 0)
    HIPCHK(c, hipMemsetAsync(c->memo + r0 * fsne::kMemo, 0xFF,
                             sizeof(int32_t) * (size_t)n * fsne::kMemo, c->stream));
  return FSNE_OK;
}

fsne_status alloc_state(fsne_ctx* c) {
  const size_t cap = (size_t)c->cap;
  TRY(dalloc(c, &c->Y, cap * c->DP));
  TRY(dalloc(c, &c->V, cap * c->DP));
  TRY(dalloc(c, &c->A, cap * c->DP));
  TRY(dalloc(c, &c->R, cap * c->DP));
  TRY(dalloc(c, &c->Zh, cap));
  TRY(dalloc(c, &c->P, cap * c->Kh));
  TRY(dalloc(c, &c->zpart, (size_t)fsne::kReduceBlocks));
  TRY(dalloc(c, &c->fpart, (size_t)fsne::kReduceBlocks));
  TRY(dalloc(c, &c->cpart, 2 * (size_t)fsne::kReduceBlocks));
  TRY(dalloc(c, &c->ldc, cap));
  for (int b = 0; b < 2; ++b) {
    TRY(dalloc(c, &c->hd_idx[b], cap * c->Kh));
    TRY(dalloc(c, &c->hd_d2[b], cap * c->Kh));
    TRY(dalloc(c, &c->ld_idx[b], cap * c->Kl));
  }
  TRY(dalloc(c, &c->rec, cap));
  TRY(dalloc(c, &c->psh, 2 * cap));
  TRY(dalloc(c, &c->flags, cap));
  TRY(dalloc(c, &c->moved, cap));
  TRY(dalloc(c, &c->memo, cap * fsne::kMemo));
  TRY(dalloc(c, &c->sc, 1));
  TRY(clear_memo(c, 0, c->cap));
  HIPCHK(c, hipMemsetAsync(c->A, 0, sizeof(float) * cap * c->DP, c->stream));
  HIPCHK(c, hipMemsetAsync(c->R, 0, sizeof(float) * cap * c->DP, c->stream));
  HIPCHK(c, hipMemsetAsync(c->Zh, 0, sizeof(float) * cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->flags, 0, cap, c->stream));
  HIPCHK(c, hipMemsetAsync(c->ldc, 0, cap, c->stream));
  return FSNE_OK;
}

fsne_status do_init(fsne_ctx* c, const void* X, int32_t x_on_device, const float* Y0) {
  TRY(alloc_state(c));
  const size_t xb = xbytes(c);
  if (x_on_device && c->cap == c->N) {
    c->X = const_cast<void*>(X);
  } else {
    void* q = nullptr;
    TRY(dalloc(c, reinterpret_cast<uint8_t**>(&q), (size_t)c->cap * c->D * xb));
    c->X = q;
    c->own_X = true;
    HIPCHK(c, hipMemcpyAsync(c->X, X, (size_t)c->N * c->D * xb,
                             x_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
  }
  if (c->xdtype == FSNE_BF16) {
    TRY(dalloc(c, &c->xnorm, (size_t)c->cap));
  }
  TRY(put_Y(c, c->Y, Y0, 0, c->N));
  HIPCHK(c, hipMemsetAsync(c->V, 0, sizeof(float) * c->cap * c->DP, c->stream));
  Scalars s{};
  s.t = 0;
  s.E = 1.0f;
  s.hd_cur = 0;
  TRY(write_scalars(c, s));
  TRY(refresh_unit_rows(c));
  StepArgs a = make_args(c);
  a.hd_buf_host = 0;
  a.ld_buf_host = 0;
  if (c->xdtype == FSNE_BF16)
    HIPCHK(c, fsne::launch_xnorm(raw_args(c), c->xnorm, 0, (int32_t)c->N, c->stream));
  HIPCHK(c, fsne::launch_init_lists(a, 0, (int32_t)c->N, c->stream));
  TRY(refresh_affinities(c, false));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

hipError_t take_event(fsne_ctx* c, hipEvent_t* e) {
  if (!c->spare.empty()) {
    *e = c->spare.back();
    c->spare.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Sum the elapsed times of the recorded kernel launches (synchronises).
fsne_status drain_timings(fsne_ctx* c) {
  if (c->pending.empty()) return FSNE_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (const auto& t : c->pending) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, t.start, t.stop));
    c->ms[t.kernel] += ms;
    c->launches[t.kernel] += 1;
    c->spare.push_back(t.start);
    c->spare.push_back(t.stop);
  }
  c->pending.clear();
  return FSNE_OK;
}

template <typename Launch>
fsne_status timed_launch(fsne_ctx* c, int kernel, Launch&& launch) {
  if (!c->prof) {
    HIPCHK(c, launch());
    return FSNE_OK;
  }
  fsne_ctx::Timed t{kernel, nullptr, nullptr};
  HIPCHK(c, take_event(c, &t.start));
  HIPCHK(c, take_event(c, &t.stop));
  HIPCHK(c, hipEventRecord(t.start, c->stream));
  HIPCHK(c, launch());
  HIPCHK(c, hipEventRecord(t.stop, c->stream));
  c->pending.push_back(t);
  if (c->pending.size() >= 4096) TRY(drain_timings(c));
  return FSNE_OK;
}

void drop_graph(fsne_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->gn = 0;
}

void release(fsne_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (const auto& t : c->pending) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (hipEvent_t e : c->spare) (void)hipEventDestroy(e);
  drop_graph(c);
  c->pending.clear();
  c->spare.clear();
  for (void* p : c->owned) (void)hipFree(p);
  c->owned.clear();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  c->stream = nullptr;
}

// One iteration's five launches (each timed when profiling is on).
fsne_status launch_iteration(fsne_ctx* c, const StepArgs& a, hipStream_t s) {
  TRY(timed_launch(c, FSNE_K_HD_REFINE, [&] { return fsne::launch_hd_refine(a, s); }));
  TRY(timed_launch(c, FSNE_K_AFFINITY, [&] { return fsne::launch_psym(a, 0, s); }));
  TRY(timed_launch(c, FSNE_K_LD_GRAD, [&] { return fsne::launch_ld_grad(a, s); }));
  TRY(timed_launch(c, FSNE_K_REDUCE, [&] { return fsne::launch_reduce(a, s); }));
  TRY(timed_launch(c, FSNE_K_UPDATE, [&] { return fsne::launch_update(a, s); }));
  return FSNE_OK;
}

// A graph of n iterations for these kernel arguments (captured on first use).
fsne_status ensure_graph(fsne_ctx* c, const StepArgs& a, int32_t n) {
  if (c->gexec && c->gn == n && std::memcmp(&c->gargs, &a, sizeof a) == 0) return FSNE_OK;
  drop_graph(c);
  hipStream_t s = c->stream;
  HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  fsne_status st = FSNE_OK;
  for (int32_t k = 0; k < n && st == FSNE_OK; ++k) st = launch_iteration(c, a, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != FSNE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(c, e, "graph capture");
  hipGraphExec_t x = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return hip_fail(c, e2, "graph instantiate");
  c->gexec = x;
  c->gn = n;
  c->gargs = a;
  return FSNE_OK;
}

// Apply a drift whose staging is on the device: n ids (int32), their new X
// rows and, if dy is not null, their new Y rows (padded, n x DP).
fsne_status drift_apply(fsne_ctx* c, const int32_t* dids, const uint8_t* dx, const float* dy,
                        int64_t n) {
  const size_t xrow = (size_t)c->D * xbytes(c);
  HIPCHK(c, fsne::launch_scatter_rows(c->X, dx, dids, (int32_t)n, (int32_t)xrow, c->stream));
  if (dy)
    HIPCHK(c, fsne::launch_scatter_rows(c->Y, dy, dids, (int32_t)n,
                                        (int32_t)(sizeof(float) * c->DP), c->stream));
  HIPCHK(c, hipMemsetAsync(c->moved, 0, (size_t)c->N, c->stream));
  HIPCHK(c, fsne::launch_mark_moved(c->moved, c->V, c->DP, dids, (int32_t)n, c->stream));
  // moved rows change distances in both directions: every rejection is void
  TRY(clear_memo(c, 0, c->cap));
  TRY(refresh_unit_rows(c));
  StepArgs a = make_args(c);
  if (c->xdtype == FSNE_BF16)
    HIPCHK(c, fsne::launch_xnorm(raw_args(c), c->xnorm, 0, (int32_t)c->N, c->stream));
  HIPCHK(c, fsne::launch_drift_rows(a, c->moved, c->stream));
  return refresh_affinities(c, false);
}

__global__ void k_narrow_ids(const int64_t* __restrict__ in, int32_t* __restrict__ out,
                             int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = (int32_t)in[k];
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The address of `scratch` on the current device, looked up once per device
// (each GPU holds its own copy of the array).
fsne_status bind_scratch(fsne_ctx* c) {
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(c, FSNE_EHIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(c, e, "scratch address");
    g_scratch[dev] = p;
  }
  c->scratch = g_scratch[dev];
  return FSNE_OK;
}

}  // namespace

extern "C" {

int32_t fsne_max_dim(int32_t xdtype, int32_t D) {
  // rows are spread over a wave in vectors of 16 bytes (when D allows) or
  // single elements, at most 16 (FP32) / 4 (BF16) vectors per lane
  if (xdtype == FSNE_F32) return D % 4 == 0 ? 64 * 4 * 16 : 64 * 16;
  return D % 8 == 0 ? 64 * 8 * 4 : 64 * 16;
}

fsne_status fsne_default_hparams(fsne_hparams* hp) {
  if (!hp) return FSNE_EINVAL;
  hp->alpha = 1.0f;
  hp->perplexity = 10.0f;
  hp->lr = 100.0f;
  hp->momentum = 0.5f;
  hp->attr = 1.0f;
  hp->rep = 1.0f;
  hp->n_neg = 16;
  hp->hd_mode = 0;
  hp->dist_mode = 0;
  hp->e_smooth = 0.1f;
  hp->p_min = 0.05f;
  hp->rerank_margin = 1.0f / 64.0f;
  hp->reject_memo = 1;
  hp->metric = 0;
  return FSNE_OK;
}

fsne_status fsne_init(fsne_ctx** out, const void* X, int64_t N, int32_t D, int32_t xdtype,
                      const float* Y0, int32_t d, int32_t K_hd, int32_t K_ld, float alpha,
                      float perplexity, uint64_t seed, const fsne_hparams* hp,
                      int32_t x_on_device, void* stream, int64_t capacity) {
  if (!out) return FSNE_EINVAL;
  *out = nullptr;
  if (!X || N < 3 || N > 2147483647LL || D < 1 || d < 1 || d > 64 || K_hd < 2 ||
      K_hd > fsne::kMaxLong || K_ld < 1 || K_ld > 64 || K_hd >= N || K_ld >= N ||
      (xdtype != FSNE_F32 && xdtype != FSNE_BF16))
    return FSNE_EINVAL;
  if (capacity < N || capacity > 2147483647LL) return FSNE_EINVAL;
  if (D > fsne_max_dim(xdtype, D)) return FSNE_EINVAL;
  fsne_ctx* c = new (std::nothrow) fsne_ctx();
  if (!c) return FSNE_ENOMEM;
  fsne_hparams h;
  if (hp)
    h = *hp;
  else
    fsne_default_hparams(&h);
  h.alpha = alpha;
  h.perplexity = perplexity;
  fsne_status st = check_hparams(c, &h, K_hd, xdtype, D);
  if (st != FSNE_OK) {
    delete c;
    return st;
  }
  c->N = N;
  c->cap = capacity;
  c->D = D;
  c->d = d;
  c->DP = pad_dim(d);
  c->Kh = K_hd;
  c->Kl = K_ld;
  c->xdtype = xdtype;
  c->seed = seed;
  c->hp = h;
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return FSNE_EHIP;
    }
    c->own_stream = true;
  }
  st = bind_scratch(c);
  if (st == FSNE_OK) st = do_init(c, X, x_on_device, Y0);
  if (st != FSNE_OK) {
    release(c);
    delete c;
    return st;
  }
  *out = c;
  return FSNE_OK;
}

fsne_status fsne_step(fsne_ctx* c, int32_t n_iters) {
  if (!c) return FSNE_EINVAL;
  if (n_iters < 0) return fail(c, FSNE_EINVAL, "n_iters < 0");
  const StepArgs a = make_args(c);
  hipStream_t s = c->stream;
  int32_t it = 0;
  // Without per-kernel timing, whole chunks of iterations go out as one
  // captured HIP graph (the iteration's five launches, kGraphIters times):
  // one launch instead of five per iteration.  The graph is kept while the
  // kernel arguments stay the same.
  if (!c->prof && c->use_graph) {
    const int32_t chunk = std::min<int32_t>(n_iters, kGraphIters);
    if (chunk >= 2) {
      TRY(ensure_graph(c, a, chunk));
      for (; it + chunk <= n_iters; it += chunk) HIPCHK(c, hipGraphLaunch(c->gexec, s));
    }
  }
  for (; it < n_iters; ++it) TRY(launch_iteration(c, a, s));
  return FSNE_OK;
}

fsne_status fsne_set_hyperparams(fsne_ctx* c, const fsne_hparams* hp) {
  if (!c) return FSNE_EINVAL;
  TRY(check_hparams(c, hp, c->Kh, c->xdtype, c->D));
  const bool perp_changed = hp->perplexity != c->hp.perplexity;
  const bool metric_changed = hp->metric != c->hp.metric;
  if (metric_changed && c->Kh > fsne::kWave)
    return fail(c, FSNE_EINVAL, "a metric switch takes HD lists of at most 64");
  // a rejection under one screen (or metric) need not be one under another
  const bool screen_changed =
      hp->dist_mode != c->hp.dist_mode || hp->rerank_margin != c->hp.rerank_margin;
  const fsne_hparams old = c->hp;
  c->hp = *hp;
  if (screen_changed || metric_changed) TRY(clear_memo(c, 0, c->cap));
  if (metric_changed) {
    const fsne_status st = switch_metric(c);
    if (st != FSNE_OK) {
      c->hp = old;   // e.g. no memory for the unit rows: nothing was recomputed
      return st;
    }
  } else if (perp_changed) {
    TRY(refresh_affinities(c, true));
  } else {
    HIPCHK(c, fsne::launch_set_fire(c->sc, make_hyper(c), c->stream));
  }
  return FSNE_OK;
}

fsne_status fsne_get_hyperparams(const fsne_ctx* c, fsne_hparams* hp) {
  if (!c || !hp) return FSNE_EINVAL;
  *hp = c->hp;
  return FSNE_OK;
}

fsne_status fsne_sync(fsne_ctx* c) {
  if (!c) return FSNE_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

fsne_status fsne_get_Y(fsne_ctx* c, float* out, int32_t out_on_device) {
  if (!c || !out) return c ? fail(c, FSNE_EINVAL, "out is NULL") : FSNE_EINVAL;
  TRY(get_rows(c, out, c->Y, out_on_device != 0));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

fsne_status fsne_get_knn(fsne_ctx* c, int32_t which, int32_t* idx, float* dist2) {
  if (!c) return FSNE_EINVAL;
  if (!idx || (which != 0 && which != 1) || (which == 1 && dist2))
    return fail(c, FSNE_EINVAL, "bad arguments to fsne_get_knn");
  Scalars s;
  TRY(read_scalars(c, &s));
  if (which == 0) {
    HIPCHK(c, hipMemcpyAsync(idx, c->hd_idx[s.hd_cur], sizeof(int32_t) * c->N * c->Kh,
                             hipMemcpyDeviceToHost, c->stream));
    if (dist2)
      HIPCHK(c, hipMemcpyAsync(dist2, c->hd_d2[s.hd_cur], sizeof(float) * c->N * c->Kh,
                               hipMemcpyDeviceToHost, c->stream));
  } else {
    HIPCHK(c, hipMemcpyAsync(idx, c->ld_idx[s.t & 1], sizeof(int32_t) * c->N * c->Kl,
                             hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

fsne_status fsne_get_state(fsne_ctx* c, const fsne_state_view* v) {
  if (!c || !v) return c ? fail(c, FSNE_EINVAL, "view is NULL") : FSNE_EINVAL;
  Scalars s;
  TRY(read_scalars(c, &s));
  const int64_t N = c->N;
  const hipMemcpyKind k = hipMemcpyDeviceToHost;
  if (v->Y) TRY(get_rows(c, v->Y, c->Y, false));
  if (v->V) TRY(get_rows(c, v->V, c->V, false));
  if (v->A) TRY(get_rows(c, v->A, c->A, false));
  if (v->R) TRY(get_rows(c, v->R, c->R, false));
  if (v->Zh) HIPCHK(c, hipMemcpyAsync(v->Zh, c->Zh, sizeof(float) * N, k, c->stream));
  if (v->hd_idx)
    HIPCHK(c, hipMemcpyAsync(v->hd_idx, c->hd_idx[s.hd_cur], sizeof(int32_t) * N * c->Kh, k,
                             c->stream));
  if (v->hd_d2)
    HIPCHK(c, hipMemcpyAsync(v->hd_d2, c->hd_d2[s.hd_cur], sizeof(float) * N * c->Kh, k,
                             c->stream));
  if (v->ld_idx)
    HIPCHK(c, hipMemcpyAsync(v->ld_idx, c->ld_idx[s.t & 1], sizeof(int32_t) * N * c->Kl, k,
                             c->stream));
  if (v->rec) HIPCHK(c, hipMemcpyAsync(v->rec, c->rec, sizeof(float4) * N, k, c->stream));
  if (v->P) HIPCHK(c, hipMemcpyAsync(v->P, c->P, sizeof(float) * N * c->Kh, k, c->stream));
  if (v->flags) HIPCHK(c, hipMemcpyAsync(v->flags, c->flags, (size_t)N, k, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (v->flags)
    for (int64_t k = 0; k < N; ++k) v->flags[k] &= 1u;
  if (v->E) *v->E = s.E;
  if (v->t) *v->t = s.t;
  return FSNE_OK;
}

fsne_status fsne_set_state(fsne_ctx* c, const fsne_state_view* v) {
  if (!c || !v) return c ? fail(c, FSNE_EINVAL, "view is NULL") : FSNE_EINVAL;
  Scalars s;
  TRY(read_scalars(c, &s));
  const int64_t N = c->N;
  const hipMemcpyKind k = hipMemcpyHostToDevice;
  const uint32_t t_new = v->t ? *v->t : s.t;
  if (((t_new ^ s.t) & 1u) && !v->ld_idx)
    HIPCHK(c, hipMemcpyAsync(c->ld_idx[t_new & 1], c->ld_idx[s.t & 1],
                             sizeof(int32_t) * N * c->Kl, hipMemcpyDeviceToDevice, c->stream));
  if (v->Y) TRY(put_Y(c, c->Y, v->Y, 0, N));
  if (v->V) TRY(put_Y(c, c->V, v->V, 0, N));
  if (v->hd_idx)
    HIPCHK(c, hipMemcpyAsync(c->hd_idx[s.hd_cur], v->hd_idx, sizeof(int32_t) * N * c->Kh, k,
                             c->stream));
  if (v->hd_d2)
    HIPCHK(c, hipMemcpyAsync(c->hd_d2[s.hd_cur], v->hd_d2, sizeof(float) * N * c->Kh, k,
                             c->stream));
  if (v->ld_idx)
    HIPCHK(c, hipMemcpyAsync(c->ld_idx[t_new & 1], v->ld_idx, sizeof(int32_t) * N * c->Kl, k,
                             c->stream));
  if (v->rec) HIPCHK(c, hipMemcpyAsync(c->rec, v->rec, sizeof(float4) * N, k, c->stream));
  if (v->P) HIPCHK(c, hipMemcpyAsync(c->P, v->P, sizeof(float) * N * c->Kh, k, c->stream));
  if (v->flags) HIPCHK(c, hipMemcpyAsync(c->flags, v->flags, (size_t)N, k, c->stream));
  // lists from outside may hold a larger K-th distance than the ones the
  // remembered rejections were measured against
  if (v->hd_idx || v->hd_d2) TRY(clear_memo(c, 0, c->cap));
  if (v->E) s.E = *v->E;
  s.t = t_new;
  s.nonfinite = 0;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  TRY(write_scalars(c, s));
  // refinements update the affinities only where a list changed, so lists or
  // records set without their affinities get theirs recomputed here
  if (!v->P && (v->hd_idx || v->hd_d2 || v->rec)) TRY(refresh_affinities(c, false));
  HIPCHK(c, fsne::launch_set_fire(c->sc, make_hyper(c), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

fsne_status fsne_get_stats(fsne_ctx* c, fsne_stats* st) {
  if (!c || !st) return c ? fail(c, FSNE_EINVAL, "stats is NULL") : FSNE_EINVAL;
  Scalars s;
  TRY(read_scalars(c, &s));
  st->N = c->N;
  st->t = s.t;
  st->E = s.E;
  st->next_fire = s.fire;
  st->last_fired = s.last_fired;
  st->n_new = s.n_new;
  st->Z = s.Z;
  st->nonfinite = s.nonfinite;
  st->hd_cand_rows = s.hd_cand;
  st->ld_cand_rows = s.ld_cand;
  st->hd_refinements = s.refinements;
  if (s.nonfinite) return fail(c, FSNE_ENONFINITE, "embedding holds a NaN or infinity");
  return FSNE_OK;
}

fsne_status fsne_insert_points(fsne_ctx* c, const void* Xnew, int64_t n, const float* Yinit) {
  if (!c) return FSNE_EINVAL;
  if (!Xnew || n < 0) return fail(c, FSNE_EINVAL, "bad arguments to fsne_insert_points");
  if (n == 0) return FSNE_OK;
  if (c->N + n > c->cap) return fail(c, FSNE_ENOMEM, "insert beyond capacity");
  if (!c->own_X) return fail(c, FSNE_ESTATE, "X is borrowed; create the context with capacity");
  Scalars s;
  TRY(read_scalars(c, &s));
  const int64_t N0 = c->N;
  const size_t xb = xbytes(c);
  HIPCHK(c, hipMemcpyAsync(static_cast<uint8_t*>(c->X) + (size_t)N0 * c->D * xb, Xnew,
                           (size_t)n * c->D * xb, hipMemcpyHostToDevice, c->stream));
  TRY(put_Y(c, c->Y, Yinit, N0, n));
  HIPCHK(c, hipMemsetAsync(c->V + N0 * c->DP, 0, sizeof(float) * n * c->DP, c->stream));
  TRY(clear_memo(c, N0, n));   // rows left by deleted points
  c->N = N0 + n;
  TRY(refresh_unit_rows(c));
  StepArgs a = make_args(c);
  a.hd_buf_host = s.hd_cur;
  a.ld_buf_host = (int32_t)(s.t & 1u);
  if (c->xdtype == FSNE_BF16)
    HIPCHK(c, fsne::launch_xnorm(raw_args(c), c->xnorm, (int32_t)N0, (int32_t)n, c->stream));
  HIPCHK(c, fsne::launch_init_lists(a, (int32_t)N0, (int32_t)n, c->stream));
  TRY(refresh_affinities(c, false));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FSNE_OK;
}

fsne_status fsne_drift_points(fsne_ctx* c, const int64_t* ids, const void* Xnew, int64_t n,
                              const float* Yinit) {
  if (!c) return FSNE_EINVAL;
  if (!ids || !Xnew || n < 0) return fail(c, FSNE_EINVAL, "bad arguments to fsne_drift_points");
  if (n == 0) return FSNE_OK;
  if (c->Kh > fsne::kWave) return fail(c, FSNE_EINVAL, "drift takes HD lists of at most 64");
  if (!c->own_X) return fail(c, FSNE_ESTATE, "X is borrowed; create the context with capacity");
  std::vector<uint8_t> seen((size_t)c->N, 0);
  std::vector<int32_t> ids32((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    if (ids[k] < 0 || ids[k] >= c->N) return fail(c, FSNE_EINVAL, "drift id out of range");
    if (seen[(size_t)ids[k]]) return fail(c, FSNE_EINVAL, "duplicate drift id");
    seen[(size_t)ids[k]] = 1;
    ids32[(size_t)k] = (int32_t)ids[k];
  }
  const size_t xrow = (size_t)c->D * xbytes(c);
  int32_t* dids = nullptr;
  uint8_t* dx = nullptr;
  float* dy = nullptr;
  fsne_status st = FSNE_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(c->stream);
    if (dids) (void)hipFree(dids);
    if (dx) (void)hipFree(dx);
    if (dy) (void)hipFree(dy);
  };
  if (hipMalloc(&dids, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&dx, xrow * n) != hipSuccess ||
      (Yinit && hipMalloc(&dy, sizeof(float) * n * c->DP) != hipSuccess)) {
    cleanup();
    return fail(c, FSNE_ENOMEM, "drift staging allocation failed");
  }
  do {
    hipError_t e;
    if ((e = hipMemcpyAsync(dids, ids32.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice,
                            c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(dx, Xnew, xrow * n, hipMemcpyHostToDevice, c->stream)) != hipSuccess) {
      st = hip_fail(c, e, "drift upload");
      break;
    }
    if (Yinit && (st = put_Y(c, dy, Yinit, 0, n)) != FSNE_OK) break;
    st = drift_apply(c, dids, dx, dy, n);
  } while (false);
  cleanup();
  return st;
}

fsne_status fsne_drift_points_noalloc(fsne_ctx* c, const int64_t* ids, const void* Xnew,
                                      int64_t n, const float* Yinit) {
  if (!c) return FSNE_EINVAL;
  if (!ids || !Xnew || n < 0)
    return fail(c, FSNE_EINVAL, "bad arguments to fsne_drift_points_noalloc");
  if (n == 0) return FSNE_OK;
  if (c->Kh > fsne::kWave) return fail(c, FSNE_EINVAL, "drift takes HD lists of at most 64");
  if (!c->own_X) return fail(c, FSNE_ESTATE, "X is borrowed; create the context with capacity");
  if (!c->scratch) return fail(c, FSNE_ESTATE, "no device scratch for this context's device");
  for (int64_t k = 0; k < n; ++k) {
    if (ids[k] < 0 || ids[k] >= c->N) return fail(c, FSNE_EINVAL, "drift id out of range");
    if (k > 0 && ids[k] <= ids[k - 1])
      return fail(c, FSNE_EINVAL, "drift ids must be strictly increasing");
  }
  const size_t xrow = (size_t)c->D * xbytes(c);
  const size_t o_ids = 0, o_ids32 = align256(sizeof(int64_t) * n);
  const size_t o_x = o_ids32 + align256(sizeof(int32_t) * n);
  const size_t o_yh = o_x + align256(xrow * n);
  const size_t o_y = o_yh + align256(sizeof(float) * n * c->d);
  const size_t need = o_y + align256(sizeof(float) * n * c->DP);
  if (need > kScratchBytes)
    return fail(c, FSNE_EINVAL,
                "drift batch too large for the fixed scratch: " + std::to_string(need) +
                    " bytes needed, " + std::to_string(kScratchBytes) + " available");
  uint8_t* w = static_cast<uint8_t*>(c->scratch);
  int64_t* d64 = reinterpret_cast<int64_t*>(w + o_ids);
  int32_t* dids = reinterpret_cast<int32_t*>(w + o_ids32);
  uint8_t* dx = w + o_x;
  float* dyh = reinterpret_cast<float*>(w + o_yh);
  float* dy = Yinit ? reinterpret_cast<float*>(w + o_y) : nullptr;
  HIPCHK(c, hipMemcpyAsync(d64, ids, sizeof(int64_t) * n, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_narrow_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     d64, dids, n);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(dx, Xnew, xrow * n, hipMemcpyHostToDevice, c->stream));
  if (Yinit) {
    HIPCHK(c, hipMemcpyAsync(dyh, Yinit, sizeof(float) * n * c->d, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, fsne::launch_restride(dy, c->DP, dyh, c->d, n, c->d, c->DP, c->stream));
  }
  const fsne_status st = drift_apply(c, dids, dx, dy, n);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return st;
}

fsne_status fsne_delete_points(fsne_ctx* c, const int64_t* ids, int64_t n) {
  if (!c) return FSNE_EINVAL;
  if (!ids || n < 0) return fail(c, FSNE_EINVAL, "bad arguments to fsne_delete_points");
  if (n == 0) return FSNE_OK;
  if (c->Kh > fsne::kWave) return fail(c, FSNE_EINVAL, "delete takes HD lists of at most 64");
  if (!c->own_X) return fail(c, FSNE_ESTATE, "X is borrowed; create the context with capacity");
  const int64_t N = c->N, N1 = N - n;
  if (N1 <= std::max(c->Kh, c->Kl)) return fail(c, FSNE_EINVAL, "too few points would remain");
  std::vector<uint8_t> del((size_t)N, 0);
  for (int64_t k = 0; k < n; ++k) {
    if (ids[k] < 0 || ids[k] >= N) return fail(c, FSNE_EINVAL, "delete id out of range");
    if (del[(size_t)ids[k]]) return fail(c, FSNE_EINVAL, "duplicate delete id");
    del[(size_t)ids[k]] = 1;
  }
  // survivors at or beyond N1 move, in increasing order, into the deleted
  // slots below N1, in increasing order
  std::vector<int32_t> newid((size_t)N), src, dst;
  for (int64_t j = N1; j < N; ++j)
    if (!del[(size_t)j]) src.push_back((int32_t)j);
  for (int64_t j = 0; j < N1; ++j)
    if (del[(size_t)j]) dst.push_back((int32_t)j);
  for (int64_t j = 0; j < N; ++j) newid[(size_t)j] = del[(size_t)j] ? -1 : (int32_t)j;
  for (size_t k = 0; k < src.size(); ++k) newid[(size_t)src[k]] = dst[k];
  Scalars s;
  TRY(read_scalars(c, &s));
  const int32_t m = (int32_t)src.size();
  int32_t *dnew = nullptr, *dsrc = nullptr, *ddst = nullptr;
  fsne_status st = FSNE_OK;
  if (hipMalloc(&dnew, sizeof(int32_t) * N) != hipSuccess ||
      hipMalloc(&dsrc, sizeof(int32_t) * (m + 1)) != hipSuccess ||
      hipMalloc(&ddst, sizeof(int32_t) * (m + 1)) != hipSuccess) {
    st = fail(c, FSNE_ENOMEM, "delete staging allocation failed");
  }
  do {
    if (st != FSNE_OK) break;
    hipError_t e;
    if ((e = hipMemcpyAsync(dnew, newid.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice,
                            c->stream)) != hipSuccess ||
        (m > 0 && (e = hipMemcpyAsync(dsrc, src.data(), sizeof(int32_t) * m,
                                      hipMemcpyHostToDevice, c->stream)) != hipSuccess) ||
        (m > 0 && (e = hipMemcpyAsync(ddst, dst.data(), sizeof(int32_t) * m,
                                      hipMemcpyHostToDevice, c->stream)) != hipSuccess)) {
      st = hip_fail(c, e, "delete upload");
      break;
    }
    struct Rows {
      void* base;
      size_t bytes;
    };
    const Rows rows[] = {
        {c->X, (size_t)c->D * xbytes(c)},
        {c->Y, sizeof(float) * c->DP},
        {c->V, sizeof(float) * c->DP},
        {c->rec, sizeof(float4)},
        {c->hd_idx[s.hd_cur], sizeof(int32_t) * c->Kh},
        {c->hd_d2[s.hd_cur], sizeof(float) * c->Kh},
        {c->ld_idx[s.t & 1u], sizeof(int32_t) * c->Kl},
        {c->flags, 1},
        {c->xdtype == FSNE_BF16 ? (void*)c->xnorm : nullptr, sizeof(float)},
    };
    for (const Rows& r : rows) {
      if (!r.base) continue;
      if ((e = fsne::launch_move_rows(r.base, dsrc, ddst, m, (int32_t)r.bytes, c->stream)) !=
          hipSuccess)
        break;
    }
    if (e != hipSuccess) {
      st = hip_fail(c, e, "delete moves");
      break;
    }
    c->N = N1;
    // ids are renumbered and lists refilled at random: every rejection is void
    if ((st = clear_memo(c, 0, c->cap)) != FSNE_OK) break;
    if ((st = refresh_unit_rows(c)) != FSNE_OK) break;
    StepArgs a = make_args(c);
    if ((e = fsne::launch_delete_fix(a, dnew, c->stream)) != hipSuccess) {
      st = hip_fail(c, e, "delete lists");
      break;
    }
    st = refresh_affinities(c, false);
  } while (false);
  (void)hipStreamSynchronize(c->stream);
  if (dnew) (void)hipFree(dnew);
  if (dsrc) (void)hipFree(dsrc);
  if (ddst) (void)hipFree(ddst);
  return st;
}

fsne_status fsne_profile(fsne_ctx* c, int32_t enable) {
  if (!c) return FSNE_EINVAL;
  TRY(drain_timings(c));
  c->prof = enable != 0;
  // events for the first 1024 launches up front: none is created between launches
  while (c->prof && c->spare.size() < 2048) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    c->spare.push_back(e);
  }
  for (int k = 0; k < FSNE_NKERNELS; ++k) {
    c->ms[k] = 0.0;
    c->launches[k] = 0;
  }
  return FSNE_OK;
}

fsne_status fsne_get_kernel_times(fsne_ctx* c, double* ms, int64_t* launches) {
  if (!c) return FSNE_EINVAL;
  if (!ms || !launches) return fail(c, FSNE_EINVAL, "ms and launches must not be NULL");
  TRY(drain_timings(c));
  for (int k = 0; k < FSNE_NKERNELS; ++k) {
    ms[k] = c->ms[k];
    launches[k] = c->launches[k];
  }
  return FSNE_OK;
}

fsne_status fsne_implode(fsne_ctx* c, float factor) {
  if (!c) return FSNE_EINVAL;
  if (!(factor > 0.0f) || !std::isfinite(factor)) return fail(c, FSNE_EINVAL, "factor must be > 0");
  HIPCHK(c, fsne::launch_scale(c->Y, c->V, c->N * c->DP, 1.0f / factor, c->stream));
  return FSNE_OK;
}

void fsne_destroy(fsne_ctx* c) {
  if (!c) return;
  release(c);
  delete c;
}

const char* fsne_last_error(const fsne_ctx* c) {
  if (!c) return kNoCtx;
  return c->err.c_str();
}

}  // extern "C"
