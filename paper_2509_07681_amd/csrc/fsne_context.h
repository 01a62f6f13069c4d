// Internal definition of the library context (shared by the step and the
// placement-network sources; not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/fsne.h"
#include "fsne_kernels.h"

struct fsne_ctx {
  int64_t N = 0, cap = 0;
  int32_t D = 0, d = 0, DP = 0, Kh = 0, Kl = 0, xdtype = 0;
  uint64_t seed = 0;
  fsne_hparams hp{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* X = nullptr;
  bool own_X = false;
  float* xnorm = nullptr;
  float *Y = nullptr, *V = nullptr, *A = nullptr, *R = nullptr, *Zh = nullptr, *P = nullptr;
  float* zpart = nullptr;
  int32_t* fpart = nullptr;
  uint32_t* cpart = nullptr;
  uint8_t* ldc = nullptr;
  int32_t* hd_idx[2] = {nullptr, nullptr};
  float* hd_d2[2] = {nullptr, nullptr};
  int32_t* ld_idx[2] = {nullptr, nullptr};
  float4* rec = nullptr;
  float4* psh = nullptr;     // cap x 2: record and list cuts a refinement leaves for the affinity pass
  uint8_t* flags = nullptr;
  uint8_t* moved = nullptr;
  int32_t* memo = nullptr;   // cap x kMemo rejected HD candidates, -1 = empty
  float* Xu = nullptr;       // cap x D rows scaled to unit length (angular metric)
  uint8_t* rwork = nullptr;  // renumbering workspace (kept between calls)
  void* scratch = nullptr;   // device address of the library's fixed staging array
  // fsne_step's captured graph: gn iterations for the kernel arguments gargs
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  int32_t gn = 0;
  fsne::StepArgs gargs{};
  size_t rwork_bytes = 0;
  fsne::Scalars* sc = nullptr;
  std::string err;
  std::vector<void*> owned;
  // per-kernel timing (fsne_profile)
  bool prof = false;
  struct Timed {
    int kernel;
    hipEvent_t start, stop;
  };
  std::vector<Timed> pending;
  std::vector<hipEvent_t> spare;
  double ms[FSNE_NKERNELS] = {0};
  int64_t launches[FSNE_NKERNELS] = {0};
};

