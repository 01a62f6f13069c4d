// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsne_device.h"

namespace fsne {

// Rejected HD candidates remembered per point: a row of kMemo ids (the row
// stride), of which the first memo_w are used, the most recent first, -1 =
// empty; the valid entries are always a prefix.
constexpr int kMemo = 64;

// Everything a step kernel needs, passed by value as the kernel argument.
struct StepArgs {
  const void* X;            // N x D, float or bfloat16 bits (xdtype 0 / 1)
  const float* xnorm;       // N squared norms of the BF16 rows (BF16 screen only)
  int32_t xdtype, xvec_ok;  // xvec_ok: X base is 16-byte aligned
  int32_t N, D, d, DP, Kh, Kl;
  Hyper h;
  Scalars* sc;
  int32_t* hd_idx[2];
  float* hd_d2[2];
  int32_t* ld_idx[2];
  float4* rec;              // per point {beta, m, r, invS}
  // two per point, written by each HD refinement for the affinity pass that
  // follows it: the record, then the distances at ranks Kh/2-1, Kh/4-1,
  // 3Kh/4-1 of the new list (0 unless Kh is a multiple of 8) and 0
  float4* psh;
  float* P;                 // N x Kh
  uint8_t* flags;           // N
  float* Y;                 // N x DP
  float* V;                 // N x DP
  float* A;                 // N x DP
  float* R;                 // N x DP
  float* Zh;                // N
  float* zpart;             // kReduceBlocks
  int32_t* fpart;           // kReduceBlocks
  uint32_t* cpart;          // 2 x kReduceBlocks: candidate-row counts (HD, LD)
  uint8_t* ldc;             // N: LD candidate rows of each point in the last step
  int32_t* memo;            // N x kMemo rejected HD candidates (nullptr: not used)
  int32_t memo_w;           // entries of a row in use: 32 or 64
  float neg_scale;          // (N - 1) / n_neg
  int32_t hd_buf_host;      // HD buffer written by init / insert
  int32_t ld_buf_host;      // LD buffer written by init / insert
};

hipError_t launch_init_lists(const StepArgs& a, int32_t i0, int32_t n, hipStream_t s);
hipError_t launch_hd_refine(const StepArgs& a, hipStream_t s);
hipError_t launch_hd_refine_bf16(const StepArgs& a, hipStream_t s);
hipError_t launch_psym(const StepArgs& a, int standalone, hipStream_t s);
hipError_t launch_ld_grad(const StepArgs& a, hipStream_t s);
hipError_t launch_reduce(const StepArgs& a, hipStream_t s);
hipError_t launch_update(const StepArgs& a, hipStream_t s);
hipError_t launch_set_fire(Scalars* sc, const Hyper& h, hipStream_t s);
hipError_t launch_scale(float* Y, float* V, int64_t n, float inv, hipStream_t s);
hipError_t launch_calibrate_all(const StepArgs& a, hipStream_t s);
hipError_t launch_drift_rows(const StepArgs& a, const uint8_t* moved, hipStream_t s);
hipError_t launch_delete_fix(const StepArgs& a, const int32_t* newid, hipStream_t s);
hipError_t launch_move_rows(void* base, const int32_t* src, const int32_t* dst, int32_t m,
                            int32_t row_bytes, hipStream_t s);
hipError_t launch_xnorm(const StepArgs& a, float* xnorm, int32_t i0, int32_t n, hipStream_t s);
// Xu rows [i0, i0 + n) = X rows scaled to unit length (FP32), for the angular metric.
hipError_t launch_unit_rows(const void* X, int32_t xdtype, float* Xu, int32_t D, int32_t i0,
                            int32_t n, hipStream_t s);
hipError_t launch_scatter_rows(void* dst, const void* src, const int32_t* ids, int32_t n,
                               int32_t row_bytes, hipStream_t s);
hipError_t launch_mark_moved(uint8_t* moved, float* V, int32_t DP, const int32_t* ids, int32_t n,
                             hipStream_t s);
hipError_t launch_restride(float* dst, int dst_stride, const float* src, int src_stride,
                           int64_t n, int width, int zero_to, hipStream_t s);

}  // namespace fsne
