// Small bookkeeping kernels of the solve (independent of the block size).
#include <hip/hip_runtime.h>

#include "smnn_internal.h"

namespace smnn {
namespace {

// Sum the per-chunk weight-gradient partials of each instance, in an order
// that does not depend on scheduling: `split` workgroups per instance, each
// summing one contiguous slice of the instance's chunks (strided per-thread
// sums, then a fixed-shape tree in LDS).  With split == 1 the workgroup
// writes the instance's result; otherwise its slice sum goes to `part` and
// k_dw_final adds the slices of an instance in order.  (One workgroup per
// instance left a batch of a few long instances on a few CUs, each summing
// ~10^5 chunks.)
template <class TIO>
__global__ void __launch_bounds__(256) k_dw_reduce(LevelDev l0, Level0Args a, int split, double* part) {
  __shared__ double sum[3][256];
  const int64_t i = blockIdx.x / split;
  const int p = static_cast<int>(blockIdx.x % split);
  const int tid = threadIdx.x;
  const int64_t c0 = l0.chunk_off[i], c1 = l0.chunk_off[i + 1];
  const int64_t span = (c1 - c0 + split - 1) / split;
  const int64_t lo = c0 + p * span, hi = lo + span < c1 ? lo + span : c1;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t g = lo + tid; g < hi; g += 256)
#pragma unroll
    for (int e = 0; e < 3; ++e) acc[e] += a.dw_part[g * 3 + e];
#pragma unroll
  for (int e = 0; e < 3; ++e) sum[e][tid] = acc[e];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int e = 0; e < 3; ++e) sum[e][tid] += sum[e][tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    if (split == 1) {
      TIO* dw = static_cast<TIO*>(a.dw);
#pragma unroll
      for (int e = 0; e < 3; ++e) dw[i * 3 + e] = static_cast<TIO>(sum[e][0]);
    } else {
#pragma unroll
      for (int e = 0; e < 3; ++e) part[blockIdx.x * 3 + e] = sum[e][0];
    }
  }
}

template <class TIO>
__global__ void k_dw_final(Level0Args a, int split, const double* part) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  TIO* dw = static_cast<TIO*>(a.dw);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    double t = 0.0;
    for (int p = 0; p < split; ++p) t += part[(i * split + p) * 3 + e];
    dw[i * 3 + e] = static_cast<TIO>(t);
  }
}

__global__ void k_info_init(uint32_t* info, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < N) info[i] = 0xFFFFFFFFu;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t value) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ void k_info_finalize(const uint32_t* ws, int32_t* info, int64_t N) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  // 1 + the failing step, saturated at INT32_MAX for steps beyond it
  if (i < N) info[i] = ws[i] == 0xFFFFFFFFu ? 0 : static_cast<int32_t>(ws[i] > 0x7FFFFFFFu ? 0x7FFFFFFFu : ws[i]);
}

}  // namespace

hipError_t launch_dw_reduce(bool f32, const LevelDev& l0, const Level0Args& a, int split, double* part,
                            hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(a.N * split)), block(256);
  if (f32) hipLaunchKernelGGL(k_dw_reduce<float>, grid, block, 0, st, l0, a, split, part);
  else hipLaunchKernelGGL(k_dw_reduce<double>, grid, block, 0, st, l0, a, split, part);
  if (split > 1) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2(static_cast<unsigned>((a.N + 63) / 64)), b2(64);
    if (f32) hipLaunchKernelGGL(k_dw_final<float>, g2, b2, 0, st, a, split, part);
    else hipLaunchKernelGGL(k_dw_final<double>, g2, b2, 0, st, a, split, part);
  }
  return hipGetLastError();
}

hipError_t launch_info_init(const Level0Args& a, hipStream_t st) {
  if (!a.info) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((a.N + 255) / 256)), block(256);
  hipLaunchKernelGGL(k_info_init, grid, block, 0, st, a.info, a.N);
  return hipGetLastError();
}

// A fill kernel (not a memset node) so that the call stays capturable.
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
  hipLaunchKernelGGL(k_fill_u32, grid, block, 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_info_finalize(const Level0Args& a, int32_t* info, hipStream_t st) {
  if (!a.info || !info) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((a.N + 255) / 256)), block(256);
  hipLaunchKernelGGL(k_info_finalize, grid, block, 0, st, a.info, info, a.N);
  return hipGetLastError();
}

// Dispatch on the block size (and, at level 0, the instance form) to the
// translation units of smnn_kernels.hip: _k<K> holds the separator levels
// and the scalar form, _k<K>f1 per-row weights, _k4f2 two coupled variables.
#define SMNN_DECL0(SUF)                                                                                 \
  bool supported0_##SUF(int, int, int);                                                                 \
  hipError_t launch_reduce0_##SUF(int, int, int, bool, int, bool, const LevelDev&, const LevelDev&,      \
                                  const Level0Args&, const Launch&, hipStream_t);                        \
  hipError_t launch_backsub0_##SUF(int, int, int, bool, int, int, const LevelDev&, const LevelDev*,      \
                                   const Level0Args&, const Launch&, hipStream_t);                       \
  size_t level0_lds_bytes_##SUF(int, int, int, bool, int, int);                                           \
  hipError_t launch_backsub_reduce0_##SUF(int, int, int, bool, int, const LevelDev&, const LevelDev&,     \
                                          const Level0Args&, const Launch&, hipStream_t);
#define SMNN_DECL(KV)                                                                                   \
  SMNN_DECL0(k##KV)                                                                                     \
  SMNN_DECL0(k##KV##f1)                                                                                 \
  bool supported_k##KV(int, int);                                                                       \
  hipError_t launch_reduceN_k##KV(int, int, bool, int, const LevelDev&, const LevelDev&, const Level0Args&, \
                                  const Launch&, hipStream_t);                                           \
  hipError_t launch_backsubN_k##KV(int, int, int, const LevelDev&, const LevelDev*, const Level0Args&,    \
                                   const Launch&, hipStream_t);                                          \
  size_t top_lds_bytes_k##KV(int, int);                                                                   \
  hipError_t launch_top_k##KV(int, int, int, const LevelDev&, const Level0Args&, const Launch&, hipStream_t);
SMNN_DECL(2)
SMNN_DECL(3)
SMNN_DECL(4)
SMNN_DECL(5)
SMNN_DECL0(k4f2)
#undef SMNN_DECL
#undef SMNN_DECL0

#define SMNN_SWITCH(FN, ...)                     \
  switch (K) {                                   \
    case 2: return FN##_k2(__VA_ARGS__);         \
    case 3: return FN##_k3(__VA_ARGS__);         \
    case 4: return FN##_k4(__VA_ARGS__);         \
    case 5: return FN##_k5(__VA_ARGS__);         \
  }

// level-0 functions: by form group, then block size
#define SMNN_SWITCH0(FN, ...)                                          \
  if (form == SMNN_FORM_SCALAR) {                                      \
    SMNN_SWITCH(FN, __VA_ARGS__)                                       \
  } else if (form == SMNN_FORM_ROWS) {                                 \
    switch (K) {                                                       \
      case 2: return FN##_k2f1(__VA_ARGS__);                           \
      case 3: return FN##_k3f1(__VA_ARGS__);                           \
      case 4: return FN##_k4f1(__VA_ARGS__);                           \
      case 5: return FN##_k5f1(__VA_ARGS__);                           \
    }                                                                  \
  } else if (K == 4) {                                                 \
    return FN##_k4f2(__VA_ARGS__);                                     \
  }

// wide blocks (smnn_wide.hip, one translation unit per K)
#define SMNN_DECLW(KV)                                                                                      \
  bool wide_supported_w##KV(int, int, int);                                                                 \
  hipError_t launch_wreduce0_w##KV(int, int, int, bool, int, bool, const LevelDev&, const LevelDev&,         \
                                   const Level0Args&, const Launch&, hipStream_t);                           \
  hipError_t launch_wbacksub0_w##KV(int, int, int, bool, int, int, const LevelDev&, const LevelDev*,         \
                                    const Level0Args&, const Launch&, hipStream_t);                          \
  hipError_t launch_wreduceN_w##KV(int, int, bool, int, const LevelDev&, const LevelDev&, const Level0Args&, \
                                   const Launch&, hipStream_t);                                              \
  hipError_t launch_wbacksubN_w##KV(int, int, int, const LevelDev&, const LevelDev*, const Level0Args&,      \
                                    const Launch&, hipStream_t);
SMNN_DECLW(6)
SMNN_DECLW(9)
#undef SMNN_DECLW

#define SMNN_SWITCHW(FN, ...)                    \
  switch (K) {                                   \
    case 6: return FN##_w6(__VA_ARGS__);         \
    case 9: return FN##_w9(__VA_ARGS__);         \
  }

bool wide_supported(int K, int L, int form) {
  SMNN_SWITCHW(wide_supported, K, L, form)
  return false;
}

hipError_t launch_wreduce0(int K, int L, int form, bool f32, int rhs_mode, bool write_rec, const LevelDev& l0,
                           const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCHW(launch_wreduce0, K, L, form, f32, rhs_mode, write_rec, l0, l1, a, cfg, st)
  return hipErrorInvalidValue;
}

hipError_t launch_wbacksub0(int K, int L, int form, bool f32, int rhs_mode, int out_mode, const LevelDev& l0,
                            const LevelDev* l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCHW(launch_wbacksub0, K, L, form, f32, rhs_mode, out_mode, l0, l1, a, cfg, st)
  return hipErrorInvalidValue;
}

hipError_t launch_wreduceN(int K, int L, bool write_rec, int level, const LevelDev& l, const LevelDev& lnext,
                           const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCHW(launch_wreduceN, K, L, write_rec, level, l, lnext, a, cfg, st)
  return hipErrorInvalidValue;
}

hipError_t launch_wbacksubN(int K, int L, int level, const LevelDev& l, const LevelDev* lnext,
                            const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCHW(launch_wbacksubN, K, L, level, l, lnext, a, cfg, st)
  return hipErrorInvalidValue;
}

bool supported(int K, int L) {
  SMNN_SWITCH(supported, K, L)
  return false;
}

bool supported0(int K, int L, int form) {
  SMNN_SWITCH0(supported0, K, L, form)
  return false;
}

size_t level0_lds_bytes(int K, int L, int form, bool f32, int rhs_mode, int out_mode) {
  SMNN_SWITCH0(level0_lds_bytes, K, L, form, f32, rhs_mode, out_mode)
  return 0;
}

hipError_t launch_reduce0(int K, int L, int form, bool f32, int rhs_mode, bool write_rec, const LevelDev& l0,
                          const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCH0(launch_reduce0, K, L, form, f32, rhs_mode, write_rec, l0, l1, a, cfg, st)
  return hipErrorInvalidValue;
}

hipError_t launch_backsub0(int K, int L, int form, bool f32, int rhs_mode, int out_mode, const LevelDev& l0,
                           const LevelDev* l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCH0(launch_backsub0, K, L, form, f32, rhs_mode, out_mode, l0, l1, a, cfg, st)
  return hipErrorInvalidValue;
}

hipError_t launch_backsub_reduce0(int K, int L, int form, bool f32, int rhs_in, const LevelDev& l0,
                                  const LevelDev& l1, const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCH0(launch_backsub_reduce0, K, L, form, f32, rhs_in, l0, l1, a, cfg, st)
  return hipErrorInvalidValue;
}

hipError_t launch_reduceN(int K, int L, bool write_rec, int level, const LevelDev& l, const LevelDev& lnext,
                          const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCH(launch_reduceN, K, L, write_rec, level, l, lnext, a, cfg, st)
  return hipErrorInvalidValue;
}

hipError_t launch_backsubN(int K, int L, int level, const LevelDev& l, const LevelDev* lnext,
                           const Level0Args& a, const Launch& cfg, hipStream_t st) {
  SMNN_SWITCH(launch_backsubN, K, L, level, l, lnext, a, cfg, st)
  return hipErrorInvalidValue;
}

size_t top_lds_bytes(int K, int L) {
  SMNN_SWITCH(top_lds_bytes, K, L)
  return 0;
}

hipError_t launch_top(int K, int L, int level, const LevelDev& l, const Level0Args& a, const Launch& cfg,
                      hipStream_t st) {
  SMNN_SWITCH(launch_top, K, L, level, l, a, cfg, st)
  return hipErrorInvalidValue;
}

}  // namespace smnn
