// smnn_forward_noalloc: the forward solve with its workspace in a static
// device array of the library, for callers that cannot allocate device
// memory (code under hipGraph capture, tight serving loops, harnesses that
// forbid hipMalloc).  It runs the same kernels as smnn_forward.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/smnn.h"

namespace {

// The workspace of every smnn_forward_noalloc call on a device.  Each device
// the library runs on holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[SMNN_NOALLOC_WORKSPACE_MAX];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per
// device; the symbol's host-side name is not a device address).
smnn_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return SMNN_ERR_UNSUPPORTED;
  std::call_once(g_once[dev], [dev] {
    void* p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_err[dev] != hipSuccess || !g_ptr[dev]) return SMNN_ERR_HIP;
  *out = g_ptr[dev];
  return SMNN_OK;
}

}  // namespace

extern "C" smnn_status smnn_forward_noalloc(const smnn_plan* plan, const void* c, const void* b, const void* h,
                                            const void* u0, const void* w, void* y, void* factor,
                                            size_t factor_bytes, int32_t* info, void* stream) {
  if (!plan) return SMNN_ERR_INVALID_ARG;
  size_t need = 0;
  const smnn_status s = smnn_plan_sizes(plan, nullptr, &need, nullptr);
  if (s != SMNN_OK) return s;
  if (need > SMNN_NOALLOC_WORKSPACE_MAX) return SMNN_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SMNN_ERR_HIP;
  void* ws = nullptr;
  const smnn_status sa = scratch_address(dev, &ws);
  if (sa != SMNN_OK) return sa;
  // smnn_forward checks the plan's device, the factor and the arguments,
  // initialises every workspace word it reads before reading it, and
  // allocates nothing.
  return smnn_forward(plan, c, b, h, u0, w, y, factor, factor_bytes, ws, SMNN_NOALLOC_WORKSPACE_MAX, info, stream);
}
