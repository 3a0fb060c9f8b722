// fwi_gradient_noalloc: the probed FWI gradient of fwi_gradient for callers
// that cannot allocate device memory.  The workspace (level ring, reduction
// partials, non-finite watch word, point tables) is a file-scope static
// device array of RTM_NOALLOC_SCRATCH_BYTES that every GPU the library runs
// on holds from the first call until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (that
// device current) and only that address is handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rtm.h"

namespace rtm {
rtm_status note_error(rtm_status s, const char *msg);  // rtm.cpp: sets rtm_last_error
}

namespace {
constexpr size_t kScratchBytes = RTM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device, or NULL
std::mutex g_scratch_mu;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's copy of `scratch` (looked up on first use).
static rtm_status scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rtm::note_error(RTM_E_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return rtm::note_error(RTM_E_UNSUPPORTED, "fwi_gradient_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return rtm::note_error(RTM_E_HIP, e != hipSuccess ? hipGetErrorString(e)
                                                         : "hipGetSymbolAddress gave NULL");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RTM_OK;
}

extern "C" rtm_status fwi_gradient_noalloc(const rtm_plan *plan, const void *m,
                                           const double *src_pos, const void *q,
                                           const double *rec_pos, const void *d_obs,
                                           const void *Z, rtm_dtype z_dtype, void *Ubar,
                                           void *Vbar, void *resid, void *grad, double *misfit,
                                           rtm_stream stream) {
  if (!plan) return rtm::note_error(RTM_E_ARG, "plan is NULL");
  size_t need = 0;
  rtm_status s = rtm_plan_workspace_bytes(plan, &need);
  if (s) return s;
  if (need > kScratchBytes) {
    char msg[256];
    snprintf(msg, sizeof msg,
             "fwi_gradient_noalloc: the plan needs %zu bytes of workspace, above the static "
             "limit of %zu bytes (use fwi_gradient with a caller-owned workspace)",
             need, kScratchBytes);
    return rtm::note_error(RTM_E_WORKSPACE, msg);
  }
  void *work = nullptr;
  if ((s = scratch_address(&work))) return s;
  return fwi_gradient(plan, m, src_pos, q, rec_pos, d_obs, Z, z_dtype, Ubar, Vbar, resid, grad,
                      misfit, work, kScratchBytes, stream);
}
