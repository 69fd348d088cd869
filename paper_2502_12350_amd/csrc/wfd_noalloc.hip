// wfd_forward_noalloc: forward modeling with the library's own static device
// scratch instead of a caller workspace, for callers that cannot allocate
// device memory.  The scratch is one file-scope __device__ array per GPU
// (each device that loads the library holds its own copy until the process
// ends); its device address is looked up once per device with that device
// current, and only that address is handed to the kernels.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "wfd.h"
#include "wfd_internal.h"

namespace {

constexpr size_t kScratchBytes = WFD_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

// The scratch array.  In host code its name is a host-side stand-in, not a
// device address: it is never passed to a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of `device`'s copy of the scratch array.
wfd_status scratch_of(int device, void **out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (device < 0 || device >= kMaxDevices)
    return wfd::set_error(WFD_E_ARG, "device index out of the scratch table's range");
  if (!g_scratch[device]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != device && hipSetDevice(device) != hipSuccess)
      return wfd::set_error(WFD_E_HIP, "hipSetDevice failed while locating the scratch array");
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
      char msg[160];
      std::snprintf(msg, sizeof(msg), "hipGetSymbolAddress(scratch) failed: %s",
                    hipGetErrorString(e));
      return wfd::set_error(WFD_E_HIP, msg);
    }
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return WFD_OK;
}

}  // namespace

extern "C" wfd_status wfd_forward_noalloc(wfd_ctx *ctx, const float *wavelet_dev,
                                          const double src_xyz[3], int32_t nrec,
                                          const double *rec_xyz, float *seis_dev,
                                          float *final_dev_or_null) {
  if (!ctx) return wfd::set_error(WFD_E_ARG, "ctx is NULL");
  size_t need = 0;
  wfd_status s = wfd_workspace_bytes(ctx, nrec, nullptr, &need);
  if (s != WFD_OK) return s;
  if (need > kScratchBytes) {
    char msg[200];
    std::snprintf(msg, sizeof(msg),
                  "this shot needs %zu bytes of workspace; the static scratch holds %zu "
                  "(use wfd_forward with a caller workspace)",
                  need, kScratchBytes);
    return wfd::set_error(WFD_E_NOMEM, msg);
  }
  void *work = nullptr;
  if ((s = scratch_of(wfd::ctx_device(ctx), &work)) != WFD_OK) return s;
  return wfd_forward(ctx, wavelet_dev, src_xyz, nrec, rec_xyz, seis_dev, final_dev_or_null, work,
                     kScratchBytes);
}
