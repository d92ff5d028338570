// Batch decompression for callers that cannot allocate device memory: the
// plan lives in a static device array of the library instead of a workspace
// the caller passes in.
//
// Each GPU holds its own copy of `scratch` (reserved while the library is
// loaded).  In host code the array's name stands for a host-side shadow, not
// a device address, so host code only ever uses the address that
// hipGetSymbolAddress returns for the current device, taken once per device
// when the library sets the device up.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "fptc_internal.h"

namespace fptc {

namespace {

constexpr size_t kScratchBytes = (size_t)FPTC_NOALLOC_WS_BYTES;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::vector<void *> g_ptr;  // per device: scratch's device address, null until set up

}  // namespace

// Record scratch's address on the current device (called once per device
// from the library's device set-up, with that device current).
int init_noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return (int)hipErrorNoDevice;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return e != hipSuccess ? (int)e : (int)hipErrorInvalidSymbol;
  std::lock_guard<std::mutex> g(g_mu);
  if ((int)g_ptr.size() <= dev) g_ptr.resize(dev + 1, nullptr);
  g_ptr[dev] = p;
  return 0;
}

void *noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return dev < (int)g_ptr.size() ? g_ptr[dev] : nullptr;
}

}  // namespace fptc

using namespace fptc;

extern "C" {

int32_t fptc_decompress_batch_noalloc(const fptc_batch *batch, const fptc_codec *codec, const fptc_launch *launch,
                                      const float *gamma, int32_t precision, float *out, int32_t *stream_status,
                                      void *stream) {
  // every check first: an error return enqueues nothing
  Shape s;
  const int rc = check_decompress(batch, codec, launch, precision, out, &s);
  if (rc) return rc;
  const Layout L = layout_for(batch, codec, s);
  if (L.total > kScratchBytes) return FPTC_ERR_WORKSPACE;
  if (ensure_device_init()) return FPTC_ERR_HIP;
  void *ws = noalloc_scratch();
  if (!ws) return FPTC_ERR_HIP;
  // the plan writes every part of the workspace the decode reads, so nothing
  // of an earlier call's contents is used
  const Plan p = plan_view(ws, L);
  const int prc = launch_plan_status(*batch, *codec, s, p, stream_status, stream);
  if (prc != FPTC_OK) return prc;
  return launch_decompress(*batch, *codec, s, p, gamma, precision, out, stream_status, stream);
}

}  // extern "C"
