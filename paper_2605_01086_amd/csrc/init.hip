// Per-device set-up of the library: done once per device, under a lock, by
// fptc_init or by the first device call made with that device current.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "fptc_internal.h"

namespace fptc {

namespace {

struct DeviceState {
  bool done = false;
  int rc = 0;
};

std::mutex g_init_mu;
std::vector<DeviceState> g_dev;

int init_current_device() {
  (void)device_cu_count();  // cache the compute-unit count the launchers size grids by
  int rc = set_decode_attributes() | set_dqidct_mfma_attributes() | set_fused_attributes() |
           set_mfma256_attributes() | set_bwd_attributes() | (init_noalloc_scratch() ? 1 : 0);
  return rc ? (int)hipErrorInvalidValue : 0;
}

}  // namespace

int ensure_device_init() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return (int)hipErrorNoDevice;
  std::lock_guard<std::mutex> g(g_init_mu);
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  DeviceState &st = g_dev[dev];
  if (!st.done) {
    st.rc = init_current_device();
    st.done = true;
  }
  return st.rc;
}

}  // namespace fptc
