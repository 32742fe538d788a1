// A plan workspace that the caller does not allocate: a fixed array in the
// library's own device memory, for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid
// it).  Each device that loads the library holds one copy of the array
// until the process ends.  One plan at a time keeps its tables there: the
// newest plan attached on a device takes the array over, and the earlier
// holder's calls return DT_E_WORKSPACE from then on.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "dt.h"
#include "dt_static.hpp"

namespace {

constexpr size_t kStaticBytes = DT_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

// The fixed workspace.  In host code this name is only a stand-in for the
// symbol: kernels receive the device address obtained below.
static __device__ __align__(256) char scratch[kStaticBytes];

std::mutex g_mu;                               // serialises set-up of the array
void* g_ptr[kMaxDevices] = {};                 // device address of scratch, per device
std::atomic<uint64_t> g_owner[kMaxDevices];    // token of the plan holding it (0: none)
uint64_t g_next_token = 1;

// Device address of the array on `dev` (the current device), looked up once.
dt_status device_ptr(int dev, void** out) {
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DT_E_HIP;
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return DT_OK;
}

}  // namespace

uint64_t dt::static_ws_owner(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return 0;
  return g_owner[dev].load(std::memory_order_acquire);
}

void dt::static_ws_release(int dev, uint64_t token) {
  if (dev < 0 || dev >= kMaxDevices || token == 0) return;
  uint64_t expect = token;
  g_owner[dev].compare_exchange_strong(expect, 0, std::memory_order_acq_rel);
}

extern "C" dt_status dt_plan_set_static_workspace(dt_plan plan, void* stream) {
  if (!plan) return DT_E_ARG;
  size_t need = 0;
  dt_status s = dt_plan_workspace_size(plan, &need);
  if (s != DT_OK) return s;
  if (need > kStaticBytes) return DT_E_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DT_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return DT_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  void* ptr = nullptr;
  s = device_ptr(dev, &ptr);
  if (s != DT_OK) return s;
  // Work of the previous holder may still be in flight on another stream:
  // wait for the device before its tables are overwritten.
  const uint64_t prev = g_owner[dev].load(std::memory_order_acquire);
  const uint64_t token = g_next_token++;
  g_owner[dev].store(token, std::memory_order_release);
  if (prev != 0 && hipDeviceSynchronize() != hipSuccess) {
    g_owner[dev].store(0, std::memory_order_release);
    return DT_E_HIP;
  }
  s = dt::plan_attach(plan, ptr, need, stream);
  if (s != DT_OK) {
    g_owner[dev].store(0, std::memory_order_release);
    return s;
  }
  dt::plan_mark_static(plan, dev, token);
  return DT_OK;
}
