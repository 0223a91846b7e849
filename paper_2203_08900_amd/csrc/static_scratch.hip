// A fixed device scratch area for the allocation-free division entry point.
//
// The array lives in the library's code object: each GPU the library runs on holds its
// own copy for the life of the process.  In host code its name is only a stand-in, so
// its device address is looked up once per device (with that device current) and
// cached; kernels receive that address like any caller workspace.  Every call on a GPU
// shares that GPU's copy and finds the previous call's contents in it: the division
// clears what it needs cleared (its failure flags) itself, and calls that overlap on one
// GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ps_internal.h"

namespace ps {

namespace {
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device (looked up on first use per
// device), or null if the lookup failed.
void* static_scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace ps
