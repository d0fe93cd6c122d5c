// Fixed device scratch for the allocation-free entry points.
//
// One file-scope device array per GPU the library runs on, held until the
// process ends. Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): its device address is looked
// up once per device, with that device current, when a context is created
// there, and kept in a per-device table. Every allocation-free call on a
// device shares that device's array, so such calls that overlap on one GPU
// race with each other.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "vrph_internal.h"

namespace vrph {

static __device__ __align__(256) uint32_t scratch[kNoAllocScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = static_cast<uint32_t*>(p);
  return hipSuccess;
}

uint32_t* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace vrph
