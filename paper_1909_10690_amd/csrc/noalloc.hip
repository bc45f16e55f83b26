// Fixed device scratch of the allocation-free entry point (mi_eval_noalloc):
// a file-scope device array that every GPU the library runs on holds, at
// its own address, until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it looks up each device's address once, with that device
// current, and hands that address to the kernels as it would a caller's
// workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/gemi.h"

namespace gemi {

namespace {

static __device__ __align__(256) unsigned char scratch[MI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

}  // namespace

// Looks up the address of the scratch array on `device`, which must be the
// current device.  Idempotent; called by mi_create.
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

// The device address of the scratch array on `device`, or NULL before
// scratch_setup() succeeded there.
void* scratch_device_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace gemi
