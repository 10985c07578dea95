// Device-resident workspace of the allocation-free forward entry point
// (cm_collide_noalloc).  The array lives in the library's code object, so each
// device the library runs on holds one copy from module load until the
// process ends; its device address is looked up once per device, at context
// creation, and host code only ever uses that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cm_kernels.h"

static __device__ __align__(256) unsigned char scratch[CM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_looked_up[kMaxDevices] = {};
hipError_t g_rc[kMaxDevices] = {};
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace cm {

hipError_t noalloc_scratch(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_looked_up[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    if (e == hipSuccess) e = hipGetSymbolAddress(&g_ptr[device], HIP_SYMBOL(scratch));
    if (e != hipSuccess) g_ptr[device] = nullptr;
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    g_rc[device] = e;
    g_looked_up[device] = true;
  }
  *out = g_ptr[device];
  return g_rc[device];
}

}  // namespace cm
