// The no-allocation array behind mfa_create_noalloc: a file-scope device
// array that serves as the workspace of a handle for callers that cannot
// allocate device memory.  Each device the library runs on holds its own
// copy (MFA_NOALLOC_MAX_BYTES) from the time the code object is loaded there
// until the process ends.
//
// In host code `scratch` names a host-side stand-in, not the device copy:
// its device address is looked up once per device with hipGetSymbolAddress,
// with that device current, and only that address is ever handed to kernels
// or copies.
#include <mutex>

#include "mfa_internal.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[MFA_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;

struct DeviceArray {
  void *ptr = nullptr;   // device address of this device's copy of `scratch`
  uint64_t gen = 0;      // last generation handed out (0: never claimed)
};

std::mutex g_mu;
DeviceArray g_dev[kMaxDevices];

}  // namespace

namespace mfa {

hipError_t noalloc_scratch(void **ptr, uint64_t *gen) {
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceArray &d = g_dev[device];
  if (!d.ptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidSymbol;
    d.ptr = p;
  }
  *ptr = d.ptr;
  *gen = ++d.gen;
  return hipSuccess;
}

uint64_t noalloc_current(int device) {
  if (device < 0 || device >= kMaxDevices) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_dev[device].gen;
}

}  // namespace mfa
