// Fixed device scratch for the entry point that allocates nothing
// (rlb_record_current_noalloc): callers that cannot allocate device memory
// (code under graph capture, tight serving loops) get the per-row current
// buffer of rlb_record_current from a file-scope device array instead of a
// workspace argument.
//
// The array exists once per device and lives until the process ends.  Its
// device address is looked up once per device, with that device current,
// and only that address is handed to kernels: in host code the array's name
// is a host-side stand-in, not a device pointer.
#include <mutex>

#include "internal.hpp"

namespace rlb {
namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
double* g_ptr[kMaxDevices];   // device address of `scratch` per device (null: not looked up)

}  // namespace
}  // namespace rlb

static __device__ __align__(256) double scratch[rlb::kStaticScratchBytes / sizeof(double)];

namespace rlb {

hipError_t static_scratch(int device, double** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = (double*)p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace rlb
