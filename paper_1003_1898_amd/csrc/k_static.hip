// The file-scope device array behind prng_generate_noalloc: scratch memory
// that exists on every GPU the library runs on from load to process end, so
// that the call needs no allocation.  Its host-side name is not a device
// address; host code uses only the address hipGetSymbolAddress returns, taken
// once per device with that device current and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace prng {
namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices || !out) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current first
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace prng
