// The device scratch array of the allocation-free integration entry point.  Every GPU the library
// runs on holds its own copy of `scratch` (a file-scope device array, 48 MiB + 4352 B) from the
// loading of libchem.so to the end of the process.  Host code never uses the array's name as an
// address: scratch_address resolves the device address once per device with the device current
// and every user takes that address.
#include <mutex>

#include "noalloc.hpp"

static __device__ __align__(256) unsigned char scratch[chem_noalloc::kBytes];

namespace chem_noalloc {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices || !out) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}
}  // namespace chem_noalloc
