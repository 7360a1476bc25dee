// scratch.hip -- the fixed device scratch array of the allocation-free entry
// point pic_fields_static, and the per-device address of that array.
//
// The array is a file-scope __device__ symbol: the runtime places one copy on
// every GPU the library's code object is loaded on, for the life of the
// process.  Host code must not pass the symbol's name to a kernel (in host
// code it names a host-side stand-in); it uses the address that
// hipGetSymbolAddress returns for the current device, kept per device here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"

namespace pic {

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};
}  // namespace

// Resolves the array's address on the current device once; later calls for
// the same device return the kept address.
int scratch_setup(int* device_out, void** addr_out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -2;
    g_scratch_addr[dev] = p;
  }
  if (device_out) *device_out = dev;
  if (addr_out) *addr_out = g_scratch_addr[dev];
  return 0;
}

void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_addr[device];
}

}  // namespace pic
