// Fixed device scratch of the allocation-free batch entry point
// (dd_batch_distance_fields_noalloc): one buffer per GPU, held until the
// process ends, whose device address is looked up once per device.
#include <mutex>

#include "dd_internal.h"

namespace dd {
namespace {

__device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

// Device address of this GPU's copy of the buffer.  `device` must be the
// current device.  The array's name is a host-side stand-in for the symbol;
// only the address returned here may be handed to kernels or copies.
hipError_t fixed_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices || !out) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace dd
