// Static device scratch of the allocation-free entry points (nlos_fk_noalloc).
//
// One file-scope device array per GPU, held from the first use of the library on that
// GPU until the process ends.  Host code never passes the array's name to a kernel: in
// host code the name is only a stand-in for the symbol, so its device address is looked
// up once per device, with that device current, and that address is what the kernels get.
#include <mutex>

#include "nlos.h"
#include "nlos_internal.hpp"

namespace nlos {

static_assert(kStaticScratchBytes == NLOS_STATIC_SCRATCH_BYTES, "one size in the header and here");
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[device] == nullptr) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (p == nullptr || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace nlos
