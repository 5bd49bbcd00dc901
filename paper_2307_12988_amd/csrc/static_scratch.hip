// Fixed device scratch for the entry point that allocates nothing
// (cg_process_batch_static): a file-scope device array that the code object
// carries, so each GPU the library runs on holds its own copy from module
// load until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): its device
// address is resolved once per device with hipGetSymbolAddress, with that
// device current, when a plan is created there, and kept per device.
#include <mutex>

#include "internal.h"

namespace cg {
namespace {

static __device__ __align__(256) unsigned char scratch[CG_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t resolve_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_ptr[device] = ptr;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace cg
