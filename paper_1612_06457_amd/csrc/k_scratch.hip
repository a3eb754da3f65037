// Device scratch of fixed size for the entry point that allocates nothing
// (cva_project_noalloc): the projection passes' block partials, their
// ticket and the range slots live in one file-scope array per GPU instead
// of context buffers grown with hipMalloc.
//
// In host code the array's name is only a stand-in for the device symbol,
// so its device address is looked up once per device, with that device
// current, by scratch_setup (called when a context is made), and every
// launch takes that address.  Each GPU holds its own copy of the array
// until the process ends; every call on a GPU shares it, so calls that
// overlap on one GPU race.
#include <mutex>

#include "launch.hpp"

static __device__ __align__(256) unsigned char scratch[cvx::kScratchBytes];

namespace cvx {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_addr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_addr[device] = p;
  return hipSuccess;
}

void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_addr[device];
}

}  // namespace cvx
