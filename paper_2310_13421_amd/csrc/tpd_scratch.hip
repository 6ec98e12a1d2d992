// tpd_scratch.hip -- the device scratch of tpd_decompose_noalloc.
//
// The pruning bitmap of the no-allocation entry point lives in a file-scope
// static device array instead of a workspace, so that entry point never
// calls hipMalloc.  Each device the library runs on holds its own copy of
// the array until the process ends; in host code its name is only a
// stand-in, so its device address is looked up here, once per device with
// that device current, and that address is what kernels receive.
#include <map>
#include <mutex>

#include "tpd_internal.h"

namespace tpd {

namespace {
static __device__ __align__(256) uint32_t scratch[kNoallocScratchWords];
std::mutex g_mu;
std::map<int, uint32_t*> g_addr;  // device -> address of its copy of `scratch`
}  // namespace

hipError_t noalloc_scratch(int dev, uint32_t** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_addr.find(dev);
  if (it == g_addr.end()) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != dev) return hipErrorInvalidDevice;
    uint32_t* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    it = g_addr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return hipSuccess;
}

}  // namespace tpd
