// sdq_noalloc.hip -- the fixed device scratch behind sdq_greens_noalloc
// (include/sdq.h): one statically sized array per device, so that the entry
// point never allocates.  Its device address is looked up once per device
// when a context is created on it (sdq_create, with that device current) and
// kept; host code never uses the array's name as an address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sdq_internal.h"

namespace sdq {
namespace {

// kNoAllocBytes of device memory on every GPU the library runs on, held until
// the process ends; every sdq_greens_noalloc call on a device shares it.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_ptr[kNoAllocMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= kNoAllocMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace sdq
