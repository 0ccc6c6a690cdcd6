// The library's static device scratch: one file-scope device array that
// serves as the workspace of the entry points that take none (for callers
// that cannot allocate device memory, such as code under graph capture or a
// serving loop).  Every device the library runs on holds its own copy, at its
// own address, until the process ends.  In host code the array's name is not
// a device address: the address is taken once per device, with that device
// current, and only that address is used afterwards.
#include <mutex>

#include "qcur_internal.hpp"

namespace qcur {

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_addr[MAX_DEVICES];
}  // namespace

hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_addr[device] = p;
  }
  *out = scratch_addr[device];
  return hipSuccess;
}

}  // namespace qcur
