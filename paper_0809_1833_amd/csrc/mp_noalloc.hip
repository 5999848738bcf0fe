// The static scratch behind mp_solve_noalloc: device memory the library holds
// for callers that cannot allocate (code under stream capture, serving loops,
// harnesses that forbid allocation), and its per-device address.
//
// The array is a file-scope device variable: each GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): noalloc_scratch() looks up the device address
// once per device, with that device current, and every user takes that.
#include <mutex>

#include "mp_internal.h"

static_assert(mp::kNoAllocBal + sizeof(mp::BalState) <= mp::kNoAllocScratchBytes,
              "the scratch layout overruns the array");
static_assert(mp::kNoAllocBal % alignof(mp::BalState) == 0 && mp::kNoAllocKeys % 8 == 0 &&
                  mp::kNoAllocR % 16 == 0 && sizeof(mp::DevState) <= mp::kNoAllocR,
              "scratch regions misaligned or overlapping");

static __device__ __align__(256) unsigned char scratch[mp::kNoAllocScratchBytes];

namespace mp {
namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();  // leave no error behind for the next launch check
      return e;
    }
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace mp
