// Fixed device scratch for the entry point that allocates nothing
// (tk_functional_dev_noalloc): one file-scope array per device, whose address
// is looked up once per device when a context is created on it.
//
// Layout of the scratch (kScratchBytes):
//   [0, 4)      kernel error bits (int)
//   [8, 16)     jump-record counter (unsigned long long)
//   [64, 64+40) one jump-record slot (never written: the pass records nothing)
//   [512, ...)  tau_k, 2 doubles per trajectory
// Every call on a device shares its array and leaves its contents behind;
// calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tk_internal.h"

namespace tk {
namespace {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// zero the error bits and the record counter (a kernel rather than a memset,
// so the call stays usable where memset nodes are not)
__global__ void k_scratch_clear(unsigned char *base) {
  if (threadIdx.x == 0) {
    *reinterpret_cast<int *>(base + kScratchErrOffset) = 0;
    *reinterpret_cast<unsigned long long *>(base + kScratchCountOffset) = 0ull;
  }
}

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_ptr[device]) return hipSuccess;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if ((e = hipSetDevice(device)) != hipSuccess) return e;
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_ptr[device] = p;
  (void)hipSetDevice(cur);
  return e;
}

void *scratch_base(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mutex);
  return g_ptr[device];
}

hipError_t scratch_clear(void *base, hipStream_t stream) {
  void *args[] = {&base};
  return hipLaunchKernel(reinterpret_cast<const void *>(&k_scratch_clear), dim3(1), dim3(64),
                         args, 0, stream);
}

}  // namespace tk
