// The aggregation + disaggregation pass for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation): fmm_tucker_pass on the streaming kernels, with the partial sums of
// split items in a file-scope device array instead of a library allocation.
//
// Every GPU the library runs on holds its own copy of `scratch` (kScratchBytes) from
// the module's load until the process ends.  Host code never passes the array's name
// to a kernel: the address of this device's copy comes from hipGetSymbolAddress,
// taken once per device at the entry point's first call with that device current,
// and only that address is used.  All calls on one GPU share the array and it keeps
// the last call's contents; the kernels overwrite every partial-sum block they read,
// so nothing needs clearing, but calls that overlap on one GPU (two streams, two
// threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

using namespace tuckfmm;

extern "C" fmm_status fmm_tucker_pass_noalloc(fmm_tucker_t h, fmm_prec prec, int32_t nrhs, const void* x, void* F,
                                              const void* G, void* V, void* stream) {
  clear_error();
  if (!h) return fail(FMM_ERR_ARG, "handle is NULL");
  if (!have_device()) return FMM_ERR_DEVICE;
  int dev = 0;
  TFMM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FMM_ERR_DEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || p == nullptr)
        return fail(FMM_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      g_scratch[dev] = p;
    }
    ptr = g_scratch[dev];
  }
  return noalloc_pass(h, prec, nrhs, x, F, G, V, static_cast<hipStream_t>(stream), ptr, kScratchBytes);
}
