// noalloc.hip -- the inclusive scan for callers that cannot allocate (code
// under HIP graph capture, tight serving loops, hosts that forbid
// hipMalloc): its look-back state lives in a fixed array in device memory
// instead of a caller's workspace.
//
// `scratch` holds the scan's workspace (a 64-byte header and one status word
// per tile) for up to kNoAllocMaxN elements.  Each GPU the library runs on
// has its own copy, for the life of the process.  In host code the array's
// name is not a device address, so its address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to kernels.  The first call on a device also clears the array with
// a fill kernel on the call's stream (the scan's state must start at zero;
// after that every call leaves it ready for the next).  All calls on one GPU
// share the array: calls that overlap in time race, as calls sharing one
// workspace do.
#include <atomic>
#include <mutex>

#include "common.hpp"
#include "launch.hpp"

namespace desc {
namespace {

constexpr int64_t kNoAllocMaxN = int64_t(1) << 31;
// header + one status word per tile of the smallest scan tile (8192)
constexpr size_t kScratchBytes = 64 + 8 * (size_t)(kNoAllocMaxN / 8192);
static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_setup;
std::atomic<void*> g_scratch[kMaxDevices];

constexpr int kClearBlock = 256;
__global__ __launch_bounds__(kClearBlock) void clear_scratch_kernel(uint64_t* __restrict__ w,
                                                                    int64_t nwords) {
  auto words = array(w, nwords);
  for (idx_t i = block_x().index() * kClearBlock + thread_x<kClearBlock>().index(); i < nwords;
       i += block_x().count() * kClearBlock)
    words[i] = 0;
}

}  // namespace

namespace launch {

int64_t scan_noalloc_max_n() { return kNoAllocMaxN; }

// The scratch array's device address on the device of `s`, set up on the
// first call there.
hipError_t noalloc_scratch(hipStream_t s, void** out, size_t* bytes) {
  *out = nullptr;
  *bytes = kScratchBytes;
  int dev = 0;
  hipError_t e = s == nullptr ? hipGetDevice(&dev) : hipStreamGetDevice(s, &dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* p = g_scratch[dev].load(std::memory_order_acquire);
  if (p != nullptr) {
    *out = p;
    return hipSuccess;
  }
  std::lock_guard<std::mutex> lock(g_setup);
  p = g_scratch[dev].load(std::memory_order_acquire);
  if (p == nullptr) {
    int cur = 0;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) {
      hipLaunchKernelGGL(clear_scratch_kernel, dim3(256), dim3(kClearBlock), 0, s, (uint64_t*)p,
                         (int64_t)(kScratchBytes / 8));
      e = hipGetLastError();
    }
    if (cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_scratch[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return hipSuccess;
}

}  // namespace launch
}  // namespace desc
