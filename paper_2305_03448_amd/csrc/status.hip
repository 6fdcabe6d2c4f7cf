// status.hip -- the device status word of a workspace: read-and-clear, and
// the debug limit on the polls of one bounded wait.
//
// Some failures can only be seen on the GPU: a bounded wait for another
// block that runs out (a workspace not zeroed before its first use, or two
// calls overlapping on one workspace), or grouped BF16X3 planes that do not
// fit the workspace.  The kernels record them in the 32-bit word at byte 4 of
// the workspace (WsHeader::error); these one-thread kernels hand that word
// to the caller in stream order, without a host read, so they can be
// captured in a graph like the calls they check.
#include "common.hpp"
#include "launch.hpp"

namespace desc {
namespace {

__global__ __launch_bounds__(64) void ws_status_kernel(WsHeader* __restrict__ hdr,
                                                       int32_t* __restrict__ out) {
  if (thread_x<64>().index() != 0) return;
  const uint32_t e = __hip_atomic_exchange(&hdr->error, 0u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
  array(out, 1)[0] = (int32_t)e;
}

__global__ __launch_bounds__(64) void ws_wait_limit_kernel(WsHeader* __restrict__ hdr,
                                                           uint32_t v) {
  if (thread_x<64>().index() != 0) return;
  __hip_atomic_store(&hdr->wait_limit, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

namespace launch {

hipError_t workspace_status(void* ws, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(ws_status_kernel, dim3(1), dim3(64), 0, s, (WsHeader*)ws, out);
  return hipGetLastError();
}

hipError_t workspace_set_wait_limit(void* ws, uint32_t encoded, hipStream_t s) {
  hipLaunchKernelGGL(ws_wait_limit_kernel, dim3(1), dim3(64), 0, s, (WsHeader*)ws, encoded);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace desc
