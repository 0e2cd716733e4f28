// k_merge.hip -- staging several invocations of one kernel as one trace, for
// the aggregate over all invocations that the paper reports per kernel
// (Evaluation section).  The event, memory and branch streams are plain
// device-to-device copies; only the work-item offsets need arithmetic.
#include <algorithm>

#include "common.h"

namespace {

// dst[i] = src[i] + base for i in [lo, n]: one invocation's work-item
// offsets (src[0] = 0, src[n] = its event count) moved behind the `base`
// events of the invocations before it.  lo = 1 except for the first
// invocation: entry 0 of a later one equals the last entry already written
// by the one before.
__global__ void __launch_bounds__(256) k_merge_offsets(u64 *__restrict__ dst,
                                                       const u64 *__restrict__ src, u64 lo,
                                                       u64 n, u64 base) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = lo + blockIdx.x * (u64)blockDim.x + threadIdx.x; i <= n; i += stride)
    dst[i] = src[i] + base;
}

}  // namespace

namespace aiwc_kernels {

hipError_t launch_merge_offsets(u64 *dst, const u64 *src, u64 n_wi, u64 base, bool first,
                                hipStream_t s) {
  const u64 lo = first ? 0 : 1;
  if (n_wi + 1 <= lo) return hipSuccess;
  const u64 blocks = std::min<u64>((n_wi + 1 - lo + 255) / 256, 8192);
  hipLaunchKernelGGL(k_merge_offsets, dim3((u32)blocks), dim3(256), 0, s, dst, src, lo, n_wi,
                     base);
  return hipGetLastError();
}

}  // namespace aiwc_kernels
