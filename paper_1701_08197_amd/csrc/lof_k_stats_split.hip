// Statistics of large float blocks split over workgroups (one launch per radix pass).
#include "lof_stats_split.hpp"
#include "lof_kernel_table.hpp"

namespace lofk {

// work item = block * maxparts + part; parts past a block's count return at once
template <bool PRE>
__global__ __launch_bounds__(WG) void lof_stats_split_kernel(const DevBlock* __restrict__ blocks, int nb, int maxparts,
                                                             int pass, SplitState* __restrict__ ss, DevParams P) {
  __shared__ SmSplit sm;
  const int item = (int)blockIdx.x;
  const int bi = item / maxparts, part = item - bi * maxparts;
  if (bi >= nb) return;
  const DevBlock b = blocks[bi];
  if (part >= split_parts(b.C, b.T)) return;
  phase_stats_split<PRE>(b, P, ss[bi], part, pass, sm);
}

const void* kernel_stats_split(bool pre) {
  return pre ? (const void*)lof_stats_split_kernel<true> : (const void*)lof_stats_split_kernel<false>;
}

}  // namespace lofk
