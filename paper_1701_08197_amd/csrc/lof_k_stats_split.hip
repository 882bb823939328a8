// Statistics of large blocks split over workgroups (one launch per radix pass).
#include "lof_stats_split.hpp"
#include "lof_kernel_table.hpp"

namespace lofk {

// work item = block * maxparts + part; parts past a block's count return at once
template <bool INT, bool PRE>
__global__ __launch_bounds__(WG) void lof_stats_split_kernel(const DevBlock* __restrict__ blocks, int nb, int maxparts,
                                                             int pass, SplitState* __restrict__ ss, DevParams P) {
  __shared__ SmSplit sm;
  const int item = (int)blockIdx.x;
  const int bi = item / maxparts, part = item - bi * maxparts;
  if (bi >= nb) return;
  const DevBlock b = blocks[bi];
  if (part >= split_parts(b.C, b.T)) return;
  phase_stats_split<INT, PRE>(b, P, ss[bi], part, pass, sm);
}

const void* kernel_stats_split(bool integer, bool pre) {
  if (integer) return pre ? (const void*)lof_stats_split_kernel<true, true> : (const void*)lof_stats_split_kernel<true, false>;
  return pre ? (const void*)lof_stats_split_kernel<false, true> : (const void*)lof_stats_split_kernel<false, false>;
}

}  // namespace lofk
