// SumThreshold along time from caller-supplied pre-flags, integer input.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_pre_int(int lanes) {
  return lanes == 32 ? (const void*)lof_time_pre_kernel<true, 32>
                     : (lanes == 48 ? (const void*)lof_time_pre_kernel<true, 48> : (const void*)lof_time_pre_kernel<true, 64>);
}
}  // namespace lofk
