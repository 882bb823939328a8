// SumThreshold along time from caller-supplied pre-flags, float input.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_pre_float(int lanes) {
  return lanes == 32 ? (const void*)lof_time_pre_kernel<false, 32>
                     : (lanes == 48 ? (const void*)lof_time_pre_kernel<false, 48> : (const void*)lof_time_pre_kernel<false, 64>);
}
}  // namespace lofk
