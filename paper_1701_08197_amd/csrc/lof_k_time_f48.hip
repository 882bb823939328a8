// SumThreshold along time, float input, 48 samples per lane.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_float48() { return (const void*)lof_time_kernel<false, 48>; }
}  // namespace lofk
