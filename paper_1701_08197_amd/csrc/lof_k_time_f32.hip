// SumThreshold along time, float input, 32 samples per lane.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_float32() { return (const void*)lof_time_kernel<false, 32>; }
const void* kernel_time_float32_cx() { return (const void*)lof_time_kernel<false, 32, true>; }
}  // namespace lofk
