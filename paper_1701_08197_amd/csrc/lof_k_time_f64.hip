// SumThreshold along time, float input, 64 samples per lane.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_float64() { return (const void*)lof_time_kernel<false, 64>; }
}  // namespace lofk
