// SumThreshold along time, integer input, 32 samples per lane.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_int32() { return (const void*)lof_time_kernel<true, 32>; }
}  // namespace lofk
