// SumThreshold along time, integer input, 64 samples per lane.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_int64() { return (const void*)lof_time_kernel<true, 64>; }
}  // namespace lofk
