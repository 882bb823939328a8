// SumThreshold along time, integer input, 48 samples per lane.
#include "lof_kernels.hpp"

namespace lofk {
const void* kernel_time_int48() { return (const void*)lof_time_kernel<true, 48>; }
}  // namespace lofk
