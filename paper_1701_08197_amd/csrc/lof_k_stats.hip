// Statistics kernels (power, median, stddev, thresholds), both input kinds.
#include "lof_kernels.hpp"
#include "lof_kernel_table.hpp"

namespace lofk {
const void* kernel_stats(bool integer) {
  return integer ? (const void*)lof_stats_kernel<true, false> : (const void*)lof_stats_kernel<false, false>;
}
const void* kernel_stats_pre(bool integer) {
  return integer ? (const void*)lof_stats_kernel<true, true> : (const void*)lof_stats_kernel<false, true>;
}
}  // namespace lofk
