// SumThreshold along frequency, both input kinds.
#include "lof_kernels.hpp"
#include "lof_kernel_table.hpp"

namespace lofk {
const void* kernel_freq(bool integer) {
  return integer ? (const void*)lof_freq_kernel<true> : (const void*)lof_freq_kernel<false>;
}
const void* kernel_freq_small() { return (const void*)lof_freq_small_kernel<16>; }
}  // namespace lofk
