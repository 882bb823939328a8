// History flagger and flag-byte kernels, both input kinds.
#include "lof_kernels.hpp"
#include "lof_kernel_table.hpp"

namespace lofk {
const void* kernel_final(bool integer) {
  return integer ? (const void*)lof_final_kernel<true> : (const void*)lof_final_kernel<false>;
}
}  // namespace lofk
