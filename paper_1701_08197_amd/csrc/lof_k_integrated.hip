// Integrated pre-correlation mode kernels, both input kinds: one workgroup per
// block, the block's spectrum and time series in dynamic LDS.
#include "lof_integrated.hpp"
#include "lof_kernel_table.hpp"

namespace lofk {

template <bool INT>
__global__ __launch_bounds__(WG, LOF_WAVES_PER_EU) void lof_integrated_kernel(const DevBlock* __restrict__ blocks, int nb, int maxch,
                                                           int* counter, DevParams P) {
  // 16-byte aligned: the areas carved from it hold 8-byte values and 64-bit LDS
  // atomics, and the array follows the work loop's 4-byte static variable
  extern __shared__ __align__(16) unsigned char integ_lds[];
  const IntegSm s = integ_carve(integ_lds, P.integ_tmax);
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const DevBlock b = blocks[it / maxch];
    phase_integrated<INT>(b, P, s);
  });
}

const void* kernel_integrated(bool integer) {
  return integer ? (const void*)lof_integrated_kernel<true> : (const void*)lof_integrated_kernel<false>;
}

}  // namespace lofk
