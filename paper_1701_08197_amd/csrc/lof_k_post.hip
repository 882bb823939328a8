// SIR operator, history flagger and flag bytes in one kernel for blocks of at
// most 64 channels and 4096 times (the block's mask in LDS), both input kinds.
#include "lof_kernel_table.hpp"
#include "lof_post.hpp"

namespace lofk {

template <bool INT>
__global__ __launch_bounds__(WG, LOF_WAVES_PER_EU) void lof_post_kernel(const DevBlock* __restrict__ blocks, int nb, int maxch,
                                                     int* counter, DevParams P) {
  __shared__ SmPost sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const DevBlock b = blocks[it / maxch];
    phase_post<INT>(b, P, sm);
  });
}

const void* kernel_post(bool integer) {
  return integer ? (const void*)lof_post_kernel<true> : (const void*)lof_post_kernel<false>;
}

}  // namespace lofk
