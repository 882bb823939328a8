// SIR operator kernels: along time (every lane width) and along frequency.
#include "lof_kernels.hpp"
#include "lof_kernel_table.hpp"

namespace lofk {
__global__ __launch_bounds__(WG, LOF_WAVES_PER_EU) void lof_sir_freq_kernel(const DevBlock* __restrict__ blocks, int nb,
                                                                            int maxch, int* counter, DevParams P) {
  __shared__ SmSirF sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= sirf_chunks(b.C, b.T)) return;
    phase_sir_freq(b, P, sm, ch);
  });
}

// prose reading of the SIR step: rows, then columns
__global__ __launch_bounds__(WG) void lof_prose_time_kernel(const DevBlock* __restrict__ blocks, int nb, int maxch,
                                                           int* counter, DevParams P) {
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= prose_time_chunks(b.C)) return;
    phase_prose_time(b, P, ch);
  });
}

__global__ __launch_bounds__(WG) void lof_prose_freq_kernel(const DevBlock* __restrict__ blocks, int nb, int maxch,
                                                           int* counter, DevParams P) {
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= prose_freq_chunks(b.T)) return;
    phase_prose_freq(b, P, ch);
  });
}

const void* kernel_prose(bool freq) {
  return freq ? (const void*)lof_prose_freq_kernel : (const void*)lof_prose_time_kernel;
}

const void* kernel_sir_time(int lanes) {
  return lanes == 32 ? (const void*)lof_sir_time_kernel<32>
                     : (lanes == 48 ? (const void*)lof_sir_time_kernel<48> : (const void*)lof_sir_time_kernel<64>);
}
const void* kernel_sir_freq() { return (const void*)lof_sir_freq_kernel; }
}  // namespace lofk
