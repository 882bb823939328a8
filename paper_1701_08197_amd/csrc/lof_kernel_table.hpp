// lof_kernel_table.hpp -- host-side handles of the phase kernels.  Each kernel
// family is instantiated in a translation unit of its own (lof_k_*.hip) so the
// library builds in parallel; the host code launches through these handles.
#pragma once

namespace lofk {
const void* kernel_stats(bool integer);
const void* kernel_time(bool integer, int lanes);   // lanes: 32, 48 or 64
const void* kernel_freq(bool integer);
const void* kernel_sir_time(int lanes);
const void* kernel_sir_freq();
const void* kernel_final(bool integer);
const void* kernel_prose(bool freq);                // prose SIR reading: rows / columns
const void* kernel_integrated(bool integer);        // integrated pre-correlation mode
const void* kernel_post(bool integer);              // SIR + history + bytes, mask in LDS
}  // namespace lofk
