// lof_kernel_table.hpp -- host-side handles of the phase kernels.  Each kernel
// family is instantiated in a translation unit of its own (lof_k_*.hip) so the
// library builds in parallel; the host code launches through these handles.
#pragma once

namespace lofk {
const void* kernel_stats(bool integer);
const void* kernel_stats_pre(bool integer);         // statistics without pre-flagged samples
const void* kernel_stats_split(bool pre);           // statistics of large float blocks, one part per workgroup
const void* kernel_time(bool integer, int lanes);   // lanes: 32, 48 or 64
const void* kernel_time_pre(bool integer, int lanes);   // starting from pre-flags
const void* kernel_time_cx();                       // float rows of complex input, 32 lanes
const void* kernel_freq(bool integer);
const void* kernel_freq_small();                    // float blocks of at most 16 channels
const void* kernel_sir_time(int lanes);
const void* kernel_sir_freq();
const void* kernel_final(bool integer);
const void* kernel_prose(bool freq);                // prose SIR reading: rows / columns
const void* kernel_integrated(bool integer);        // integrated pre-correlation mode
const void* kernel_post(bool integer);              // SIR + history + bytes, mask in LDS
const void* kernel_partial_integrate(bool integer); // partial integration: tile means
const void* kernel_partial_spread();                // partial integration: flag bytes
}  // namespace lofk
