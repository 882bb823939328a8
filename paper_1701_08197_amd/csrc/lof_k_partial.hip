// 2-D flagging with partial integration: the integration and spread kernels.
#include "lof_kernel_table.hpp"
#include "lof_partial.hpp"

namespace lofk {

// tile means of every block: items (block, row of tiles x time segment)
template <bool INT>
__global__ __launch_bounds__(WG, LOF_WAVES_PER_EU) void lof_partial_integrate_kernel(
    const PartialBlock* __restrict__ blocks, int nb, int maxch, lof_block_stats* stats) {
  __shared__ SmPartial<INT> sm;
  const int it = (int)blockIdx.x;
  const int bi = it / maxch, item = it - bi * maxch;
  if (bi >= nb) return;
  const PartialBlock pb = blocks[bi];
  if ((pb.fine.dtype == LOF_CI8) != INT || item >= part_items(pb.Cc, pb.Tc, pb.ft)) return;
  if (stats && item == 0 && threadIdx.x == 0)
    *(unsigned long long*)((char*)stats + (int64_t)pb.fine.out_idx * STATS_BYTES + STATS_NFLAG) = 0ull;
  phase_partial_integrate<INT>(pb, item, sm);
}

// flag bytes of every block from its tile flags: items (block, 8 rows)
__global__ __launch_bounds__(WG, LOF_WAVES_PER_EU) void lof_partial_spread_kernel(
    const PartialBlock* __restrict__ blocks, int nb, int maxch, const lof_block_stats* cstats,
    lof_block_stats* stats) {
  const int it = (int)blockIdx.x;
  const int bi = it / maxch, chunk = it - bi * maxch;
  if (bi >= nb) return;
  const PartialBlock pb = blocks[bi];
  if (chunk >= part_spread_chunks(pb.fine.C)) return;
  phase_partial_spread(pb, chunk, pb.fine.out_idx, cstats, stats);
}

const void* kernel_partial_integrate(bool integer) {
  return integer ? (const void*)lof_partial_integrate_kernel<true> : (const void*)lof_partial_integrate_kernel<false>;
}
const void* kernel_partial_spread() { return (const void*)lof_partial_spread_kernel; }

}  // namespace lofk
