// lof_stats_split.hpp -- statistics of large float blocks split over workgroups
// (gfx950).
//
// Method: van Nieuwpoort, "Towards exascale real-time RFI mitigation", arXiv
// 1701.08197, Sec. 2.1 (thresholds from the block's median and stddev), Sec. 4.2
// (an O(N) median; the MAD as the robust stddev).
//
// The one-workgroup statistics of a float block are a 3-pass radix select over
// its samples on one CU (a 262144-sample block: about 0.25 ms), so a call with
// few large float blocks waits on a few CUs.  Here a block's samples are cut
// into parts of about SPLIT_PART_ITEMS chunks of 8 samples, one workgroup per
// part, and each radix pass is a launch of its own:
//   - every part histograms its samples' current key digit in LDS (the keys whose
//     higher digits match the prefixes chosen so far) and adds its nonzero bins
//     to the block's global histogram; pass 0 also writes the part's float64
//     moments and count of statistics samples;
//   - the part that finishes last (a device-scope counter) picks the digit of
//     ranks r0 and r1 from the global histogram, clears it for the next pass, and
//     after the last pass forms median, stddev and thresholds with the code of
//     the one-workgroup kernel (the part sums are added in part order, so the
//     stddev may differ from the one-workgroup kernel's in its last bits).
// Keys: the order-preserving 32-bit key of the float32 power (the MAD: of the
// absolute deviation from the median), digits 12 + 12 + 8.  Integer input keeps
// the one-workgroup kernel: its exact full-resolution histogram is faster than
// this split at every call size measured (the split's global histogram merges
// contend on the few bins where noise powers crowd).
#pragma once
#include "lof_kernels.hpp"

namespace lofk {

constexpr int SPLIT_MAX_PARTS = 64;
constexpr int SPLIT_PART_ITEMS = 1024;      // chunks of 8 samples per part (at least, below 64 parts)
constexpr int SPLIT_MAX_BLOCKS = 16;        // float blocks of a call that take the split path
constexpr int64_t SPLIT_MIN_SAMPLES = 65536;   // the largest of them (up to 4 blocks)
constexpr int64_t SPLIT_BIG_SAMPLES = 1 << 20; // the largest of them (5 to 16 blocks)
constexpr int SPLIT_PASSES = 3;             // radix passes of one order statistic

// The host's choice: a call's float blocks take the split statistics when there
// are at most 4 of them and the largest has at least 65536 samples, or at most 16
// and the largest has at least 2^20 (measured: 1 or 4 blocks of 64 x 4096
// complex64 take 0.20 / 0.24 ms instead of 0.34 / 0.35 ms per call, 1 or 8 blocks
// of 256 x 12000 float32 0.33 / 0.72 ms instead of 2.1 / 2.3 ms; 16 blocks of
// 64 x 4096 are faster on one workgroup each).
__host__ __device__ inline bool split_chosen(int nblocks, int64_t largest) {
  return (nblocks <= 4 && largest >= SPLIT_MIN_SAMPLES) || (nblocks <= SPLIT_MAX_BLOCKS && largest >= SPLIT_BIG_SAMPLES);
}

// per block of a split launch, in call scratch; hist and done are zero between
// passes
struct SplitState {
  uint32_t hist[2][HBINS];
  double pd[SPLIT_MAX_PARTS][2];               // part sums of p and p^2
  uint32_t plive[SPLIT_MAX_PARTS];             // statistics samples per part
  uint32_t done;                               // parts finished in this pass
  uint32_t N;                                  // statistics samples of the block
  uint32_t pre0, pre1, r0, r1;                 // radix state: prefixes and remaining ranks
  uint32_t k0, k1;                             // keys of the middle order statistics
  uint32_t _pad[6];
};

__host__ __device__ inline int split_parts(int C, int T) {
  const int64_t items = (int64_t)C * ((T + 7) / 8);
  const int64_t p = (items + SPLIT_PART_ITEMS - 1) / SPLIT_PART_ITEMS;
  return (int)(p < 1 ? 1 : (p > SPLIT_MAX_PARTS ? SPLIT_MAX_PARTS : p));
}
// launches of the median (and, robust, of the MAD)
__host__ __device__ inline int split_passes(bool robust) { return SPLIT_PASSES * (robust ? 2 : 1); }

struct SmSplit {
  uint32_t hist[2][HBINS];
  double red_d[2][NW];
  uint32_t red_n[NW];
  uint32_t scan[NW];
  uint32_t sel[4];
  int last;
  double T[16];
  float Tf[16];
  double median, sigma;
};

template <bool PRE>
__device__ __forceinline__ void phase_stats_split(const DevBlock& b, const DevParams& P, SplitState& ss, int part,
                                                  int pass, SmSplit& sm) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int parts = split_parts(b.C, b.T);
  const bool dev = pass >= SPLIT_PASSES;            // the MAD's passes
  const int j = dev ? pass - SPLIT_PASSES : pass;   // digit of this pass: 12, 12, 8 bits
  const int db = j < 2 ? 12 : 8;
  const int lo = j < 2 ? 20 - 12 * j : 0;
  const int hi = lo + db;
  const uint32_t dmask = (1u << db) - 1u;
  // the previous passes' results (written by earlier launches)
  const uint32_t pre0 = j ? ss.pre0 : 0u, pre1 = j ? ss.pre1 : 0u;
  const bool two = j > 0 && pre1 != pre0;
  const bool skip = pass > 0 && ss.N == 0;   // nothing to select
  double med = 0.0;
  if (dev) {
    const uint32_t k0 = ss.k0, k1 = ss.k1, N = ss.N;
    const double v0 = (double)fkey_inv(k0), v1 = (double)fkey_inv(k1);
    med = (N & 1) ? v0 : (v0 + v1) / 2.0;
  }
  auto key = [&](float v) -> uint32_t {
    return dev ? fkey((float)__builtin_fabs((double)v - med)) : fkey(v);
  };

  for (int i = tid; i < 2 * HBINS; i += WG) (&sm.hist[0][0])[i] = 0u;
  __syncthreads();
  const int nch = (b.T + 7) >> 3;
  const uint32_t items = (uint32_t)b.C * (uint32_t)nch;
  const FastDiv fd((uint32_t)nch);
  const uint32_t per = (items + (uint32_t)parts - 1u) / (uint32_t)parts;
  const uint32_t it0 = (uint32_t)part * per, it1 = min(items, it0 + per);
  double s1d = 0.0, s2d = 0.0;
  uint32_t live = 0;
  if (!skip) {
    for (uint32_t it = it0 + (uint32_t)tid; it < it1; it += WG) {
      const int row = (int)fd.div(it);
      const int t0 = (int)(it - (uint32_t)row * (uint32_t)nch) * 8;
      float v[8];
      const int nv = load8<false>(b, row, t0, v);
      const uint32_t pm = pre8<PRE>(b, row, t0, nv);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q < nv && !((pm >> q) & 1u)) {
          if (pass == 0) {
            ++live;
            const double d = (double)v[q];
            s1d += d;
            s2d += d * d;
          }
          const uint32_t kv = key(v[q]);
          const uint32_t top = hi >= 32 ? 0u : (kv >> hi);
          const uint32_t dg = (kv >> lo) & dmask;
          if (top == pre0) atomicAdd(&sm.hist[0][dg], 1u);
          if (two && top == pre1) atomicAdd(&sm.hist[1][dg], 1u);
        }
      }
    }
  }
  __syncthreads();
  // the part's nonzero bins into the block's histogram
  for (int i = tid; i < (two ? 2 : 1) * HBINS; i += WG) {
    const uint32_t c = (&sm.hist[0][0])[i];
    if (c) atomicAdd(&ss.hist[0][0] + i, c);
  }
  if (pass == 0) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      s1d += __shfl_xor(s1d, d);
      s2d += __shfl_xor(s2d, d);
      live += __shfl_xor(live, d);
    }
    if (lane == 0) {
      sm.red_d[0][wv] = s1d;
      sm.red_d[1][wv] = s2d;
      sm.red_n[wv] = live;
    }
    __syncthreads();
    if (tid == 0) {
      double x = 0.0, y = 0.0;
      uint32_t n = 0;
      for (int w = 0; w < NW; ++w) {
        x += sm.red_d[0][w];
        y += sm.red_d[1][w];
        n += sm.red_n[w];
      }
      ss.pd[part][0] = x;
      ss.pd[part][1] = y;
      ss.plive[part] = n;
    }
  }
  // the last part to finish takes the pass's digit
  __threadfence();
  __syncthreads();
  if (tid == 0) sm.last = atomicAdd(&ss.done, 1u) == (uint32_t)parts - 1u ? 1 : 0;
  __syncthreads();
  if (!sm.last) return;
  __threadfence();
  uint32_t N;
  if (pass == 0) {
    if (PRE) {
      N = 0;
      for (int q = 0; q < parts; ++q) N += ss.plive[q];
    } else {
      N = (uint32_t)b.C * (uint32_t)b.T;
    }
  } else {
    N = ss.N;
  }
  const uint32_t r0 = j ? ss.r0 : (N > 0 ? (N - 1) / 2 : 0u);
  const uint32_t r1 = j ? ss.r1 : N / 2;
  for (int i = tid; i < 2 * HBINS; i += WG) {
    (&sm.hist[0][0])[i] = __hip_atomic_load(&ss.hist[0][0] + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    (&ss.hist[0][0])[i] = 0u;
  }
  __syncthreads();
  uint32_t b0 = 0, q0 = 0, b1 = 0, q1 = 0;
  if (N > 0) {
    find_bin(sm.hist[0], r0, sm, b0, q0);
    find_bin(two ? sm.hist[1] : sm.hist[0], r1, sm, b1, q1);
  }
  const uint32_t np0 = (pre0 << db) | b0, np1 = (pre1 << db) | b1;
  if (tid == 0) {
    ss.done = 0u;
    ss.N = N;
    ss.pre0 = np0;
    ss.pre1 = np1;
    ss.r0 = q0;
    ss.r1 = q1;
    if (j == SPLIT_PASSES - 1 && !dev) {
      ss.k0 = np0;
      ss.k1 = np1;
    }
  }
  if (pass != split_passes(P.robust != 0) - 1) return;
  // the last pass: the block's statistics
  if (tid == 0) {
    double S1d = 0.0, S2d = 0.0;
    for (int q = 0; q < parts; ++q) {
      S1d += ss.pd[q][0];
      S2d += ss.pd[q][1];
    }
    uint32_t k0 = np0, k1 = np1, m0 = 0, m1 = 0;
    if (dev) {
      k0 = ss.k0;
      k1 = ss.k1;
      m0 = np0;
      m1 = np1;
    }
    if (N == 0) k0 = k1 = m0 = m1 = 0u;
    stats_finish<false>(P, (int64_t)N, k0, k1, m0, m1, 0ull, 0ull, S1d, S2d, sm);
  }
  __syncthreads();
  write_block_stats(b, P, sm);
}

}  // namespace lofk
