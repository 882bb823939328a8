// lof_stats_split.hpp -- statistics of a large block split over workgroups
// (gfx950).
//
// Method: van Nieuwpoort, "Towards exascale real-time RFI mitigation", arXiv
// 1701.08197, Sec. 2.1 (thresholds from the block's median and stddev), Sec. 4.2
// (an O(N) median; the MAD as the robust stddev).
//
// A call with few blocks leaves most of the chip idle while one workgroup per
// block computes its statistics.  Here a block's samples are cut into parts of
// about SPLIT_PART_ITEMS chunks of 8 samples, one workgroup per part, and the
// median (and the MAD) is a radix select whose passes are separate launches:
//   - every part histograms its samples' current key digit in LDS (the keys whose
//     higher digits match the prefixes chosen so far) and adds its nonzero bins
//     to the block's global histogram; pass 0 also writes the part's moments and
//     count of statistics samples;
//   - the part that finishes last (a device-scope counter) picks the digit of
//     ranks r0 and r1 from the global histogram, clears it for the next pass, and
//     after the last pass forms median, stddev and thresholds exactly as the
//     one-workgroup kernel does (integer input: the same exact sums; float input:
//     float64 part sums added in part order, so the stddev may differ from the
//     one-workgroup kernel's in its last bits).
// Digits: integer power (16 bits) 8 + 8; integer doubled deviation (<= 2^17, a
// 20-bit key) 12 + 8; float keys (32 bits) 12 + 12 + 8.
#pragma once
#include "lof_kernels.hpp"

namespace lofk {

constexpr int SPLIT_MAX_PARTS = 64;
constexpr int SPLIT_PART_ITEMS = 1024;      // chunks of 8 samples per part (at least, below 64 parts)
constexpr int SPLIT_MAX_BLOCKS = 64;        // blocks of one kind in a split launch
constexpr int64_t SPLIT_MIN_SAMPLES = 65536;   // the host splits calls whose largest block reaches this

// per block of a split launch, in call scratch; hist, done are zero between passes
struct SplitState {
  uint32_t hist[2][HBINS];
  unsigned long long pu[SPLIT_MAX_PARTS][2];   // integer part sums of p and p^2
  double pd[SPLIT_MAX_PARTS][2];               // float part sums of p and p^2
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
// radix passes of the median (and, robust, of the MAD)
__host__ __device__ inline int split_select_passes(bool integer) { return integer ? 2 : 3; }
__host__ __device__ inline int split_passes(bool integer, bool robust) {
  return split_select_passes(integer) * (robust ? 2 : 1);
}
// digit of pass j of a select: bits [lo, lo + db) of a key of kb bits
__host__ __device__ inline void split_digit(bool integer, bool dev, int j, int& kb, int& lo, int& db) {
  if (integer) {
    kb = dev ? 20 : 16;
    const int w0 = dev ? 12 : 8;
    db = j == 0 ? w0 : 8;
    lo = j == 0 ? kb - w0 : 0;
  } else {
    kb = 32;
    db = j < 2 ? 12 : 8;
    lo = kb - 12 * (j + 1);
    if (j == 2) lo = 0;
  }
}

struct SmSplit {
  uint32_t hist[2][HBINS];
  double red_d[2][NW];
  unsigned long long red_u[2][NW];
  uint32_t red_n[NW];
  uint32_t scan[NW];
  uint32_t sel[4];
  int last;
  double T[16];
  float Tf[16];
  double median, sigma;
};

template <bool INT, bool PRE>
__device__ __forceinline__ void phase_stats_split(const DevBlock& b, const DevParams& P, SplitState& ss, int part,
                                                  int pass, SmSplit& sm) {
  typedef typename PowT<INT>::T VT;
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int parts = split_parts(b.C, b.T);
  const int nsel = split_select_passes(INT);
  const bool dev = pass >= nsel;
  const int j = dev ? pass - nsel : pass;
  int kb, lo, db;
  split_digit(INT, dev, j, kb, lo, db);
  const uint32_t dmask = (1u << db) - 1u;
  const int hi = lo + db;
  // the previous passes' results (written by earlier launches)
  const uint32_t pre0 = j ? ss.pre0 : 0u, pre1 = j ? ss.pre1 : 0u;
  const bool two = j > 0 && pre1 != pre0;
  const bool skip = pass > 0 && ss.N == 0;   // nothing to select
  uint32_t med2 = 0;
  double med = 0.0;
  if (dev) {
    const uint32_t k0 = ss.k0, k1 = ss.k1, N = ss.N;
    med2 = k0 + k1;
    if (!INT) {
      const double v0 = (double)fkey_inv(k0), v1 = (double)fkey_inv(k1);
      med = (N & 1) ? v0 : (v0 + v1) / 2.0;
    }
  }
  auto key = [&](VT v) -> uint32_t {
    if (!dev) return INT ? (uint32_t)v : fkey((float)v);
    if (INT) {
      const int d = 2 * (int)(uint32_t)v - (int)med2;
      return (uint32_t)(d < 0 ? -d : d);
    }
    return fkey((float)__builtin_fabs((double)v - med));
  };

  for (int i = tid; i < 2 * HBINS; i += WG) (&sm.hist[0][0])[i] = 0u;
  __syncthreads();
  const int nch = (b.T + 7) >> 3;
  const uint32_t items = (uint32_t)b.C * (uint32_t)nch;
  const FastDiv fd((uint32_t)nch);
  const uint32_t per = (items + (uint32_t)parts - 1u) / (uint32_t)parts;
  const uint32_t it0 = (uint32_t)part * per, it1 = min(items, it0 + per);
  unsigned long long s1u = 0, s2u = 0;
  double s1d = 0.0, s2d = 0.0;
  uint32_t live = 0;
  if (!skip) {
    for (uint32_t it = it0 + (uint32_t)tid; it < it1; it += WG) {
      const int row = (int)fd.div(it);
      const int t0 = (int)(it - (uint32_t)row * (uint32_t)nch) * 8;
      VT v[8];
      const int nv = load8<INT>(b, row, t0, v);
      const uint32_t pm = pre8<PRE>(b, row, t0, nv);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q < nv && !((pm >> q) & 1u)) {
          if (pass == 0) {
            ++live;
            if (INT) {
              const uint32_t p = (uint32_t)v[q];
              s1u += p;
              s2u += (unsigned long long)(p * p);   // p <= 32768: p*p <= 2^30
            } else {
              const double d = (double)v[q];
              s1d += d;
              s2d += d * d;
            }
          }
          const uint32_t kv = key(v[q]);
          const uint32_t top = hi >= kb ? 0u : (kv >> hi);
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
      s1u += __shfl_xor(s1u, d);
      s2u += __shfl_xor(s2u, d);
      s1d += __shfl_xor(s1d, d);
      s2d += __shfl_xor(s2d, d);
      live += __shfl_xor(live, d);
    }
    if (lane == 0) {
      sm.red_u[0][wv] = s1u;
      sm.red_u[1][wv] = s2u;
      sm.red_d[0][wv] = s1d;
      sm.red_d[1][wv] = s2d;
      sm.red_n[wv] = live;
    }
    __syncthreads();
    if (tid == 0) {
      unsigned long long a = 0, c = 0;
      double x = 0.0, y = 0.0;
      uint32_t n = 0;
      for (int w = 0; w < NW; ++w) {
        a += sm.red_u[0][w];
        c += sm.red_u[1][w];
        x += sm.red_d[0][w];
        y += sm.red_d[1][w];
        n += sm.red_n[w];
      }
      ss.pu[part][0] = a;
      ss.pu[part][1] = c;
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
  const bool sel_done = j == nsel - 1;
  if (tid == 0) {
    ss.done = 0u;
    ss.N = N;
    ss.pre0 = np0;
    ss.pre1 = np1;
    ss.r0 = q0;
    ss.r1 = q1;
    if (sel_done && !dev) {
      ss.k0 = np0;
      ss.k1 = np1;
    }
  }
  if (pass != split_passes(INT, P.robust != 0) - 1) return;
  // the last pass: the block's statistics
  if (tid == 0) {
    unsigned long long S1u = 0, S2u = 0;
    double S1d = 0.0, S2d = 0.0;
    for (int q = 0; q < parts; ++q) {
      S1u += ss.pu[q][0];
      S2u += ss.pu[q][1];
      S1d += ss.pd[q][0];
      S2d += ss.pd[q][1];
    }
    uint32_t k0, k1, m0 = 0, m1 = 0;
    if (dev) {
      k0 = ss.k0;
      k1 = ss.k1;
      m0 = np0;
      m1 = np1;
    } else {
      k0 = np0;
      k1 = np1;
    }
    if (N == 0) {
      k0 = k1 = m0 = m1 = 0u;
    }
    stats_finish<INT>(P, (int64_t)N, k0, k1, m0, m1, S1u, S2u, S1d, S2d, sm);
  }
  __syncthreads();
  write_block_stats(b, P, sm);
}

}  // namespace lofk
