// lof_kernels.hpp -- the per-block phases of the LOF flagging kernel (gfx950).
// See lof_device.hpp for the layouts.  Citations are to van Nieuwpoort,
// "Towards exascale real-time RFI mitigation", arXiv 1701.08197.
#pragma once
#include "lof_device.hpp"

namespace lofk {

constexpr double MAD_TO_SIGMA = 1.4826;   // normal stddev per unit of MAD (1 / 0.6745)

// Exact unsigned 32-bit division by a block-uniform divisor d >= 1 (round-up
// multiplier method: l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// q = (hi + ((n - hi) >> 1)) >> (l - 1) with hi = mulhi(m, n); l = 0 for d = 1).
struct FastDiv {
  uint32_t d, m;
  int l;
  __device__ explicit FastDiv(uint32_t dd) : d(dd) {
    l = 0;
    while ((1ull << l) < dd) ++l;
    m = (uint32_t)((((1ull << l) - dd) << 32) / dd + 1ull);
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    if (l == 0) return n;
    const uint32_t hi = __umulhi(m, n);
    return (hi + ((n - hi) >> 1)) >> (l - 1);
  }
};

// ===================================================================== phase A
// Block median and population standard deviation over all C*T samples
// (Sec. 2.1 threshold definition; Sec. 4.2 asks for an O(N) median).
// Integer input: one pass accumulates exact moments and a full-resolution
// histogram of the integer power (32769 bins as 16-bit counters, two per LDS
// word); if any bin could have wrapped (the 16-bit fields no longer sum to N) the
// block falls back to a 2-pass radix select.  Float input: 3-pass radix select
// over an order-preserving 32-bit key (12 + 12 + 8 bits), float64 moments.

// block-wide: bin holding `rank` (0-based) of a 4096-bin histogram
template <class SM>
__device__ void find_bin(const uint32_t* h, uint32_t rank, SM& sm, uint32_t& bin, uint32_t& rem) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  constexpr int PER = HBINS / WG;
  uint32_t loc[PER];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    loc[j] = h[tid * PER + j];
    s += loc[j];
  }
  uint32_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) sm.scan[wv] = x;
  __syncthreads();
  uint32_t off = 0;
  for (int w = 0; w < wv; ++w) off += sm.scan[w];
  const uint32_t excl = off + x - s;
  if (rank >= excl && rank < excl + s) {
    uint32_t c = excl;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (rank < c + loc[j]) {
        sm.sel[0] = (uint32_t)(tid * PER + j);
        sm.sel[1] = rank - c;
        break;
      }
      c += loc[j];
    }
  }
  __syncthreads();
  bin = sm.sel[0];
  rem = sm.sel[1];
  __syncthreads();
}

// block-wide: value (bin) holding `rank` in the packed 32769-bin histogram;
// thread t owns words [32t, 32t+32), the last thread also word 16384.
template <class SM>
__device__ uint32_t find_bin16(const uint32_t* h, uint32_t rank, SM& sm) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  constexpr int PW = (IHIST_WORDS - 1) / WG;   // 32
  const int w0 = tid * PW;
  const int nw = PW + (tid == WG - 1 ? 1 : 0);
  uint32_t s = 0;
  for (int j = 0; j < nw; ++j) {
    const uint32_t w = h[w0 + j];
    s += (w & 0xffffu) + (w >> 16);
  }
  uint32_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) sm.scan[wv] = x;
  __syncthreads();
  uint32_t off = 0;
  for (int w = 0; w < wv; ++w) off += sm.scan[w];
  const uint32_t excl = off + x - s;
  if (rank >= excl && rank < excl + s) {
    uint32_t c = excl;
    for (int j = 0; j < nw; ++j) {
      const uint32_t w = h[w0 + j];
      const uint32_t lo = w & 0xffffu, hi = w >> 16;
      if (rank < c + lo) {
        sm.sel[0] = (uint32_t)(2 * (w0 + j));
        break;
      }
      c += lo;
      if (rank < c + hi) {
        sm.sel[0] = (uint32_t)(2 * (w0 + j) + 1);
        break;
      }
      c += hi;
    }
  }
  __syncthreads();
  const uint32_t v = sm.sel[0];
  __syncthreads();
  return v;
}

__device__ __forceinline__ uint32_t fkey(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fkey_inv(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k ^ 0x80000000u) : ~k);
}

// Radix select of the order statistics r0 <= r1 over the block's keys
// key(power) of KB bits (16: 12 + 4, 32: 12 + 12 + 8).  If have_pass0, hist[0]
// already holds the first-digit histogram.
// cand (32-bit keys, 3 passes only): the middle pass also writes the keys it
// histograms (those whose first digit is a chosen one) to the block's candidate
// list, up to ccap of them; if all fit, the last pass reads the list instead of
// the block.
template <bool INT, int KB, bool PRE, class SM, class KF>
__device__ __forceinline__ void radix_select_k(const DevBlock& b, SM& sm, uint32_t r0, uint32_t r1, bool have_pass0,
                                               KF key, uint32_t& k0, uint32_t& k1, GLB uint32_t* cand = nullptr,
                                               uint32_t ccap = 0) {
  typedef typename PowT<INT>::T VT;
  const int tid = thread_id(), lane = tid & 63;
  const int nch = (b.T + 7) >> 3;
  const uint32_t items = (uint32_t)b.C * (uint32_t)nch;
  const FastDiv fd((uint32_t)nch);
  const int npass = KB == 16 ? 2 : 3;
  const int dbits[3] = {12, KB == 16 ? 4 : 12, 8};
  const bool use_cand = KB == 32 && cand != nullptr && ccap > 0;
  uint32_t pre0 = 0, pre1 = 0;
  int hi = KB;
  for (int pass = 0; pass < npass; ++pass) {
    const int db = dbits[pass];
    const int lo = hi - db;
    const uint32_t dmask = (1u << db) - 1u;
    if (pass > 0 || !have_pass0) {
      for (int i = tid; i < 2 * HBINS; i += WG) (&sm.u.hist[0][0])[i] = 0u;
      if (tid == 0 && pass == 1) sm.ncand = 0u;
      __syncthreads();
      const bool two = pre1 != pre0;
      const bool collect = use_cand && pass == 1;
      auto add = [&](uint32_t kv) __attribute__((always_inline)) {
        const uint32_t top = pass == 0 ? 0u : (kv >> hi);
        const uint32_t dg = (kv >> lo) & dmask;
        if (top == pre0) atomicAdd(&sm.u.hist[0][dg], 1u);
        if (two && top == pre1) atomicAdd(&sm.u.hist[1][dg], 1u);
      };
      if (use_cand && pass == 2 && sm.ncand <= ccap) {
        // the candidates of the middle pass instead of the block
        const uint32_t nc = sm.ncand;
        for (uint32_t i = tid; i < nc; i += WG) add(cand[i]);
      } else {
        for (uint32_t it = tid; it < items; it += WG) {
          const int row = (int)fd.div(it);
          const int t0 = (int)(it - (uint32_t)row * (uint32_t)nch) * 8;
          VT v[8];
          const int nv = load8<INT>(b, row, t0, v);
          const uint32_t pm = pre8<PRE>(b, row, t0, nv);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const bool live = j < nv && !((pm >> j) & 1u);
            const uint32_t kv = live ? key(v[j]) : 0u;
            if (live) add(kv);
            if (collect) {
              // one LDS atomic per wave for the wave's candidates
              const uint32_t top = kv >> hi;
              const bool c = live && (top == pre0 || top == pre1);
              const unsigned long long bal = __ballot(c);
              if (bal) {
                const int lead = __ffsll(bal) - 1;
                uint32_t base = 0;
                if (lane == lead) base = atomicAdd(&sm.ncand, (uint32_t)__popcll(bal));
                base = (uint32_t)__shfl(base, lead);
                const uint32_t idx = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
                if (c && idx < ccap) cand[idx] = kv;
              }
            }
          }
        }
      }
      __syncthreads();
    }
    uint32_t b0, q0, b1, q1;
    const bool two = pass > 0 && pre1 != pre0;
    find_bin(sm.u.hist[0], r0, sm, b0, q0);
    find_bin(two ? sm.u.hist[1] : sm.u.hist[0], r1, sm, b1, q1);
    pre0 = (pre0 << db) | b0;
    pre1 = (pre1 << db) | b1;
    r0 = q0;
    r1 = q1;
    hi = lo;
  }
  k0 = pre0;
  k1 = pre1;
}

template <bool INT, bool PRE, class SM>
__device__ __forceinline__ void radix_select(const DevBlock& b, SM& sm, uint32_t r0, uint32_t r1, bool have_pass0,
                                             uint32_t& k0, uint32_t& k1, GLB uint32_t* cand = nullptr,
                                             uint32_t ccap = 0) {
  typedef typename PowT<INT>::T VT;
  radix_select_k<INT, INT ? 16 : 32, PRE>(b, sm, r0, r1, have_pass0,
                                     [](VT v) { return INT ? (uint32_t)v : fkey((float)v); }, k0, k1, cand, ccap);
}

// Robust stddev (Sec. 4.2 lists the MAD): the value of rank `rank` among the
// doubled deviations d = |2p - med2| (med2 = twice the median) of integer powers,
// read from the packed 32769-bin histogram: deviation d counts the bins
// (med2 + d) / 2 and (med2 - d) / 2 when d has the parity of med2.  Thread t
// walks d in [128t, 128t + 128).
template <class SM>
__device__ uint32_t find_dev_rank(const uint32_t* h, uint32_t med2, uint32_t rank, SM& sm) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  auto bin = [&](int p) -> uint32_t {
    if (p < 0 || p > 32768) return 0u;
    const uint32_t w = h[p >> 1];
    return (p & 1) ? (w >> 16) : (w & 0xffffu);
  };
  auto cnt = [&](uint32_t d) -> uint32_t {
    if ((d ^ med2) & 1u) return 0u;
    uint32_t c = bin((int)((med2 + d) >> 1));
    if (d > 0 && d <= med2) c += bin((int)((med2 - d) >> 1));
    return c;
  };
  const uint32_t d0 = (uint32_t)tid * 128u;
  uint32_t s = 0;
  for (uint32_t d = d0; d < d0 + 128u; ++d) s += cnt(d);
  uint32_t x = s;
#pragma unroll
  for (int dd = 1; dd < 64; dd <<= 1) {
    const uint32_t y = __shfl_up(x, dd);
    if (lane >= dd) x += y;
  }
  if (lane == 63) sm.scan[wv] = x;
  __syncthreads();
  uint32_t off = 0;
  for (int w = 0; w < wv; ++w) off += sm.scan[w];
  const uint32_t excl = off + x - s;
  if (rank >= excl && rank < excl + s) {
    uint32_t c = excl;
    for (uint32_t d = d0; d < d0 + 128u; ++d) {
      const uint32_t k = cnt(d);
      if (rank < c + k) {
        sm.sel[0] = d;
        break;
      }
      c += k;
    }
  }
  __syncthreads();
  const uint32_t v = sm.sel[0];
  __syncthreads();
  return v;
}

// Median, stddev (or 1.4826 * MAD) and thresholds T_k of a block from its middle
// order statistics' keys (k0, k1; MAD keys m0, m1) and moments (integer: exact
// sums S1u, S2u; float: float64 sums S1d, S2d) over its N statistics samples, into
// sm.median, sm.sigma, sm.T and sm.Tf.  One thread.
template <bool INT, class SM>
__device__ __forceinline__ void stats_finish(const DevParams& P, int64_t N, uint32_t k0, uint32_t k1, uint32_t m0,
                                             uint32_t m1, unsigned long long S1u, unsigned long long S2u, double S1d,
                                             double S2d, SM& sm) {
  double v0, v1;
  if (INT || N == 0) {
    v0 = (double)k0;
    v1 = (double)k1;
  } else {
    v0 = (double)fkey_inv(k0);
    v1 = (double)fkey_inv(k1);
  }
  const double med = (N & 1) ? v0 : (v0 + v1) / 2.0;
  const double n = (double)N;
  double mu, ex2;
  if (INT) {
    mu = (double)S1u / n;     // S1, S2 < 2^53: exact conversions
    ex2 = (double)S2u / n;
  } else {
    mu = S1d / n;
    ex2 = S2d / n;
  }
  double var = ex2 - mu * mu;
  if (var < 0.0 || N == 0) var = 0.0;
  double sd = __builtin_sqrt(var);
  if (P.robust && N > 0) {
    // 1.4826 * MAD; integer input: m0, m1 are doubled deviations
    double mad;
    if (INT) mad = ((double)m0 + (double)m1) / 4.0;
    else mad = (N & 1) ? (double)fkey_inv(m0) : ((double)fkey_inv(m0) + (double)fkey_inv(m1)) / 2.0;
    sd = MAD_TO_SIGMA * mad;
  }
  sm.median = med;
  sm.sigma = sd;
  const int nT = max(P.nl_t, P.nl_f);
  double pk = 1.0;
  for (int k = 0; k < 16; ++k) {
    if (k < nT) {
      const double f = P.start * pk / (double)(1 << k);
      sm.T[k] = med + sd * (f * P.sens);
      sm.Tf[k] = (float)sm.T[k];
      pk = pk * P.p;
    } else {
      sm.T[k] = 0.0;
      sm.Tf[k] = 0.0f;
    }
  }
}

// The statistics of block b (sm.median, sm.sigma, sm.T) into its BlockState and
// the caller's stats entry (flag totals cleared for the final kernel); threads
// 0 .. max(18, STATS_BYTES / 8) - 1 of the workgroup
template <class SM>
__device__ __forceinline__ void write_block_stats(const DevBlock& b, const DevParams& P, const SM& sm) {
  const int k = threadIdx.x;
  if (k < 18) {
    GLB BlockState* bs = gp<BlockState>(P.bstate) + b.sidx;
    if (k == 0) bs->median = sm.median;
    else if (k == 1) bs->sigma = sm.sigma;
    else bs->T[k - 2] = sm.T[k - 2];
  }
  if (P.stats && k < STATS_BYTES / 8) {
    GLB double* st = (GLB double*)(gp<char>(P.stats) + (int64_t)b.out_idx * STATS_BYTES);
    if (k == 0) st[0] = sm.median;
    else if (k == 1) st[1] = sm.sigma;
    else if (k < 2 + LOF_MAX_LEVELS) st[k] = sm.T[k - 2];
    else *(GLB long long*)(st + k) = 0;   // flagged samples; history rows and padding
  }
}

// PRE: the caller's pre-flagged samples (LOF_OPT_PREFLAGGED) leave every
// statistic; N is then the number of the others (with none, median and stddev 0)
template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

template <bool INT, bool PRE, class SM>
__device__ __forceinline__ void phase_stats(const DevBlock& b, const DevParams& P, SM& sm) {
  typedef typename PowT<INT>::T VT;
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int nch = (b.T + 7) >> 3;
  const uint32_t items = (uint32_t)b.C * (uint32_t)nch;
  const FastDiv fd((uint32_t)nch);
  int64_t N = (int64_t)b.C * b.T;
  if (PRE && tid == 0) sm.nlive = 0u;

  if (INT) {
    for (int i = tid; i < IHIST_WORDS; i += WG) sm.u.ihist[i] = 0u;
  } else {
    for (int i = tid; i < 2 * HBINS; i += WG) (&sm.u.hist[0][0])[i] = 0u;
  }
  __syncthreads();

  unsigned long long s1u = 0, s2u = 0;
  double s1d = 0.0, s2d = 0.0;
  constexpr int U = INT ? 8 : 4;   // chunks of 8 samples in flight per thread
  auto consume = [&](const VT (&v)[8], int nv, uint32_t pm) {
    if (PRE) {
      const int live = __popc(~pm & ((1u << nv) - 1u));
      if (live) atomicAdd(&sm.nlive, (uint32_t)live);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < nv && !((pm >> j) & 1u)) {
        if (INT) {
          // the exact histogram also yields sum(p) and sum(p^2) afterwards
          const uint32_t p = (uint32_t)v[j];
          atomicAdd(&sm.u.ihist[p >> 1], (p & 1u) ? 0x10000u : 1u);
        } else {
          const double d = (double)v[j];
          s1d += d;
          s2d += d * d;
          atomicAdd(&sm.u.hist[0][fkey((float)v[j]) >> 20], 1u);
        }
      }
    }
  };
  // rows back to back (row stride = T): chunk it starts at element 8 * it
  const bool lin = b.dstride == (int64_t)b.T;
  // integer input, every chunk full and aligned: U raw 16-byte loads in flight per
  // thread, then per sample the doubled power 2p = sdot4(d, d) with d = (re, im,
  // re, im): the histogram word of p is at byte offset 2p & ~3 and its counter
  // is 1 << 16 (p & 1)
  auto int_chunks = [&](auto lin_c) __attribute__((always_inline)) {
    constexpr bool LIN = decltype(lin_c)::value;
    const GLB uint8_t* base8 = gp<const uint8_t>(b.data);
    auto load = [&](uint32_t it, uint32_t& pm) __attribute__((always_inline)) {
      int64_t eoff;
      if constexpr (LIN) {
        eoff = (int64_t)it * 8;
        pm = 0u;
      } else {
        const int row = (int)fd.div(it);
        const int t0 = (int)(it - (uint32_t)row * (uint32_t)nch) * 8;
        eoff = (int64_t)row * b.dstride + t0;
        pm = pre8<PRE>(b, row, t0, 8);
      }
      return *(const GLB u32x4*)(base8 + eoff * 2);
    };
    auto add8 = [&](const u32x4& q, uint32_t pm) __attribute__((always_inline)) {
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
      uint32_t p2[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const uint32_t d = __builtin_amdgcn_perm(w[m >> 1], w[m >> 1], (m & 1) ? 0x03020302u : 0x01000100u);
        p2[m] = (uint32_t)__builtin_amdgcn_sdot4((int)d, (int)d, 0, false);
      }
      if (PRE) {
        const int live = __popc(~pm & 0xffu);
        if (live) atomicAdd(&sm.nlive, (uint32_t)live);
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        if (PRE && ((pm >> m) & 1u)) continue;
        atomicAdd((uint32_t*)((unsigned char*)sm.u.ihist + (p2[m] & ~3u)), 1u << ((p2[m] << 3) & 31u));
      }
    };
    uint32_t base = tid;
    // whole rounds of U chunks: every load issued before the first is used
    for (; base + (uint32_t)(U - 1) * WG < items; base += (uint32_t)WG * U) {
      u32x4 q[U];
      uint32_t pm[U];
#pragma unroll
      for (int u = 0; u < U; ++u) q[u] = load(base + (uint32_t)u * WG, pm[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) add8(q[u], pm[u]);
    }
    for (; base < items; base += WG) {
      uint32_t pm;
      const u32x4 q = load(base, pm);
      add8(q, pm);
    }
  };
  if (INT && b.aligned && (b.T & 7) == 0) {
    if (lin && !PRE) int_chunks(BoolC<true>{});
    else int_chunks(BoolC<false>{});
  } else if (b.aligned && (b.T & 7) == 0) {
    // float input, every chunk full and aligned: unconditional loads (clamped
    // index, masked count) so all U loads of a thread are in flight together
    for (uint32_t base = tid; base < items; base += (uint32_t)WG * U) {
      VT v[U][8];
      uint32_t pm[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t it = base + (uint32_t)u * WG;
        const uint32_t ic = it < items ? it : items - 1;
        if (lin && !PRE) {
          load8v_off<INT>(b, (int64_t)ic * 8, v[u]);
          pm[u] = 0u;
        } else {
          const int row = (int)fd.div(ic);
          const int t0 = (int)(ic - (uint32_t)row * (uint32_t)nch) * 8;
          load8v<INT>(b, row, t0, v[u]);
          pm[u] = pre8<PRE>(b, row, t0, 8);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) consume(v[u], base + (uint32_t)u * WG < items ? 8 : 0, pm[u]);
    }
  } else {
    for (uint32_t it = tid; it < items; it += WG) {
      const int row = (int)fd.div(it);
      const int t0 = (int)(it - (uint32_t)row * (uint32_t)nch) * 8;
      VT v[8];
      const int nv = load8<INT>(b, row, t0, v);
      consume(v, nv, pre8<PRE>(b, row, t0, nv));
    }
  }
  if (PRE) {
    __syncthreads();
    N = (int64_t)sm.nlive;
  }
  const uint32_t r0 = N > 0 ? (uint32_t)((N - 1) / 2) : 0u, r1 = (uint32_t)(N / 2);
  bool hist_ok = false;
  if (INT) {
    __syncthreads();   // every wave's histogram increments done
    // the 16-bit fields sum to N exactly when no counter wrapped; then bin p with
    // count c adds c*p and c*p^2 to the exact sums
    uint32_t s = 0;
    for (int i = tid; i < IHIST_WORDS; i += WG) {
      const uint32_t w = sm.u.ihist[i];
      const uint32_t c0 = w & 0xffffu, c1 = w >> 16;
      const uint32_t p0 = 2u * (uint32_t)i, p1 = p0 + 1u;
      s += c0 + c1;
      s1u += (unsigned long long)(c0 * p0 + c1 * p1);   // c <= 2^16 - 1, p0 + p1 < 2^16: below 2^32
      s2u += (unsigned long long)c0 * (p0 * p0) + (unsigned long long)c1 * (p1 * p1);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane == 0) sm.scan[wv] = s;
    __syncthreads();
    uint32_t tot = 0;
    for (int w = 0; w < NW; ++w) tot += sm.scan[w];
    __syncthreads();
    hist_ok = tot == (uint32_t)N;
    if (!hist_ok) {
      // a counter wrapped (some power value occurs 2^16 times or more): the sums
      // from the samples themselves
      s1u = 0;
      s2u = 0;
      for (uint32_t it = tid; it < items; it += WG) {
        const int row = (int)fd.div(it);
        const int t0 = (int)(it - (uint32_t)row * (uint32_t)nch) * 8;
        VT v[8];
        const int nv = load8<INT>(b, row, t0, v);
        const uint32_t pm = pre8<PRE>(b, row, t0, nv);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (j < nv && !((pm >> j) & 1u)) {
            const uint32_t p = (uint32_t)v[j];
            s1u += p;
            s2u += (unsigned long long)(p * p);     // p <= 32768: p*p <= 2^30
          }
        }
      }
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    s1u += __shfl_xor(s1u, d);
    s2u += __shfl_xor(s2u, d);
    s1d += __shfl_xor(s1d, d);
    s2d += __shfl_xor(s2d, d);
  }
  if (lane == 0) {
    sm.red_u[0][wv] = s1u;
    sm.red_u[1][wv] = s2u;
    sm.red_d[0][wv] = s1d;
    sm.red_d[1][wv] = s2d;
  }
  __syncthreads();

  // the block's candidate list for the last pass of a 3-pass radix select (in the
  // call's candidate scratch at the block's mask-word offset; null: read the block)
  GLB uint32_t* cand = P.cand ? gp<uint32_t>(P.cand) + b.mask_off * CAND_PER_WORD : nullptr;
  const uint32_t ccap = (uint32_t)b.C * (uint32_t)((b.T + 63) >> 6) * (uint32_t)CAND_PER_WORD;
  uint32_t k0 = 0, k1 = 0;
  if (N == 0) {
    // every sample pre-flagged: no statistics (median and stddev 0)
  } else if (INT && hist_ok) {
    k0 = find_bin16(sm.u.ihist, r0, sm);
    k1 = (r1 == r0) ? k0 : find_bin16(sm.u.ihist, r1, sm);
  } else {
    radix_select<INT, PRE>(b, sm, r0, r1, !INT, k0, k1, cand, ccap);
  }
  // robust stddev: the middle order statistics of the deviations from the median
  uint32_t m0 = 0, m1 = 0;
  if (P.robust && N > 0) {
    if (INT) {
      const uint32_t med2 = k0 + k1;   // twice the median (an integer)
      if (hist_ok) {
        m0 = find_dev_rank(sm.u.ihist, med2, r0, sm);
        m1 = (r1 == r0) ? m0 : find_dev_rank(sm.u.ihist, med2, r1, sm);
      } else {
        radix_select_k<INT, 32, PRE>(b, sm, r0, r1, false, [med2](VT v) {
          const int d = 2 * (int)(uint32_t)v - (int)med2;
          return (uint32_t)(d < 0 ? -d : d);
        }, m0, m1, cand, ccap);
      }
    } else {
      const double v0 = (double)fkey_inv(k0), v1 = (double)fkey_inv(k1);
      const double med = (N & 1) ? v0 : (v0 + v1) / 2.0;
      radix_select_k<INT, 32, PRE>(b, sm, r0, r1, false, [med](VT v) {
        return fkey((float)__builtin_fabs((double)v - med));
      }, m0, m1, cand, ccap);
    }
  }

  if (tid == 0) {
    unsigned long long S1u = 0, S2u = 0;
    double S1d = 0.0, S2d = 0.0;
    for (int w = 0; w < NW; ++w) {
      S1u += sm.red_u[0][w];
      S2u += sm.red_u[1][w];
      S1d += sm.red_d[0][w];
      S2d += sm.red_d[1][w];
    }
    stats_finish<INT>(P, N, k0, k1, m0, m1, S1u, S2u, S1d, S2d, sm);
  }
  __syncthreads();
}

// Thresholds of a block from its BlockState into shared memory.  Integer input
// also gets exact window thresholds: flag iff S > floor(c * T_k), stored packed
// against the window word D = S*256 + 4c as G = floor(c*T_k)*256 + 4c + 255,
// indexed by the low bits (D >> 2) & 63.  Count 64 and count 0 share index 0: a
// window with no unflagged sample has D = 0, so that entry is max(G_64, 0), which
// D = 0 never exceeds and every 64-sample window with G_64 < 0 does.
template <bool INT, class SM>
__device__ __forceinline__ void load_thresholds(const DevBlock& b, const DevParams& P, SM& sm) {
  const int tid = thread_id();
  const GLB BlockState* bs = gp<const BlockState>(P.bstate) + b.sidx;
  if (tid < 16) {
    const double t = bs->T[tid];
    sm.T[tid] = t;
    sm.Tf[tid] = (float)t;
  }
  __syncthreads();
  if (INT) {
    for (int i = tid; i < ST_MAX_LEVELS * 128; i += WG) {
      const int k = i >> 7, idx = i & 127;
      const int c = idx == 0 ? 64 : idx;
      const double T = sm.T[k];
      const double cd = (double)c;
      const double prod = cd * T;
      const double err = __builtin_fma(cd, T, -prod);
      double fl = __builtin_floor(prod);
      if (prod == fl && err < 0.0) fl -= 1.0;
      // S lies in [0, 2^21]: a floor at or above 2^21 never flags, one below 0 always
      int32_t g;
      if (fl >= 2097152.0) g = 0x7fffffff;
      else g = (int32_t)__builtin_fmax(fl, -1.0) * 256 + 4 * c + 255;
      if (idx == 0) g = g > 0 ? g : 0;
      sm.G[k][idx] = g;
    }
    __syncthreads();
  }
}

// ===================================================================== SumThreshold core
// One-dimensional SumThreshold (Sec. 2.1) over a sequence of n positions held by
// a group of lanes (L per lane, lane_in_group = lig).  Levels are synchronous:
// every window of level k is judged on the mask after level k-1; flagged samples
// are left out of the window's sum and count; a window whose unflagged mean
// exceeds T_k flags all its samples.  Only full windows (s + I <= n) are judged.
//
// Integer input: v = p*256 + 4 for an unflagged sample, 0 for a flagged one, so a
// window word D = S*256 + 4c packs the exact unflagged sum S and count c; the test
// S > floor(c*T_k) is D > G_k[c].  Float input: float32 sums and counts, test
// S > c*T_k in float32.  Window sums of level k are D_k(s) = D_{k-1}(s) +
// D_{k-1}(s + I/2); after a level that changed the mask they are rebuilt from v.

template <int L, int H, class VT>
__device__ __forceinline__ void dbl_step(VT (&D)[L]) {
  static_assert(H <= L, "window half must fit in one lane");
  VT nb[H];
#pragma unroll
  for (int m = 0; m < H; ++m) nb[m] = shl1(D[m]);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const VT o = (i + H < L) ? D[(i + H < L) ? i + H : 0] : nb[(i + H >= L) ? i + H - L : 0];
    D[i] = D[i] + o;
  }
}

template <int L, int J, int M, class VT>
__device__ __forceinline__ void rebuild(VT (&D)[L]) {
  if constexpr (J < M) {
    dbl_step<L, (1 << J)>(D);
    rebuild<L, J + 1, M>(D);
  }
}

// window-start bits wf (bit i <-> start lig*L+i) -> flagged positions of this lane:
// OR over starts s in [j-I+1, j], with starts of up to two lanes to the left.
template <int L, int I>
__device__ __forceinline__ uint64_t spread(uint64_t wf, int lig) {
  uint64_t p1 = shr1_64(wf);
  uint64_t p2 = 0;
  if (L < 64) p2 = shr1_64(p1);
  if (lig == 0) p1 = 0;
  if (lig <= 1) p2 = 0;
  uint64_t xlo;
  if (L == 64) xlo = p1;
  else if (L == 48) xlo = (p1 << 16) | (p2 >> 32);
  else if (L == 32) xlo = (p1 << 32) | p2;
  else xlo = 0;  // L < 32 only with groups of one lane
  uint64_t xhi = wf;
#pragma unroll
  for (int d = 1; d < I; d <<= 1) {
    xhi |= (xhi << d) | (xlo >> (64 - d));
    xlo |= xlo << d;
  }
  return xhi;
}

template <bool INT, int L, int K, class LD, class SM>
__device__ __forceinline__ void st_level(LD& ld, typename PowT<INT>::T (&D)[L], float (&Nc)[L], uint64_t& fm,
                                         bool& dirty, const int lig, const int n, const int pos0,
                                         const uint64_t vmask, const SM& sm) {
  constexpr int I = 1 << K;
  if constexpr ((I >> 1) <= L) {
    if constexpr (K > 0) {
      if (dirty) {
        ld.fill(fm, D, Nc);
        rebuild<L, 0, K - 1>(D);
        if constexpr (!INT) rebuild<L, 0, K - 1>(Nc);
      }
      dbl_step<L, (I >> 1)>(D);
      if constexpr (!INT) dbl_step<L, (I >> 1)>(Nc);
    }
    // judge the windows: first only whether any window of the wave exceeds
    // (compare + scalar OR; windows past the sequence end may raise a false
    // alarm, which costs only the second loop), then the per-lane window bits.
    const int nvw = n - I + 1 - pos0;      // valid window starts in this lane: i < nvw
    unsigned long long any = 0;
    uint32_t lo = 0, hi = 0;
    if constexpr (INT) {
      const int32_t* Gk = sm.G[K];
      bool scalar = false;
      if constexpr (K == 0) scalar = __ballot(fm != 0) == 0;
      if (scalar) {
        const int32_t g = Gk[1];
#pragma unroll
        for (int i = 0; i < L; ++i) any |= __ballot((int32_t)(uint32_t)D[i] > g);
        if (any) {
#pragma unroll
          for (int i = 0; i < L; ++i) {
            const uint32_t h = ((int32_t)(uint32_t)D[i] > g) ? 1u : 0u;
            if (i < 32) lo |= h << i; else hi |= h << (i - 32);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < L; ++i) {
          const uint32_t d = (uint32_t)D[i];
          any |= __ballot((int32_t)d > Gk[(d >> 2) & 63u]);
          if ((i & 15) == 15) __builtin_amdgcn_sched_barrier(0);   // bound the hoisted table reads
        }
        if (any) {
#pragma unroll
          for (int i = 0; i < L; ++i) {
            const uint32_t d = (uint32_t)D[i];
            const uint32_t h = ((int32_t)d > Gk[(d >> 2) & 63u]) ? 1u : 0u;
            if (i < 32) lo |= h << i; else hi |= h << (i - 32);
            if ((i & 15) == 15) __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    } else {
      const float Tk = sm.Tf[K];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const float c = Nc[i];
        any |= __ballot(c > 0.0f && (float)D[i] > c * Tk);
      }
      if (any) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
          const float c = Nc[i];
          const uint32_t h = (c > 0.0f && (float)D[i] > c * Tk) ? 1u : 0u;
          if (i < 32) lo |= h << i; else hi |= h << (i - 32);
        }
      }
    }
    if (any == 0) {
      dirty = false;
      return;
    }
    uint64_t wf = (uint64_t)lo | ((uint64_t)hi << 32);
    wf &= lowmask(nvw) & vmask;
    const uint64_t nb = spread<L, I>(wf, lig) & vmask;
    const uint64_t changed = nb & ~fm;
    fm |= nb;
    dirty = __ballot(changed != 0) != 0;
  }
}

// Loader interface: fill(fm, D, Nc) sets D (and Nc, float path) to the level-0
// window values of the lane's L positions under mask fm.
template <bool INT, int L, class LD, class SM>
__device__ __forceinline__ uint64_t st_core(LD& ld, uint64_t fm, const int lig, const int n, const int kfirst,
                            const int nlev, const SM& sm) {
  typedef typename PowT<INT>::T VT;
  VT D[L];
  float Nc[L];
  const int pos0 = lig * L;
  const int nval = clampi(n - pos0, 0, L);
  const uint64_t vmask = lowmask(nval);
  int kend = 0;
  while (kend < nlev && (1 << kend) <= n) ++kend;   // levels with I <= n
  ld.fill(fm, D, Nc);
  bool dirty = false;
#define LOF_LEVEL(K) \
  if (kfirst <= K && K < kend) st_level<INT, L, K>(ld, D, Nc, fm, dirty, lig, n, pos0, vmask, sm);
  LOF_LEVEL(0)
  LOF_LEVEL(1)
  LOF_LEVEL(2)
  LOF_LEVEL(3)
  LOF_LEVEL(4)
  LOF_LEVEL(5)
  LOF_LEVEL(6)
#undef LOF_LEVEL
  return fm;
}

// Integer input, prefix form.  A lane keeps the inclusive prefix sums
// bit b of x as 0 or 1 (v_bfe_u32).  Opaque, so that `acc + __umul24(bit01(x, b), v)`
// stays one bit-field extract and one v_mad_u32_u24 instead of a compare and a
// select.  A packed sample value is below 2^24 (p <= 2^15), as the 24-bit multiply
// needs.
__device__ __forceinline__ uint32_t bit01(uint32_t x, int b) {
  uint32_t k = __builtin_amdgcn_ubfe(x, b, 1);
  asm("" : "+v"(k));
  return k;
}

// Window bits are assembled most significant first: acc = (acc << 1) | sign(g - d),
// one v_alignbit per window.  For every full window d <= 2^30 and
// -2^30 < g < 2^31, so g - d does not overflow and its sign is (d > g).
// g - d is an opaque subtract: left to the compiler, g is folded into the window
// difference, (g + Y[i-1]) - dpp(Y[j]), and that combined DPP subtract gave wrong
// lane-crossing windows on gfx950 while the plain form, dpp(Y[j]) - Y[i-1], is
// exact.  (An empty asm on d has the same effect but costs a copy of d.)
__device__ __forceinline__ uint32_t push_bit(uint32_t acc, int32_t g, uint32_t d) {
  uint32_t t;
  asm("v_sub_u32 %0, %1, %2" : "=v"(t) : "v"(g), "v"(d));
  return __builtin_amdgcn_alignbit(acc, t, 31);
}

// Y[i] = sum of v over the group's positions up to lig*L + i, modulo 2^32: every
// true window word is below 2^30, so differences of prefixes are exact.  The
// window of I starting at lane position i is Y(i+I-1) - Y(i-1); Y(j) for j >= L
// comes from the next one or two lanes by DPP, Y(-1) is the prefix before the
// lane (0 in the first lane of a group).  A level that changed the mask rebuilds
// the prefixes of each lane from its own samples only: the later lanes are not
// told, so a lane's prefixes stay too large by what the lanes before it dropped.
// Windows inside a lane do not see that offset; a window reaching into the next
// lane subtracts E, the total this lane has dropped so far, and one reaching two
// lanes ahead subtracts E + E(next lane).
template <int L>
__device__ __forceinline__ uint32_t px_get(const uint32_t (&Y)[L], int j) {
  if (j < L) return Y[j < L ? j : 0];
  if (j < 2 * L) return shl1(Y[(j >= L && j < 2 * L) ? j - L : 0]);
  return shl1(shl1(Y[(j >= 2 * L && j < 3 * L) ? j - 2 * L : 0]));
}

// CORR: the wave has dropped samples, so windows crossing lanes take e1 / e2
template <int L, bool CORR>
__device__ __forceinline__ uint32_t px_win(const uint32_t (&Y)[L], uint32_t yprev, int i, int I, uint32_t e1,
                                           uint32_t e2) {
  const uint32_t lo = (i == 0) ? yprev : Y[(i > 0) ? i - 1 : 0];
  const int j = i + I - 1;
  if (!CORR || j < L) return px_get<L>(Y, j) - lo;
  return px_get<L>(Y, j) - (lo + (j < 2 * L ? e1 : e2));
}

// v under mask fm -> prefixes; returns Y(-1)
// The rows start with nothing flagged, so level 0 (windows of one sample, count 1)
// is tested on the loaded values themselves: w0 gets bit i iff v_i > g0.
template <int L, class LD>
__device__ __forceinline__ uint32_t px_fill(LD& ld, uint32_t (&Y)[L], int lig, int G, uint32_t& lane_total,
                                            const int32_t g0, uint64_t& w0) {
  float unused[L];
  ld.fill(0ull, Y, unused);
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int i = L - 1; i >= 0; --i) {
    if (i >= 32) hi = push_bit(hi, g0, Y[i]); else lo = push_bit(lo, g0, Y[i]);
  }
  w0 = (uint64_t)lo | ((uint64_t)hi << 32);
  uint32_t run = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    run += Y[i];
    Y[i] = run;
  }
  lane_total = run;
  uint32_t incl = run;
  for (int d = 1; d < G; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, G);
    if (lig >= d) incl += y;
  }
  const uint32_t off = incl - run;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    Y[i] += off;
    // opaque from here on: otherwise the compiler keeps the L loaded values
    // alive to re-derive Y[i] - Y[i-1] later, which costs L registers
    asm("" : "+v"(Y[i]));
  }
  return off;
}

// Remove the samples of `drop` (newly flagged positions of the lane) from the
// lane's prefixes: a sample's packed value is Y[i] - Y[i-1], and the prefixes are
// re-accumulated from yprev over the kept samples.  E grows by what the lane lost.
template <int L>
__device__ __forceinline__ void px_drop(uint32_t (&Y)[L], const uint32_t yprev, uint64_t drop, uint32_t& E) {
  const uint32_t klo = ~(uint32_t)drop, khi = ~(uint32_t)(drop >> 32);
  const uint32_t old_end = Y[L - 1];
  // sample values first, last to first, then the kept ones re-accumulated: both
  // steps overwrite Y[i] in place (no register rotation)
#pragma unroll
  for (int i = L - 1; i >= 0; --i) Y[i] -= (i > 0) ? Y[(i > 0) ? i - 1 : 0] : yprev;
  uint32_t acc = yprev;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    acc += __umul24(bit01((i < 32 ? klo : khi), i & 31), Y[i]);   // one v_mad_u32_u24
    Y[i] = acc;
  }
  E += old_end - acc;
}

#ifndef LOF_PXB
#define LOF_PXB 8
#endif
constexpr int PXB = LOF_PXB;   // windows per batch of table reads

template <int L, int K, class SM>
__device__ __forceinline__ void st_level_px(uint32_t (&Y)[L], const uint32_t yprev, uint32_t& E, uint64_t& fm,
                                            uint64_t& pend, const int lig, const int n, const int pos0,
                                            const uint64_t vmask, const SM& sm) {
  constexpr int I = 1 << K;
  static_assert(I <= 2 * L && L % PXB == 0, "a window may reach at most two lanes ahead");
  if (__ballot(pend != 0) != 0) px_drop<L>(Y, yprev, pend, E);
  pend = 0;
  const int nvw = n - I + 1 - pos0;
  const int32_t* Gk = sm.G[K];
  uint32_t lo = 0, hi = 0;
  if (__ballot(fm != 0) == 0) {
    // nothing flagged in the wave: every full window counts I samples
    const int32_t g = Gk[I];
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
      const uint32_t d = px_win<L, false>(Y, yprev, i, I, 0u, 0u);
      if (i >= 32) hi = push_bit(hi, g, d); else lo = push_bit(lo, g, d);
      if (i % PXB == 0) __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // PXB windows at a time: their table reads in flight before they are used
    const uint32_t e1 = E, e2 = (I + L - 1 > 2 * L) ? E + shl1(E) : E;
#pragma unroll
    for (int i0 = L - PXB; i0 >= 0; i0 -= PXB) {
      uint32_t d[PXB];
      int32_t g[PXB];
#pragma unroll
      for (int j = 0; j < PXB; ++j) {
        d[j] = px_win<L, true>(Y, yprev, i0 + j, I, e1, e2);
        g[j] = Gk[(d[j] >> 2) & 63u];
      }
#pragma unroll
      for (int j = PXB - 1; j >= 0; --j) {
        if (i0 + j >= 32) hi = push_bit(hi, g[j], d[j]); else lo = push_bit(lo, g[j], d[j]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  uint64_t wf = (uint64_t)lo | ((uint64_t)hi << 32);
  wf &= lowmask(nvw) & vmask;
  if (__ballot(wf != 0) == 0) return;
  const uint64_t nb = spread<L, I>(wf, lig) & vmask;
  pend = nb & ~fm;
  fm |= nb;
}

// psum: the power sum of the lane's samples (the first fill runs with no flags:
// its lane total is 256 * sum(p) + 4 * nval, exactly, below 2^30)
template <int L, class LD, class SM>
__device__ __forceinline__ uint64_t st_core_px(LD& ld, const int lig, const int G, const int n, const int nlev,
                                               const SM& sm, uint32_t& psum, GLB uint64_t* row_sum = nullptr) {
  uint32_t Y[L];
  uint64_t fm = 0;
  const int pos0 = lig * L;
  const int nval = clampi(n - pos0, 0, L);
  const uint64_t vmask = lowmask(nval);
  int kend = 0;
  while (kend < nlev && (1 << kend) <= n) ++kend;   // levels with I <= n
  uint32_t lane_total;
  uint64_t w0;
  const uint32_t yprev = px_fill<L>(ld, Y, lig, G, lane_total, sm.G[0][1], w0);
  psum = (lane_total - 4u * (uint32_t)nval) >> 8;
  if (row_sum != nullptr) {
    // the row's power sum (exact) for the history flagger, stored now so that
    // nothing extra stays live through the levels
    uint32_t rs = psum;
    for (int d = G >> 1; d >= 1; d >>= 1) rs += __shfl_xor(rs, d, G);
    if (ld.ok && lig == 0) *row_sum = rs;
  }
  uint64_t pend = 0;
  uint32_t E = 0;
  if (kend > 0) {
    // level 0: every valid position is a full window; a window flags only itself
    fm = w0 & vmask;
    pend = fm;
  }
#define LOF_PLEVEL(K) \
  if (K < kend) st_level_px<L, K>(Y, yprev, E, fm, pend, lig, n, pos0, vmask, sm);
  LOF_PLEVEL(1)
  LOF_PLEVEL(2)
  LOF_PLEVEL(3)
  LOF_PLEVEL(4)
  LOF_PLEVEL(5)
  LOF_PLEVEL(6)
#undef LOF_PLEVEL
  return fm;
}

// ---- loaders
struct RowSrc {        // the descriptor fields a row loader needs, by value
  const void* data;
  int64_t dstride;
  int dtype, aligned;
  __device__ explicit RowSrc(const DevBlock& d) : data(d.data), dstride(d.dstride), dtype(d.dtype), aligned(d.aligned) {}
};

template <bool INT, int L>
struct TimeLoader {
  RowSrc s;
  int row, q, nval;   // q: absolute time of the lane's first position
  bool ok;
  __device__ __forceinline__ void fill(uint64_t fm, typename PowT<INT>::T (&D)[L], float (&Nc)[L]) {
    if (INT) {
      const GLB uint8_t* rb = gp<const uint8_t>(s.data) + ((int64_t)row * s.dstride + q) * 2;
      if (ok && nval == L && s.aligned) {
#pragma unroll
        for (int j = 0; j < L / 8; ++j) {
          const u32x4 w = *(const GLB u32x4*)(rb + 16 * j);
          const uint32_t a[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int i0 = 8 * j + 2 * m;
            const uint32_t p0 = ci8_power(a[m] & 0xffffu), p1 = ci8_power(a[m] >> 16);
            D[i0] = ((fm >> i0) & 1ull) ? 0u : p0 * 256u + 4u;
            D[i0 + 1] = ((fm >> (i0 + 1)) & 1ull) ? 0u : p1 * 256u + 4u;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < L; ++i) {
          const bool live = ok && i < nval && !((fm >> i) & 1ull);
          D[i] = live ? ci8_power(*(const GLB uint16_t*)(rb + 2 * i)) * 256u + 4u : 0u;
        }
      }
    } else {
      float p[L];
      if (s.dtype == 2) {
        const GLB float* rb = gp<const float>(s.data) + (int64_t)row * s.dstride + q;
        if (ok && nval == L && s.aligned) {
#pragma unroll
          for (int j = 0; j < L / 4; ++j) {
            const f32x4 w = *(const GLB f32x4*)(rb + 4 * j);
            p[4 * j] = w.x; p[4 * j + 1] = w.y; p[4 * j + 2] = w.z; p[4 * j + 3] = w.w;
          }
        } else {
#pragma unroll
          for (int i = 0; i < L; ++i) p[i] = (ok && i < nval) ? rb[i] : 0.0f;
        }
      } else {
        const GLB f32x2* rb = gp<const f32x2>(s.data) + (int64_t)row * s.dstride + q;
        const bool amp = s.dtype == 3;
        if (ok && nval == L && s.aligned) {
#pragma unroll
          for (int j = 0; j < L / 2; ++j) {
            const f32x4 w = *(const GLB f32x4*)(rb + 2 * j);
            p[2 * j] = amp ? c64_amp(w.x, w.y) : c64_power(w.x, w.y);
            p[2 * j + 1] = amp ? c64_amp(w.z, w.w) : c64_power(w.z, w.w);
          }
        } else {
#pragma unroll
          for (int i = 0; i < L; ++i) {
            float r = 0.0f;
            if (ok && i < nval) {
              const f32x2 z = rb[i];
              r = amp ? c64_amp(z.x, z.y) : c64_power(z.x, z.y);
            }
            p[i] = r;
          }
        }
      }
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const bool live = i < nval && ok && !((fm >> i) & 1ull);
        D[i] = (typename PowT<INT>::T)(live ? p[i] : 0.0f);
        Nc[i] = live ? 1.0f : 0.0f;
      }
    }
  }
};

// float rows of complex input: the lane's powers (or amplitudes) formed once and
// kept, so a level that changed the mask rebuilds its window sums from registers
// instead of reloading the row and forming them again
template <int L>
struct CachedRow {
  float V[L];
  int nval;
  bool ok;
  template <class LD>
  __device__ __forceinline__ explicit CachedRow(LD& ld) : nval(ld.nval), ok(ld.ok) {
    float Nc[L];
    ld.fill(0ull, V, Nc);
  }
  __device__ __forceinline__ void fill(uint64_t fm, float (&D)[L], float (&Nc)[L]) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const bool live = ok && i < nval && !((fm >> i) & 1ull);
      D[i] = live ? V[i] : 0.0f;
      Nc[i] = live ? 1.0f : 0.0f;
    }
  }
};

// frequency loader: one column of the LDS slab (rows = channels)
template <bool INT, int L>
struct TileLoader {
  const typename TileOf<INT>::T* tile;
  int stride, col, ch0, nval;
  bool ok;
  __device__ __forceinline__ void fill(uint64_t fm, typename PowT<INT>::T (&D)[L], float (&Nc)[L]) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const bool valid = ok && i < nval;
      const bool live = valid && !((fm >> i) & 1ull);
      if (INT) {
        const uint32_t p = valid ? (uint32_t)tile[(ch0 + i) * stride + col] : 0u;
        D[i] = (typename PowT<INT>::T)(live ? p * 256u + 4u : 0u);
      } else {
        const float p = valid ? (float)tile[(ch0 + i) * stride + col] : 0.0f;
        D[i] = (typename PowT<INT>::T)(live ? p : 0.0f);
        Nc[i] = live ? 1.0f : 0.0f;
      }
    }
  }
};

// ---- bit output of a row layout (lane bits at lig*L) into u64 row words
template <int L>
__device__ __forceinline__ void write_row_bits(GLB uint64_t* rowp, int W, uint64_t fm, int lig, int G, bool ok) {
  if (L == 64) {
    if (ok && lig < W) rowp[lig] = fm;
  } else if (L == 32) {
    const uint64_t nx = shl1_64(fm);
    if (G == 1) {
      if (ok) rowp[0] = fm;
    } else if ((lig & 1) == 0) {
      if (ok && (lig >> 1) < W) rowp[lig >> 1] = fm | (nx << 32);
    }
  } else if (L == 48) {
    const uint64_t nx = quad_next_64(fm);
    const int j = lig & 3;
    if (j < 3) {
      const uint64_t word = (fm >> (16 * j)) | (nx << (48 - 16 * j));
      const int widx = (lig >> 2) * 3 + j;
      if (ok && widx < W) rowp[widx] = word;
    }
  } else {
    if (ok && G == 1) rowp[0] = fm;   // L < 32: one lane per row
  }
}

__device__ __forceinline__ uint64_t get_bits(const GLB uint64_t* rowp, int W, int q, int L) {
  const int w = q >> 6, o = q & 63;
  uint64_t r = (w < W) ? (ld_mask(rowp + w) >> o) : 0ull;
  if (o != 0 && o + L > 64 && w + 1 < W) r |= ld_mask(rowp + w + 1) << (64 - o);
  return r & lowmask(L);
}

// set one bit of a u64 word array in LDS (32-bit atomic on the half that holds it)
__device__ __forceinline__ void or_bit_lds(uint64_t* w, int idx, int bit) {
  uint32_t* h = reinterpret_cast<uint32_t*>(w) + 2 * idx + (bit >> 5);
  atomicOr(h, 1u << (bit & 31));
}

// ===================================================================== phase B
// CX: float rows of complex input, the formed powers kept in registers
template <bool INT, int L, bool CX, class SM>
__device__ __forceinline__ void phase_time(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, C = b.C;
  const int W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int nlev = min(P.nl_t, ST_MAX_LEVELS);
  if (T <= 64 * L) {
    int G = 1;
    while (G * L < T) G <<= 1;
    const int R = 64 / G, lig = lane & (G - 1), grp = lane / G;
    // a chunk is NW * R rows: each wave takes its R rows once (no loop, so
    // nothing is hoisted and held across rows)
    const int rb = chunk * NW * R + wv * R;
    if (rb < C) {
      const int row = rb + grp;
      const bool ok = row < C;
      TimeLoader<INT, L> ld{RowSrc(b), ok ? row : 0, lig * L, clampi(T - lig * L, 0, L), ok};
      uint64_t fm;
      if constexpr (INT) {
        uint32_t psum;
        fm = st_core_px<L>(ld, lig, G, T, nlev, sm, psum,
                           gp<uint64_t>(P.rowsum) + (int64_t)b.sidx * P.maxC + (ok ? row : 0));
      } else if constexpr (CX) {
        // complex input: the powers (or amplitudes) are formed once per lane
        CachedRow<L> cr(ld);
        fm = st_core<INT, L>(cr, 0ull, lig, T, 0, nlev, sm);
      } else {
        fm = st_core<INT, L>(ld, 0ull, lig, T, 0, nlev, sm);
      }
      // the row index again from the thread id: holding it through the levels
      // would take registers the levels need
      const int t2 = thread_id();
      const int row2 = chunk * NW * R + (t2 >> 6) * R + (t2 & 63) / G;
      write_row_bits<L>(m0 + (int64_t)(ok ? row2 : 0) * W, W, fm, lig, G, ok);
    }
  } else if constexpr (L == 64) {
    // long rows (only laid out with L == 64): segments of 64*L positions,
    // SEG_CORE finished positions each
    const int row = chunk * NW + wv;
    if (row < C) {
      uint64_t rsum = 0;
      for (int c0 = 0; c0 < T; c0 += SEG_CORE) {
        const int c1 = min(T, c0 + SEG_CORE);
        const int q0 = max(0, c0 - SEG_HALO);
        const int n = min(T, q0 + 64 * L) - q0;
        TimeLoader<INT, L> ld{RowSrc(b), row, q0 + lane * L, clampi(n - lane * L, 0, L), true};
        uint64_t fm;
        const int pos = q0 + lane * L;   // L == 64: one word per lane
        const bool core = pos >= c0 && pos < c1;
        if constexpr (INT) {
          uint32_t psum;
          fm = st_core_px<L>(ld, lane, 64, n, nlev, sm, psum);
          if (!core) psum = 0;
          for (int d = 32; d >= 1; d >>= 1) psum += __shfl_xor(psum, d);   // < 2^27 per segment
          rsum += psum;
        } else {
          fm = st_core<INT, L>(ld, 0ull, lane, n, 0, nlev, sm);
        }
        if (core) m0[(int64_t)row * W + (pos >> 6)] = fm;
      }
      if (INT && lane == 0) gp<uint64_t>(P.rowsum)[(int64_t)b.sidx * P.maxC + row] = rsum;
    }
  }
}

// ---- Phase B with caller-supplied pre-flags (LOF_OPT_PREFLAGGED)
// pre-flag bits of a lane's nval <= L positions from time q of a row
template <int L>
__device__ __forceinline__ uint64_t pre_bits(const DevBlock& b, int row, int q, int nval) {
  const GLB uint8_t* fb = gp<const uint8_t>(b.flags) + (int64_t)row * b.fstride + q;
  uint64_t m = 0;
  if (b.faligned && nval == L && (q & 15) == 0) {
#pragma unroll
    for (int j = 0; j < L / 16; ++j) {
      const u32x4 w = *(const GLB u32x4*)(fb + 16 * j);
      const uint32_t a[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int k = 0; k < 16; ++k) m |= ((a[k >> 2] >> (8 * (k & 3))) & 0xffu) ? (1ull << (16 * j + k)) : 0ull;
    }
  } else {
    for (int i = 0; i < nval; ++i) m |= fb[i] ? (1ull << i) : 0ull;
  }
  return m;
}

// exact power sum of a lane's valid positions, pre-flagged ones included (the
// history flagger subtracts the power of every flagged sample from the row sum)
template <int L>
__device__ __forceinline__ uint32_t lane_power_sum(TimeLoader<true, L>& ld) {
  uint32_t D[L];
  float Nc[L];
  ld.fill(0ull, D, Nc);
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) s += D[i];
  return (s - 4u * (uint32_t)(ld.ok ? ld.nval : 0)) >> 8;   // D = 256 p + 4: below 2^30
}

// SumThreshold along time from the pre-flags: each lane's positions start with
// its pre-flag bits (pre-flagged samples leave the window sums and counts), the
// windows built by doubling; integer rows also store their exact power sum
template <bool INT, int L, class SM>
__device__ __forceinline__ void phase_time_pre(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, C = b.C;
  const int W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int nlev = min(P.nl_t, ST_MAX_LEVELS);
  if (T <= 64 * L) {
    int G = 1;
    while (G * L < T) G <<= 1;
    const int R = 64 / G, lig = lane & (G - 1), grp = lane / G;
    const int rb = chunk * NW * R + wv * R;
    if (rb < C) {
      const int row = rb + grp;
      const bool ok = row < C;
      const int q = lig * L, nval = clampi(T - q, 0, L);
      TimeLoader<INT, L> ld{RowSrc(b), ok ? row : 0, q, nval, ok};
      const uint64_t pre = ok ? pre_bits<L>(b, row, q, nval) : 0ull;
      if constexpr (INT) {
        uint32_t rs = lane_power_sum<L>(ld);
        for (int d = G >> 1; d >= 1; d >>= 1) rs += __shfl_xor(rs, d, G);
        if (ok && lig == 0) gp<uint64_t>(P.rowsum)[(int64_t)b.sidx * P.maxC + row] = rs;
      }
      const uint64_t fm = st_core<INT, L>(ld, pre, lig, T, 0, nlev, sm);
      write_row_bits<L>(m0 + (int64_t)(ok ? row : 0) * W, W, fm, lig, G, ok);
    }
  } else if constexpr (L == 64) {
    // long rows: segments of 64*L positions, SEG_CORE finished positions each
    const int row = chunk * NW + wv;
    if (row < C) {
      uint64_t rsum = 0;
      for (int c0 = 0; c0 < T; c0 += SEG_CORE) {
        const int c1 = min(T, c0 + SEG_CORE);
        const int q0 = max(0, c0 - SEG_HALO);
        const int n = min(T, q0 + 64 * L) - q0;
        const int pos = q0 + lane * L;
        const int nvl = clampi(n - lane * L, 0, L);
        TimeLoader<INT, L> ld{RowSrc(b), row, pos, nvl, true};
        const uint64_t pre = pre_bits<L>(b, row, pos, nvl);
        const bool core = pos >= c0 && pos < c1;
        if constexpr (INT) {
          uint32_t ps = core ? lane_power_sum<L>(ld) : 0u;
          for (int d = 32; d >= 1; d >>= 1) ps += __shfl_xor(ps, d);   // < 2^27 per segment
          rsum += ps;
        }
        const uint64_t fm = st_core<INT, L>(ld, pre, lane, n, 0, nlev, sm);
        if (core) m0[(int64_t)row * W + (pos >> 6)] = fm;
      }
      if (INT && lane == 0) gp<uint64_t>(P.rowsum)[(int64_t)b.sidx * P.maxC + row] = rsum;
    }
  }
}

// Frequency layout: columns of C channels; LF channels per lane, G lanes per
// column (LF = 16 or 32 with G = 1 for C <= 32, else LF = 32 and G = C/32 rounded
// up to a power of two).  The block is walked in slabs of NW*64/G columns staged
// in LDS (powers and the mask words covering the slab).
struct FreqShape {
  int LFc, G, cpw, cpi, stride, lig, colw, ch0, nval;
  __device__ FreqShape(int C, int lane) {
    LFc = C <= 16 ? 16 : 32;
    G = 1;
    while (G * LFc < C) G <<= 1;
    cpw = 64 / G;
    cpi = NW * cpw;
    stride = cpi + 1;
    lig = lane & (G - 1);
    colw = lane / G;
    ch0 = lig * LFc;
    nval = clampi(C - ch0, 0, LFc);
  }
};

template <bool INT, bool POWERS, class SM>
__device__ __forceinline__ void stage_slab(const DevBlock& b, SM& sm, const GLB uint64_t* m0, int W, int it0, int ncols, int wb,
                           int nwl, int stride) {
  typedef typename PowT<INT>::T VT;
  const int tid = thread_id(), C = b.C;
  const FastDiv fw((uint32_t)nwl);
  for (int i = tid; i < C * nwl; i += WG) {
    const int c = (int)fw.div((uint32_t)i), j = i - c * nwl;
    sm.u.f.w[i] = m0[(int64_t)c * W + wb + j];
  }
  if constexpr (POWERS) {
    const int nch8 = (ncols + 7) >> 3;
    const FastDiv f8((uint32_t)nch8);
    for (int i = tid; i < C * nch8; i += WG) {
      const int c = (int)f8.div((uint32_t)i), j = i - c * nch8;
      VT v[8];
      if (b.aligned && it0 + 8 * j + 8 <= b.T) load8v<INT>(b, c, it0 + 8 * j, v);
      else load8<INT>(b, c, it0 + 8 * j, v);
#pragma unroll
      for (int q = 0; q < 8; ++q) sm.u.f.t[c * stride + 8 * j + q] = (typename TileOf<INT>::T)v[q];
    }
  }
}

template <bool INT, int LF, class SM>
__device__ __forceinline__ void phase_freq_l(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, C = b.C;
  const int W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int nlev = min(P.nl_f, ST_MAX_LEVELS);
  const FreqShape fs(C, lane);
  const int span = max(fs.cpi, 64);
  for (int it0 = chunk * span; it0 < T && it0 < (chunk + 1) * span; it0 += fs.cpi) {
    const int ncols = min(fs.cpi, T - it0);
    const int wb = it0 >> 6;
    const int nwl = ((it0 + ncols - 1) >> 6) - wb + 1;
    stage_slab<INT, true>(b, sm, m0, W, it0, ncols, wb, nwl, fs.stride);
    __syncthreads();
    const int col = wv * fs.cpw + fs.colw;
    const int t = it0 + col;
    const bool ok = col < ncols;
    const int tt = ok ? t : it0;
    const int wsel = (tt >> 6) - wb, bsel = tt & 63;
    uint64_t fm0 = 0;
#pragma unroll
    for (int i = 0; i < LF; ++i)
      if (i < fs.nval) fm0 |= ((sm.u.f.w[(fs.ch0 + i) * nwl + wsel] >> bsel) & 1ull) << i;
    if (!ok) fm0 = 0;
    TileLoader<INT, LF> ld{sm.u.f.t, fs.stride, ok ? col : 0, fs.ch0, fs.nval, ok};
    const uint64_t fm = st_core<INT, LF>(ld, fm0, fs.lig, C, 1, nlev, sm);
    uint64_t nb = ok ? (fm & ~fm0) : 0ull;
    while (nb) {
      const int i = __builtin_ctzll(nb);
      nb &= nb - 1;
      or_bit_lds(sm.u.f.w, (fs.ch0 + i) * nwl + wsel, bsel);
    }
    __syncthreads();
    for (int i = tid; i < C * nwl; i += WG) {
      const int c = i / nwl, j = i - c * nwl;
      m0[(int64_t)c * W + wb + j] = sm.u.f.w[i];
    }
    __syncthreads();
  }
}

// 64 x 64 bit transpose across a wave (all 64 lanes take part): on entry lane r
// holds row r (bit c = column c), on exit lane c holds column c (bit r = row r).
// Stage s trades with lane r ^ s and swaps the off-diagonal s x s blocks.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, int lane) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int s = 32 >> k;
    const uint64_t m = k == 0 ? 0x00000000FFFFFFFFull
                     : k == 1 ? 0x0000FFFF0000FFFFull
                     : k == 2 ? 0x00FF00FF00FF00FFull
                     : k == 3 ? 0x0F0F0F0F0F0F0F0Full
                     : k == 4 ? 0x3333333333333333ull
                              : 0x5555555555555555ull;
    const uint32_t ylo = __shfl_xor((unsigned)(uint32_t)x, s);
    const uint32_t yhi = __shfl_xor((unsigned)(uint32_t)(x >> 32), s);
    const uint64_t y = ((uint64_t)yhi << 32) | ylo;
    x = (lane & s) ? ((x & ~m) | ((y & ~m) >> s)) : ((x & m) | ((y & m) << s));
  }
  return x;
}

// Integer input with exactly NC (16, 32 or 64) channels.  A wave takes 64
// columns, i.e. one mask word of every channel: lane c reads channel c's word
// and a bit transpose gives every lane its column's channel mask.  The lane
// loads its column straight from global memory (each 2-byte load instruction
// reads 128 contiguous bytes across the wave) and keeps inclusive prefix sums
// Q[i] of the packed words, as the time rows do, with every window inside the
// lane: Q[i + I - 1] - Q[i - 1].  Newly flagged channels are removed from the
// prefixes in registers; the new flags go back through the transpose, one
// store per channel word.
template <int NC>
__device__ __forceinline__ void col_drop(uint32_t (&Q)[NC], uint64_t drop) {
  const uint32_t klo = ~(uint32_t)drop, khi = ~(uint32_t)(drop >> 32);
#pragma unroll
  for (int i = NC - 1; i > 0; --i) Q[i] -= Q[i - 1];
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    acc += __umul24(bit01((i < 32 ? klo : khi), i & 31), Q[i]);
    Q[i] = acc;
  }
}

template <int NC>
__device__ __forceinline__ uint32_t col_win(const uint32_t (&Q)[NC], int i, int I) {
  const uint32_t hi = Q[(i + I - 1 < NC) ? i + I - 1 : 0];
  return i == 0 ? hi : hi - Q[(i > 0) ? i - 1 : 0];
}

template <int NC, int K, class SM>
__device__ __forceinline__ void col_level_px(uint32_t (&Q)[NC], uint64_t& fm, uint64_t& pend, const bool ok,
                                             const SM& sm) {
  constexpr int I = 1 << K;
  if constexpr (I <= NC) {
    if (__ballot(pend != 0) != 0) col_drop<NC>(Q, pend);
    pend = 0;
    const int32_t* Gk = sm.G[K];
    constexpr int NWIN = NC - I + 1;   // full windows of the column
    uint32_t lo = 0, hi = 0;
    // (one path for every wave: a second, scalar-threshold branch over the same
    // window differences makes the compiler compute them all ahead of the branch)
#pragma unroll
    for (int i0 = ((NWIN - 1) / PXB) * PXB; i0 >= 0; i0 -= PXB) {
      uint32_t d[PXB];
      int32_t g[PXB];
#pragma unroll
      for (int j = 0; j < PXB; ++j) {
        if (i0 + j < NWIN) {
          d[j] = col_win<NC>(Q, i0 + j, I);
          g[j] = Gk[(d[j] >> 2) & 63u];
        }
      }
#pragma unroll
      for (int j = PXB - 1; j >= 0; --j) {
        if (i0 + j < NWIN) {
          if (i0 + j >= 32) hi = push_bit(hi, g[j], d[j]); else lo = push_bit(lo, g[j], d[j]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    uint64_t wf = (uint64_t)lo | ((uint64_t)hi << 32);
    if (!ok) wf = 0;
    if (__ballot(wf != 0) == 0) return;
    uint64_t nb = wf;
#pragma unroll
    for (int d = 1; d < I; d <<= 1) nb |= nb << d;
    nb &= lowmask(NC);
    pend = nb & ~fm;
    fm |= nb;
  }
}

template <int NC, class SM>
__device__ __forceinline__ void phase_freq_col(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T;
  const int W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int nlev = min(P.nl_f, ST_MAX_LEVELS);
  const int word = chunk * NW + wv;   // this wave's 64 columns (wave-uniform)
  if (word >= W) return;
  const int t = word * 64 + lane;
  const bool ok = t < T;
  const uint64_t rw = lane < NC ? ld_mask(m0 + (int64_t)lane * W + word) : 0ull;
  uint64_t fm = wave_transpose64(rw, lane);
  fm = ok ? (fm & lowmask(NC)) : 0ull;
  const uint64_t fm0 = fm;
  const GLB uint16_t* col = gp<const uint16_t>(b.data) + (ok ? t : 0);
  uint32_t Q[NC];
  uint32_t run = 0;
#pragma unroll
  for (int i0 = 0; i0 < NC; i0 += 16) {
    uint32_t w[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) w[j] = col[(int64_t)(i0 + j) * b.dstride];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int i = i0 + j;
      const uint32_t v = (ok && !((fm >> i) & 1ull)) ? ci8_power(w[j]) * 256u + 4u : 0u;
      run += v;
      Q[i] = run;
      asm("" : "+v"(Q[i]));   // opaque: the loaded values need not stay alive
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  uint64_t pend = 0;
#define LOF_CLEVEL(K) \
  if (K < nlev) col_level_px<NC, K>(Q, fm, pend, ok, sm);
  LOF_CLEVEL(1)
  LOF_CLEVEL(2)
  LOF_CLEVEL(3)
  LOF_CLEVEL(4)
  LOF_CLEVEL(5)
  LOF_CLEVEL(6)
#undef LOF_CLEVEL
  const uint64_t nbits = ok ? (fm & ~fm0) : 0ull;
  if (__ballot(nbits != 0) == 0) return;
  const uint64_t rnew = wave_transpose64(nbits, lane);
  if (lane < NC && rnew != 0) m0[(int64_t)lane * W + word] = rw | rnew;
}

template <bool INT, class SM>
__device__ __forceinline__ void phase_freq(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int C = b.C;
  if (C <= 1 || P.nl_f <= 1) return;
  if constexpr (INT) {
    if (C == 64) return phase_freq_col<64>(b, P, sm, chunk);
    if (C == 32) return phase_freq_col<32>(b, P, sm, chunk);
    if (C == 16) return phase_freq_col<16>(b, P, sm, chunk);
  }
  if (C <= 16) phase_freq_l<INT, 16>(b, P, sm, chunk);
  else phase_freq_l<INT, 32>(b, P, sm, chunk);
}

// ===================================================================== phase C: SIR
// Scale-invariant rank operator (Sec. 2.2), linear form: weights num (flagged) /
// num-den (unflagged), W = running sum; y is flagged iff
// max_{b > y} W[b] - min_{a <= y} W[a] >= 0.  Lanes of a group hold consecutive
// positions; segment carries chain long rows.

struct SirSum {
  int tot, mn, mx;   // lane: sum, min of W before each position, max of W after each
};

template <int L>
__device__ __forceinline__ SirSum sir_lane_summary(uint64_t bits, int nval, int num, int den) {
  const uint64_t vm = lowmask(nval);
  const uint64_t fb = bits & vm, ub = ~bits & vm;
  const int nmd = num - den;
  int W = 0, mn = BIG, mx = -BIG;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    mn = min(mn, W);
    W += (int)((fb >> i) & 1ull) * num + (int)((ub >> i) & 1ull) * nmd;
    mx = max(mx, W);
  }
  return SirSum{W, mn, mx};
}

// group scans: base = exclusive sum, pmin = min over earlier lanes of (base+mn),
// smax = max over later lanes of (base+mx)
__device__ __forceinline__ void sir_group_scan(const SirSum s, int lig, int G, int& base, int& pmin, int& smax,
                                               int& gtot, int& gmn, int& gmx) {
  int x = s.tot;
  for (int d = 1; d < G; d <<= 1) {
    const int y = __shfl_up(x, d, G);
    if (lig >= d) x += y;
  }
  base = x - s.tot;
  gtot = __shfl(x, G - 1, G);
  int a = base + s.mn;
  for (int d = 1; d < G; d <<= 1) {
    const int y = __shfl_up(a, d, G);
    if (lig >= d) a = min(a, y);
  }
  gmn = __shfl(a, G - 1, G);
  int pa = __shfl_up(a, 1, G);
  pmin = (lig == 0) ? BIG : pa;
  int c = base + s.mx;
  for (int d = 1; d < G; d <<= 1) {
    const int y = __shfl_down(c, d, G);
    if (lig + d < G) c = max(c, y);
  }
  gmx = __shfl(c, 0, G);
  int nc = __shfl_down(c, 1, G);
  smax = (lig == G - 1) ? -BIG : nc;
}

template <int L>
__device__ __forceinline__ uint64_t sir_lane_apply(uint64_t bits, int nval, int num, int den, int Wstart,
                                                   int pmin_in, int smax_in) {
  const uint64_t vm = lowmask(nval);
  const uint64_t fb = bits & vm, ub = ~bits & vm;
  const int nmd = num - den;
  int PM[L];
  int W = Wstart, pm = pmin_in;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    pm = min(pm, W);
    PM[i] = pm;
    W += (int)((fb >> i) & 1ull) * num + (int)((ub >> i) & 1ull) * nmd;
  }
  int sm = smax_in;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int i = L - 1; i >= 0; --i) {
    sm = max(sm, W);
    const uint32_t h = (sm >= PM[i]) ? 1u : 0u;
    if (i < 32) lo |= h << i; else hi |= h << (i - 32);
    W -= (int)((fb >> i) & 1ull) * num + (int)((ub >> i) & 1ull) * nmd;
  }
  return ((uint64_t)lo | ((uint64_t)hi << 32)) & vm;
}

// SIR on one lane's sequence of n <= 64 positions (bit i = position i flagged),
// run by run.  With weights a = num (flagged) and -c = num - den (unflagged), a
// maximal stretch [s, e) of unflagged positions has alpha, the best sum (>= 0)
// of an interval ending at s - 1, and beta, the best sum (>= 0) of an interval
// starting at e; its position s + j is flagged iff some interval through it sums
// to >= 0, i.e. iff j < floor(alpha/c), or j >= len - floor(beta/c), or
// alpha + beta >= len*c.  alpha and beta follow the runs: m flagged positions add
// m*a, a stretch of len positions takes x to max(0, x - len*c).  alpha0 / beta0
// are the best sums of intervals ending just before position 0 and starting just
// after position n - 1 (0 for a whole sequence).  64 positions hold at most 32
// stretches; each is kept in one word: start | len << 6 | min(alpha, len*c) << 13
// (alpha >= len*c already flags the whole stretch; c <= 1024, so 17 bits).
constexpr int SIR_RUNS = 32;
// trailing one bits of x (64 when all are set; ctz of 0 is not defined)
__device__ __forceinline__ int trailing_ones(uint64_t x) { return x == ~0ull ? 64 : __builtin_ctzll(~x); }

__device__ __forceinline__ uint64_t sir_runs_lane(uint64_t bits, int n, int a, int c, const FastDiv& fc,
                                                  int alpha0 = 0, int beta0 = 0) {
  const uint64_t vm = lowmask(n);
  bits &= vm;
  const uint64_t z = ~bits & vm;
  uint64_t out = bits;
  uint32_t st[SIR_RUNS];
  int K = 0, alpha = alpha0, pos = 0;
  // no gaps, or nothing flagged anywhere near: nothing to add
  bool more = z != 0 && (bits != 0 || alpha0 > 0 || beta0 > 0);
  int kw = SIR_RUNS;   // stretches seen by the wave (uniform): the backward pass skips the rest
#pragma unroll
  for (int k = 0; k < SIR_RUNS; ++k) {
    if (__ballot(more) == 0) {
      kw = k;
      break;
    }
    if (more) {
      const uint64_t rest = z >> pos;
      if (rest == 0) {
        more = false;
      } else {
        const int m = __builtin_ctzll(rest);
        alpha += m * a;
        pos += m;
        const int len = min(n - pos, trailing_ones(z >> pos));
        st[k] = (uint32_t)pos | ((uint32_t)len << 6) | ((uint32_t)min(alpha, len * c) << 13);
        const int P = min(len, (int)fc.div((uint32_t)alpha));
        out |= lowmask(P) << pos;
        alpha = max(0, alpha - len * c);
        pos += len;
        K = k + 1;
        if (pos >= n) more = false;
      }
    }
  }
  int beta = beta0, nxt = n;
#pragma unroll
  for (int k = SIR_RUNS - 1; k >= 0; --k) {
    if (k >= kw) continue;
    if (k < K) {
      const int s0 = (int)(st[k] & 63u), len = (int)((st[k] >> 6) & 127u), al = (int)(st[k] >> 13);
      const int e = s0 + len;
      beta += (nxt - e) * a;
      const int Q = min(len, (int)fc.div((uint32_t)beta));
      out |= lowmask(Q) << (e - Q);
      if (al + beta >= len * c) out |= lowmask(len) << s0;
      beta = max(0, beta - len * c);
      nxt = s0;
    }
  }
  return out;
}

// A lane's effect on the best interval sums crossing it: an incoming alpha (best
// sum of an interval ending just before the lane) leaves as max(Pf, alpha + Q),
// an incoming beta (best sum starting just after it) as max(Pb, beta + Q), with
// Q the lane's total weight, Pf its best suffix sum and Pb its best prefix sum
// (both >= 0).  With W the running weight sum (W = 0 before the lane), Q is W at
// the end, Pf = Q - min W and Pb = max W; the extremes are at run boundaries.
__device__ __forceinline__ void sir_lane_maps(uint64_t bits, int n, int a, int c, int& Pf, int& Pb, int& Q) {
  const uint64_t vm = lowmask(n);
  const uint64_t z = ~bits & vm;
  int W = 0, wmin = 0, wmax = 0, pos = 0;
  while (pos < n) {
    const uint64_t rest = z >> pos;
    const int m = rest == 0 ? n - pos : min(n - pos, __builtin_ctzll(rest));   // flagged run
    W += m * a;
    wmax = max(wmax, W);
    pos += m;
    if (pos >= n) break;
    const int len = min(n - pos, trailing_ones(z >> pos));                   // unflagged stretch (>= 1)
    W -= len * c;
    wmin = min(wmin, W);
    pos += len;
  }
  Q = W;
  Pf = W - wmin;
  Pb = wmax;
}

// Exclusive scans of the lane maps along a group of G lanes: alpha_in from the
// lanes before (composition in lane order), beta_in from the lanes after.
__device__ __forceinline__ void sir_map_scans(int Pf, int Pb, int Q, int lig, int G, int& alpha_in, int& beta_in) {
  // forward: composed map of lanes [0, lig] as (P, Q); apply to 0 -> P
  int P = Pf, S = Q;
  for (int d = 1; d < G; d <<= 1) {
    const int Pp = __shfl_up(P, d, G), Sp = __shfl_up(S, d, G);
    if (lig >= d) {
      P = max(P, Pp + S);
      S = Sp + S;
    }
  }
  const int Pe = __shfl_up(P, 1, G);
  alpha_in = lig == 0 ? 0 : max(0, Pe);
  // backward: composed map of lanes [lig, G) in reverse order
  P = Pb;
  S = Q;
  for (int d = 1; d < G; d <<= 1) {
    const int Pn = __shfl_down(P, d, G), Sn = __shfl_down(S, d, G);
    if (lig + d < G) {
      P = max(P, Pn + S);
      S = Sn + S;
    }
  }
  const int Pn = __shfl_down(P, 1, G);
  beta_in = lig == G - 1 ? 0 : max(0, Pn);
}

template <int L, class SM>
__device__ __forceinline__ void phase_sir_time(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, C = b.C;
  const int W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int num = P.eta_num, den = P.eta_den;
  if (T <= 64 * L) {
    int G = 1;
    while (G * L < T) G <<= 1;
    const int R = 64 / G, lig = lane & (G - 1), grp = lane / G;
    const int rb = chunk * NW * R + wv * R;   // this wave's R rows of the chunk
    if (rb < C) {
      const int row = rb + grp;
      const bool ok = row < C;
      GLB uint64_t* rp = m0 + (int64_t)(ok ? row : 0) * W;
      const int nval = ok ? clampi(T - lig * L, 0, L) : 0;
      const uint64_t bits = ok ? (get_bits(rp, W, lig * L, L) & lowmask(nval)) : 0ull;
      const bool any = __ballot(bits != 0) != 0;
      if (num >= den) {   // eta = 1: every interval qualifies
        write_row_bits<L>(rp, W, lowmask(nval), lig, G, ok);
      } else if (any) {   // nothing flagged and eta < 1: nothing to add
        // run by run, with the best interval sums entering from the
        // neighbouring lanes of the row
        const int a = num, c = den - num;
        int Pf, Pb, Q, ain, bin;
        sir_lane_maps(bits, nval, a, c, Pf, Pb, Q);
        sir_map_scans(Pf, Pb, Q, lig, G, ain, bin);
        const FastDiv fc((uint32_t)c);
        const uint64_t out = sir_runs_lane(bits, nval, a, c, fc, ain, bin);
        write_row_bits<L>(rp, W, out, lig, G, ok);
      }
    }
  } else if constexpr (L == 64) {
    // long rows (only laid out with L == 64): SIR_SEG positions per segment, two
    // passes with carries
    const int nseg = (T + SIR_SEG - 1) / SIR_SEG;
    int(*seg)[3] = sm.u.c.seg[wv];
    for (int row = chunk * NW + wv; row < C && row < (chunk + 1) * NW; row += NW) {
      GLB uint64_t* rp = m0 + (int64_t)row * W;
      bool any = false;
      for (int s = 0; s < nseg; ++s) {
        const int q = s * SIR_SEG + lane * L;
        const int nval = clampi(T - q, 0, L);
        const uint64_t bits = get_bits(rp, W, q, L) & lowmask(nval);
        any = any || (__ballot(bits != 0) != 0);
        const SirSum ss = sir_lane_summary<L>(bits, nval, num, den);
        int base, pmin, smax, gt, gn, gx;
        sir_group_scan(ss, lane, 64, base, pmin, smax, gt, gn, gx);
        if (lane == 0) {
          seg[s][0] = gt;
          seg[s][1] = gn;
          seg[s][2] = gx;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (!any && num < den) continue;
      // carries: lane s <-> segment s
      SirSum cs{0, BIG, -BIG};
      if (lane < nseg) cs = SirSum{seg[lane][0], seg[lane][1], seg[lane][2]};
      int base, pmin, smax, gt, gn, gx;
      sir_group_scan(cs, lane, 64, base, pmin, smax, gt, gn, gx);
      __builtin_amdgcn_wave_barrier();
      if (lane < nseg) {
        seg[lane][0] = base;
        seg[lane][1] = pmin;
        seg[lane][2] = smax;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int s = 0; s < nseg; ++s) {
        const int q = s * SIR_SEG + lane * L;
        const int nval = clampi(T - q, 0, L);
        const uint64_t bits = get_bits(rp, W, q, L) & lowmask(nval);
        const SirSum ss = sir_lane_summary<L>(bits, nval, num, den);
        int lb, lp, lx, a1, a2, a3;
        sir_group_scan(ss, lane, 64, lb, lp, lx, a1, a2, a3);
        const int sb = seg[s][0], sp = seg[s][1], sx = seg[s][2];
        const int pmin_in = min(sp, lp == BIG ? BIG : sb + lp);
        const int smax_in = max(sx, lx == -BIG ? -BIG : sb + lx);
        const uint64_t out = sir_lane_apply<L>(bits, nval, num, den, sb + lb, pmin_in, smax_in);
        // segments are word aligned: every lane owns one word (L == 64)
        if (nval > 0) rp[q >> 6] = out;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <int LF, class SM>
__device__ __forceinline__ void phase_sir_freq_l(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, C = b.C;
  const int W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int num = P.eta_num, den = P.eta_den;
  const FreqShape fs(C, lane);
  const int span = max(fs.cpi, 64);
  for (int it0 = chunk * span; it0 < T && it0 < (chunk + 1) * span; it0 += fs.cpi) {
    const int ncols = min(fs.cpi, T - it0);
    const int wb = it0 >> 6;
    const int nwl = ((it0 + ncols - 1) >> 6) - wb + 1;
    stage_slab<true, false>(b, sm, m0, W, it0, ncols, wb, nwl, fs.stride);
    __syncthreads();
    const int col = wv * fs.cpw + fs.colw;
    const int t = it0 + col;
    const bool ok = col < ncols;
    const int tt = ok ? t : it0;
    const int wsel = (tt >> 6) - wb, bsel = tt & 63;
    uint64_t bits = 0;
#pragma unroll
    for (int i = 0; i < LF; ++i)
      if (i < fs.nval) bits |= ((sm.u.f.w[(fs.ch0 + i) * nwl + wsel] >> bsel) & 1ull) << i;
    if (!ok) bits = 0;
    const bool work = (__ballot(bits != 0) != 0) || num >= den;
    if (work) {
      const int nv = ok ? fs.nval : 0;
      const SirSum s = sir_lane_summary<LF>(bits, nv, num, den);
      int base = 0, pmin = BIG, smax = -BIG, gt, gn, gx;
      if (fs.G > 1) sir_group_scan(s, fs.lig, fs.G, base, pmin, smax, gt, gn, gx);
      const uint64_t out = sir_lane_apply<LF>(bits, nv, num, den, base, pmin, smax);
      uint64_t nb = out & ~bits;
      while (nb) {
        const int i = __builtin_ctzll(nb);
        nb &= nb - 1;
        or_bit_lds(sm.u.f.w, (fs.ch0 + i) * nwl + wsel, bsel);
      }
    }
    __syncthreads();
    for (int i = tid; i < C * nwl; i += WG) {
      const int c = i / nwl, j = i - c * nwl;
      m0[(int64_t)c * W + wb + j] = sm.u.f.w[i];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- prose reading
// The range-extension reading of Sec. 2.2: every maximal range of consecutive
// flagged positions, of length L, gains floor(eta L) positions before and after
// it; the extensions of all ranges of the input mask are OR-ed.  A forward scan
// carries `reach`, the end of the furthest right extension of the ranges that
// have ended, and covers every position below it; a backward scan carries the
// start of the furthest left extension of the ranges that have begun.  The
// forward result goes to the second mask buffer, the backward scan reads the
// input mask and that buffer and writes the result over the input mask.
struct ProseScan {
  uint32_t run;   // length of the flagged range the scan is in
  int reach;
};

// forward step over one word of positions pos0 .. pos0+nb-1 (bit i <-> pos0+i)
__device__ __forceinline__ uint64_t prose_fwd_word(uint64_t x, int pos0, int nb, ProseScan& sc, uint32_t num,
                                                   const FastDiv& fd) {
  if (x == 0 && sc.run == 0) {
    const int c = clampi(sc.reach - pos0, 0, nb);
    return lowmask(c);
  }
  if (x == lowmask(nb)) {
    sc.run += (uint32_t)nb;
    return x;
  }
  uint64_t out = x;
  for (int i = 0; i < nb; ++i) {
    if ((x >> i) & 1ull) {
      ++sc.run;
    } else {
      if (sc.run) {
        sc.reach = max(sc.reach, pos0 + i + (int)fd.div(num * sc.run));
        sc.run = 0;
      }
      if (pos0 + i < sc.reach) out |= 1ull << i;
    }
  }
  return out;
}

// backward step: positions pos0+nb-1 down to pos0; sc.reach starts at the length
__device__ __forceinline__ uint64_t prose_bwd_word(uint64_t x, int pos0, int nb, ProseScan& sc, uint32_t num,
                                                   const FastDiv& fd) {
  if (x == 0 && sc.run == 0) {
    const int c = clampi(sc.reach - pos0, 0, nb);   // positions >= reach are covered
    return lowmask(nb) & ~lowmask(c);
  }
  if (x == lowmask(nb)) {
    sc.run += (uint32_t)nb;
    return 0;
  }
  uint64_t out = 0;
  for (int i = nb - 1; i >= 0; --i) {
    if ((x >> i) & 1ull) {
      ++sc.run;
    } else {
      if (sc.run) {
        sc.reach = min(sc.reach, pos0 + i + 1 - (int)fd.div(num * sc.run));
        sc.run = 0;
      }
      if (pos0 + i >= sc.reach) out |= 1ull << i;
    }
  }
  return out;
}

// rows: lane = row, 64 rows a wave, words walked in order
__device__ __forceinline__ void phase_prose_time(const DevBlock& b, const DevParams& P, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, W = (T + 63) >> 6;
  const int row = (chunk * NW + wv) * 64 + lane;
  if (row >= b.C || P.eta_num == 0) return;
  GLB uint64_t* mrow = gp<uint64_t>(P.maskw) + b.mask_off + (int64_t)row * W;
  GLB uint64_t* brow = gp<uint64_t>(P.maskw2) + b.mask_off + (int64_t)row * W;
  const FastDiv fd((uint32_t)P.eta_den);
  const uint32_t num = (uint32_t)P.eta_num;
  ProseScan f{0u, 0};
  for (int w = 0; w < W; ++w) {
    const int nb = min(64, T - 64 * w);
    brow[w] = prose_fwd_word(mrow[w] & lowmask(nb), 64 * w, nb, f, num, fd);
  }
  ProseScan r{0u, T};
  for (int w = W - 1; w >= 0; --w) {
    const int nb = min(64, T - 64 * w);
    const uint64_t x = mrow[w] & lowmask(nb);
    mrow[w] = brow[w] | prose_bwd_word(x, 64 * w, nb, r, num, fd);
  }
}

// columns: lane = column of one 64-column word (wave-uniform), channels walked
// in order, each channel's word of the result assembled by a ballot
__device__ __forceinline__ void phase_prose_freq(const DevBlock& b, const DevParams& P, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, C = b.C, W = (T + 63) >> 6;
  const int wi = chunk * NW + wv;
  if (wi >= W || C <= 1 || P.eta_num == 0) return;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off + wi;
  GLB uint64_t* b0 = gp<uint64_t>(P.maskw2) + b.mask_off + wi;
  const bool ok = wi * 64 + lane < T;
  const FastDiv fd((uint32_t)P.eta_den);
  const uint32_t num = (uint32_t)P.eta_num;
  ProseScan f{0u, 0};
  for (int c = 0; c < C; ++c) {
    const uint64_t x = m0[(int64_t)c * W];
    const uint64_t o = prose_fwd_word(ok ? ((x >> lane) & 1ull) : 0ull, c, 1, f, num, fd);
    const uint64_t word = __ballot(o != 0);
    if (lane == 0) b0[(int64_t)c * W] = word;
  }
  ProseScan r{0u, C};
  for (int c = C - 1; c >= 0; --c) {
    const uint64_t x = m0[(int64_t)c * W];
    const uint64_t o = prose_bwd_word(ok ? ((x >> lane) & 1ull) : 0ull, c, 1, r, num, fd);
    const uint64_t word = __ballot(o != 0);
    if (lane == 0) m0[(int64_t)c * W] = b0[(int64_t)c * W] | word;
  }
}

// flag bytes of one row word: nv (<= 64) samples from t0, bit j -> byte j
// four flag bits -> four 0/1 bytes: bit k of nib times 2^(7k) lands at bit 8k
// (the shifted copies of a 4-bit value do not overlap, so nothing carries)
__device__ __forceinline__ uint32_t nibble_bytes(uint32_t nib) { return (nib * 0x00204081u) & 0x01010101u; }

__device__ __forceinline__ void write_word_bytes(const DevBlock& b, int row, int t0, int nv, uint64_t w) {
  GLB uint8_t* fp = gp<uint8_t>(b.flags) + (int64_t)row * b.fstride + t0;
  if (b.faligned && nv == 64) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t h = (uint32_t)(w >> (16 * q)) & 0xffffu;
      uint32_t o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t nib = (h >> (4 * j)) & 0xfu;
        o[j] = nibble_bytes(nib);
      }
      *(GLB u32x4*)(fp + 16 * q) = u32x4{o[0], o[1], o[2], o[3]};
    }
  } else {
    for (int j = 0; j < nv; ++j) fp[j] = (uint8_t)((w >> j) & 1ull);
  }
}

// Up to 64 channels: a wave takes 64 columns (one mask word per channel), the
// transpose gives each lane its whole column, SIR runs in the lane, and the new
// flags go back through the transpose.  This is the last pass over the mask, so
// it also writes the flag bytes of its 64 columns (the history pass rewrites
// only rows it flags) and counts the flagged samples.
__host__ __device__ inline bool sirf_writes_bytes(int eta_num, int prose, int C) {
  return eta_num > 0 && !prose && C > 1 && C <= 64;
}

__device__ __forceinline__ void phase_sir_freq_col(const DevBlock& b, const DevParams& P, const int chunk) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int T = b.T, C = b.C;
  const int W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int num = P.eta_num, den = P.eta_den;
  const int word = chunk * NW + wv;   // wave-uniform
  if (word >= W || num == 0) return;
  const int t = word * 64 + lane;
  const bool ok = t < T;
  const int nv = min(64, T - word * 64);
  const uint64_t rw = lane < C ? ld_mask(m0 + (int64_t)lane * W + word) : 0ull;
  uint64_t rnew = 0;
  uint64_t bits = wave_transpose64(rw, lane);
  bits = ok ? (bits & lowmask(C)) : 0ull;
  if (__ballot(bits != 0) != 0) {
    uint64_t out = bits;
    if (num >= den) {
      out = ok ? lowmask(C) : 0ull;   // eta = 1: every interval qualifies
    } else {
      const FastDiv fc((uint32_t)(den - num));
      out = sir_runs_lane(bits, C, num, den - num, fc);
    }
    const uint64_t nb = ok ? (out & ~bits) : 0ull;
    if (__ballot(nb != 0) != 0) {
      rnew = wave_transpose64(nb, lane);
      if (lane < C && rnew != 0) m0[(int64_t)lane * W + word] = rw | rnew;
    }
  }
  const uint64_t fw = (rw | rnew) & lowmask(nv);
  if (lane < C) write_word_bytes(b, lane, word * 64, nv, fw);
  if (P.stats) {
    unsigned long long nfl = lane < C ? (unsigned long long)__popcll(fw) : 0ull;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nfl += __shfl_xor(nfl, d);
    char* st = (char*)P.stats + (int64_t)b.out_idx * STATS_BYTES;
    if (lane == 0 && nfl) atomicAdd((unsigned long long*)(st + STATS_NFLAG), nfl);
  }
}

template <class SM>
__device__ __forceinline__ void phase_sir_freq(const DevBlock& b, const DevParams& P, SM& sm, const int chunk) {
  const int C = b.C;
  if (C <= 1) return;
  if (sirf_colpath(C)) return phase_sir_freq_col(b, P, chunk);
  phase_sir_freq_l<32>(b, P, sm, chunk);
}

// ===================================================================== phase D
// History flagger (Sec. 4.1) on the rows [r0, r1) of a block: per channel, the
// mean of this block's unflagged samples against mean + history_sensitivity *
// stddev of the committed means.  One wave per row; the ring's state does not
// depend on this block, so its loads are issued first and overlap the loads of
// the row's mask and samples.
// mrow: the row's mask words (global memory or LDS)
template <bool INT, class MP>
__device__ __forceinline__ void row_unflagged(const DevBlock& b, MP mrow, int row, int lane, uint64_t rowsum,
                                              double& usum, int& cnt) {
  const int T = b.T;
  const int W = (T + 63) >> 6;
  if constexpr (INT) {
    // the row's power sum (exact, from the time pass) minus the flagged
    // samples' power: input is read only for mask words with flags
    const GLB uint8_t* rbase = gp<const uint8_t>(b.data) + (int64_t)row * b.dstride * 2;
    uint32_t sf = 0;   // < 64 words * 64 * 32768 = 2^27 per lane
    int nf = 0;
    for (int wi = lane; wi < W; wi += 64) {
      const int t0 = wi * 64;
      const int nv = min(64, T - t0);
      const uint64_t fw = mrow[wi] & lowmask(nv);
      nf += __popcll(fw);
      if (fw == 0) continue;
      const GLB uint8_t* rb = rbase + (int64_t)t0 * 2;
      if (b.aligned && nv == 64) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const u32x4 q = *(const GLB u32x4*)(rb + 16 * j);
          const uint32_t a4[4] = {q.x, q.y, q.z, q.w};
          const int f8 = (int)(uint32_t)(fw >> (8 * j));
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            // the word's two samples kept by their flag bits (sign-extended bit
            // fields), then re^2 + im^2 of the kept ones in one int8 dot product
            const uint32_t lo = (uint32_t)__builtin_amdgcn_sbfe(f8, 2 * m, 1);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_sbfe(f8, 2 * m + 1, 1);
            const uint32_t keep = (lo & 0xffffu) | (hi & 0xffff0000u);
            sf = (uint32_t)__builtin_amdgcn_sdot4((int)(a4[m] & keep), (int)a4[m], (int)sf, false);
          }
        }
      } else {
        uint64_t bits = fw;
        while (bits) {
          const int i = __builtin_ctzll(bits);
          bits &= bits - 1;
          sf += ci8_power(*(const GLB uint16_t*)(rb + 2 * i));
        }
      }
    }
    unsigned long long sfl = sf;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      sfl += __shfl_xor(sfl, d);
      nf += __shfl_xor(nf, d);
    }
    usum = (double)(rowsum - sfl);   // integer sums < 2^53: exact
    cnt = T - nf;
  } else {
    const int nch = (T + 7) >> 3;
    double sd = 0.0;
    int c = 0;
    const bool fast = b.aligned && (T & 7) == 0;
    for (int ci = lane; ci < nch; ci += 64) {
      const int t0 = ci * 8;
      const uint32_t fb = (uint32_t)(mrow[t0 >> 6] >> (t0 & 63)) & 0xffu;
      float v[8];
      int nv = 8;
      if (fast) load8v<false>(b, row, t0, v);
      else nv = load8<false>(b, row, t0, v);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j < nv && !((fb >> j) & 1u)) {
          sd += (double)v[j];
          ++c;
        }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      sd += __shfl_xor(sd, d);
      c += __shfl_xor(c, d);
    }
    usum = sd;
    cnt = c;
  }
}

// The history decision of one row (one wave): the row's current mean (usum /
// cnt over its unflagged samples) against mean + history_sensitivity * stddev of
// the committed ring (L entries, head = next write slot; lane j holds ring slot
// j in xs when the ring fits one wave), sums in ring order as the sequential
// definition has them; stages the pushed value and sets the row's bit in
// rowflag (LDS) when it flags.
__device__ __forceinline__ void history_judge(const DevParams& P, int64_t idx, int L, int head,
                                              const GLB double* ring, double xs, bool small_ring, double usum,
                                              int cnt, int lane, uint32_t* rowflag, int row) {
  const bool judge = L >= P.Hmin;
  // the first 64 entries in ring order, oldest first (lane j holds entry j)
  int k0 = head - L + lane;
  if (k0 < 0) k0 += P.H;
  const int ks = (lane < L) ? k0 : 0;
  const double xr = small_ring ? __shfl(xs, ks) : ((judge && lane < L) ? ring[k0] : 0.0);
  const double x0 = (judge && lane < L) ? xr : 0.0;
  if (cnt == 0) {
    if (lane == 0) gp<uint8_t>(P.pvalid)[idx] = 0;
    return;
  }
  const double cur = usum / (double)cnt;
  bool flag = false;
  double pushv = cur;
  if (judge) {
    // winsorized history (rings of at most 64): the values of rank k and L-1-k
    // (ties by ring order) bound every committed mean
    double xw = x0;
    if (P.winsor > 0 && L > 0) {
      const int k = min(P.winsor, (L - 1) / 2);
      int rank = 0;
      for (int q = 0; q < L; ++q) {
        const double y = lane_double(x0, q);
        rank += (y < x0 || (y == x0 && q < lane)) ? 1 : 0;
      }
      const uint64_t blo = __ballot(lane < L && rank == k);
      const uint64_t bhi = __ballot(lane < L && rank == L - 1 - k);
      const double lo = lane_double(x0, __ffsll((unsigned long long)blo) - 1);
      const double hi = lane_double(x0, __ffsll((unsigned long long)bhi) - 1);
      if (lane < L) xw = x0 < lo ? lo : (x0 > hi ? hi : x0);
    }
    double acc = 0.0;
    for (int j0 = 0; j0 < L; j0 += 64) {
      double x = xw;
      if (j0 > 0) {
        int k = head - L + j0 + lane;
        if (k < 0) k += P.H;
        x = j0 + lane < L ? ring[k] : 0.0;
      }
      const int m = min(64, L - j0);
      for (int q = 0; q < m; ++q) acc += lane_double(x, q);
    }
    const double hm = acc / (double)L;
    acc = 0.0;
    for (int j0 = 0; j0 < L; j0 += 64) {
      double x = xw;
      if (j0 > 0) {
        int k = head - L + j0 + lane;
        if (k < 0) k += P.H;
        x = j0 + lane < L ? ring[k] : 0.0;
      }
      const int m = min(64, L - j0);
      for (int q = 0; q < m; ++q) {
        const double d = lane_double(x, q) - hm;
        acc += d * d;
      }
    }
    const double hv = acc / (double)L;
    const double thr = hm + P.hs * __builtin_sqrt(hv);
    flag = P.literal ? (cur >= thr) : (cur > thr);
    if (flag) pushv = thr;
  }
  if (lane == 0) {
    gp<double>(P.pend)[idx] = pushv;
    gp<uint8_t>(P.pvalid)[idx] = 1;
    if (flag) atomicOr(&rowflag[row >> 5], 1u << (row & 31));
  }
}

template <bool INT, class SM>
__device__ __forceinline__ void phase_history(const DevBlock& b, const DevParams& P, SM& sm, const int r0,
                                              const int r1) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < MAXC / 32; i += WG) sm.rowflag[i] = 0u;
  __syncthreads();
  const int s = b.stream_id;
  const int row = r0 + wv;   // one row per wave (a chunk is NW rows)
  if (s >= 0 && row < r1) {
    const int64_t idx = (int64_t)s * P.maxC + row;
    // every load that does not depend on another is issued first: count, head,
    // the ring in storage order (lane j reads slot j) and the row's power sum
    const int L = gp<const int32_t>(P.rcount)[idx];
    const int head = gp<const int32_t>(P.rhead)[idx];
    const GLB double* ring = gp<const double>(P.ring) + idx * P.H;
    const bool small_ring = P.H <= 64;
    const double xs = (small_ring && lane < P.H) ? ring[lane] : 0.0;
    const uint64_t rowsum = INT ? gp<const uint64_t>(P.rowsum)[(int64_t)b.sidx * P.maxC + row] : 0ull;
    const int W = (b.T + 63) >> 6;
    const GLB uint64_t* mrow = gp<uint64_t>(P.maskw) + b.mask_off + (int64_t)row * W;
    double usum;
    int cnt;
    row_unflagged<INT>(b, mrow, row, lane, rowsum, usum, cnt);
    history_judge(P, idx, L, head, ring, xs, small_ring, usum, cnt, lane, sm.rowflag, row);
  }
  __syncthreads();
}

// final flags of the rows [r0, r1) = SIR mask OR history rows; one byte per
// sample.  The block's flagged-sample and history-row totals are accumulated in
// the caller's stats entry (zeroed by the statistics kernel).
// With bytes_done the SIR pass already wrote and counted the SIR flags: only
// rows the history flags are rewritten (all ones) and their extra flags counted.
template <class SM>
__device__ __forceinline__ void phase_write(const DevBlock& b, const DevParams& P, SM& sm, const int r0, const int r1,
                                            const bool bytes_done) {
  const int tid = thread_id(), lane = tid & 63;
  const int T = b.T;
  const int W = (T + 63) >> 6;
  const GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  const int nch = (T + 15) >> 4;
  const uint32_t items = (uint32_t)(r1 - r0) * (uint32_t)nch;
  const FastDiv fd((uint32_t)nch);
  unsigned long long nfl = 0;
  for (uint32_t it = tid; it < items; it += WG) {
    const int rr = (int)fd.div(it);
    const int row = r0 + rr;
    const int t0 = (int)(it - (uint32_t)rr * (uint32_t)nch) * 16;
    const bool hrow = (sm.rowflag[row >> 5] >> (row & 31)) & 1u;
    if (bytes_done && !hrow) continue;
    const uint64_t w = ld_mask(m0 + (int64_t)row * W + (t0 >> 6));
    uint32_t fb = (uint32_t)(w >> (t0 & 63)) & 0xffffu;
    const int nv = min(16, T - t0);
    const uint32_t vm16 = (nv >= 16) ? 0xffffu : ((1u << nv) - 1u);
    fb &= vm16;
    if (hrow) {
      nfl += (unsigned long long)__builtin_popcount(vm16 & ~fb);   // added by the history flag
      if (!bytes_done) nfl += (unsigned long long)__builtin_popcount(fb);
      fb = vm16;
    } else {
      nfl += (unsigned long long)__builtin_popcount(fb);
    }
    GLB uint8_t* fp = gp<uint8_t>(b.flags) + (int64_t)row * b.fstride + t0;
    if (b.faligned && nv == 16) {
      uint32_t o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t nib = (fb >> (4 * j)) & 0xfu;
        o[j] = nibble_bytes(nib);
      }
      *(GLB u32x4*)fp = u32x4{o[0], o[1], o[2], o[3]};
    } else {
      for (int j = 0; j < nv; ++j) fp[j] = (uint8_t)((fb >> j) & 1u);
    }
  }
  if (!P.stats) return;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) nfl += __shfl_xor(nfl, d);
  char* st = (char*)P.stats + (int64_t)b.out_idx * STATS_BYTES;
  if (lane == 0 && nfl) atomicAdd((unsigned long long*)(st + STATS_NFLAG), nfl);
  if (tid == 0) {
    int hr = 0;
    for (int row = r0; row < r1; ++row) hr += (sm.rowflag[row >> 5] >> (row & 31)) & 1u;
    if (hr) atomicAdd((int*)(st + STATS_HROWS), hr);
  }
}

// ===================================================================== kernels
// One kernel per phase; a phase's mask stores reach the next kernel through the
// kernel boundary on the same stream.
#ifndef LOF_WAVES_PER_EU
#define LOF_WAVES_PER_EU 4
#endif
// Float SumThreshold keeps sums and counts per position (twice the registers of
// the packed integer form): 2 waves per SIMD, 256 VGPRs, no spills.  The float
// frequency slab (81 KB of LDS) allows one workgroup per CU anyway.
constexpr int float_waves_per_eu = 2;
// The history-and-bytes kernel is a chain of dependent global loads per row
// (ring and row sum, mask words, flagged samples): 8 waves per SIMD hide them.
#ifndef LOF_FINAL_WAVES_PER_EU
#define LOF_FINAL_WAVES_PER_EU 8
#endif
// SIR along time moves little data per work item and waits on dependent global
// loads: more resident waves (6 per SIMD) pay more than the few spills they cost.
#ifndef LOF_SIRT_WAVES_PER_EU
#define LOF_SIRT_WAVES_PER_EU 6
#endif

// A kernel's work items are (block, chunk) pairs, item = block * maxch + chunk;
// chunks past a smaller block's count return at once.  With counter == nullptr
// each workgroup takes one item; otherwise a persistent grid takes the next item
// from a device counter until all are done.
template <class F>
__device__ __forceinline__ void run_items(int nitems, int* counter, F&& f) {
  if (counter == nullptr) {
    // one item per workgroup: a body with no loop around it, so nothing is
    // hoisted and held across items
    if ((int)blockIdx.x < nitems) f((int)blockIdx.x);
    return;
  }
  __shared__ int cur;
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = cur;
    __syncthreads();
    if (it >= nitems) break;
    f(it);
    __syncthreads();
  }
}

// Phase A: power, median, stddev and thresholds of each block -> BlockState and
// the caller's stats entry (whose flag totals the final kernel accumulates).
template <bool INT, bool PRE>
__global__ __launch_bounds__(WG, INT ? LOF_WAVES_PER_EU : 8) void lof_stats_kernel(const DevBlock* __restrict__ blocks, int nb,
                                                                         int* counter, DevParams P) {
  __shared__ SmStats<INT> sm;
  run_items(nb, counter, [&](int bi) __attribute__((always_inline)) {
    const DevBlock b = blocks[bi];
    phase_stats<INT, PRE>(b, P, sm);
    write_block_stats(b, P, sm);
  });
}

// Phase B, time direction: rows of a block in chunks (CX: float rows of complex
// input with the formed powers kept, 32 samples per lane)
template <bool INT, int L, bool CX = false>
__global__ __launch_bounds__(WG, (INT && L == 64) ? 2 : ((INT || (L == 32 && !CX)) ? LOF_WAVES_PER_EU : float_waves_per_eu)) void lof_time_kernel(const DevBlock* __restrict__ blocks, int nb,
                                                                        int maxch, int* counter, DevParams P) {
  __shared__ SmThr sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= time_chunks(b.C, b.T, L)) return;
    load_thresholds<INT>(b, P, sm);
    phase_time<INT, L, CX>(b, P, sm, ch);
  });
}

// Phase B, time direction, from caller-supplied pre-flags
template <bool INT, int L>
__global__ __launch_bounds__(WG, (INT && L == 64) ? 2 : (INT ? LOF_WAVES_PER_EU : float_waves_per_eu)) void lof_time_pre_kernel(
    const DevBlock* __restrict__ blocks, int nb, int maxch, int* counter, DevParams P) {
  __shared__ SmThr sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= time_chunks(b.C, b.T, L)) return;
    load_thresholds<INT>(b, P, sm);
    phase_time_pre<INT, L>(b, P, sm, ch);
  });
}

// Phase B, frequency direction: column slabs of a block
template <bool INT>
__global__ __launch_bounds__(WG, INT ? LOF_WAVES_PER_EU : float_waves_per_eu) void lof_freq_kernel(const DevBlock* __restrict__ blocks, int nb,
                                                                        int maxch, int* counter, DevParams P) {
  __shared__ SmFreq<INT> sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= freq_chunks(INT, b.C, b.T) || b.C <= 1 || P.nl_f <= 1) return;
    load_thresholds<INT>(b, P, sm);
    phase_freq<INT>(b, P, sm, ch);
  });
}

// Phase B along frequency, float blocks of at most 16 channels: the generic slab
// path with a slab of 16 channels, whose smaller LDS and register needs let 4
// waves per SIMD share a CU
template <int LF>
__global__ __launch_bounds__(WG, LOF_WAVES_PER_EU) void lof_freq_small_kernel(const DevBlock* __restrict__ blocks,
                                                                             int nb, int maxch, int* counter,
                                                                             DevParams P) {
  __shared__ SmFreqS sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= freq_chunks(false, b.C, b.T) || b.C <= 1 || b.C > LF || P.nl_f <= 1) return;
    load_thresholds<false>(b, P, sm);
    phase_freq_l<false, LF>(b, P, sm, ch);
  });
}

// Phase C: SIR operator along time (rows in chunks), then along frequency (slabs)
template <int L>
__global__ __launch_bounds__(WG, L == 64 ? 2 : LOF_SIRT_WAVES_PER_EU) void lof_sir_time_kernel(const DevBlock* __restrict__ blocks, int nb,
                                                                            int maxch, int* counter, DevParams P) {
  __shared__ SmSirT sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= time_chunks(b.C, b.T, L)) return;
    phase_sir_time<L>(b, P, sm, ch);
  });
}

// Phase D: history flagger and flag bytes, rows in chunks of NW
template <bool INT>
__global__ __launch_bounds__(WG, LOF_FINAL_WAVES_PER_EU) void lof_final_kernel(const DevBlock* __restrict__ blocks, int nb,
                                                                         int maxch, int* counter, DevParams P) {
  __shared__ SmFinal sm;
  run_items(nb * maxch, counter, [&](int it) __attribute__((always_inline)) {
    const int bi = it / maxch, ch = it - bi * maxch;
    const DevBlock b = blocks[bi];
    if (ch >= final_chunks(b.C)) return;
    const int r0 = ch * NW, r1 = min(b.C, r0 + NW);
    phase_history<INT>(b, P, sm, r0, r1);
    phase_write(b, P, sm, r0, r1, sirf_writes_bytes(P.eta_num, P.prose | P.integrated, b.C));
  });
}

// Commit staged history values (Sec. 4.1 addToHistory) of a list of streams.
struct IdList {
  int32_t n;
  int32_t ids[255];
};

}  // namespace lofk
