// lof_integrated.hpp -- the integrated pre-correlation mode (gfx950).
//
// Sec. 4 (integration paragraph) of van Nieuwpoort, "Towards exascale real-time
// RFI mitigation", arXiv 1701.08197: integrate time fully and flag the spectrum
// along frequency first, then integrate the unflagged channels fully and flag
// the time series along time; a flagged channel flags its row, a flagged time
// its column.  Each series gets its own median, stddev and thresholds (Sec. 2.1),
// one-dimensional SumThreshold and the SIR step (Sec. 2.2).  The history
// flagger and the flag bytes follow in the final kernel, as for full-rate
// flagging.
//
// One workgroup per block.  A single pass over the input builds the spectrum
// (row sums) and the all-channel time series (column sums, each thread owning
// its columns in registers); both stay in LDS.  The flagged channels are then
// taken out of the series (exactly, by subtraction, for integer input; by a
// second sum over the unflagged channels for float input), the series is
// flagged, and the block's mask words are written.  Integer input stays exact:
// sums in 64-bit integers, second moments in 128-bit integers with the
// correctly rounded quotient, window tests against floor(c * T_k).
#pragma once
#include "lof_kernels.hpp"

namespace lofk {

constexpr int INTEG_MAX_T = 16384;         // time series held in LDS
constexpr int INTEG_SEG = INTEG_MAX_T / WG;   // positions per thread in the series passes (32)

// dynamic LDS of the integrated kernel for blocks of up to Tmax samples (the
// value and mask areas also hold the spectrum, up to MAXC channels)
__host__ __device__ inline size_t integ_lds_bytes(int Tmax) {
  const size_t n = (size_t)(Tmax > MAXC ? Tmax : MAXC);
  return n * 8 + (size_t)MAXC * 8 + (size_t)NW * 64 * 8 + (n / 64 + 2) * 8 + 17 * 8 + 1024 + 16 * 8 + 128 * 8 + 256;
}

struct IntegSm {
  uint64_t* val;      // series values (u64 integers / double bits), up to Tmax
  uint64_t* spec;     // spectrum, up to MAXC
  uint64_t* part;     // [NW][64] per-wave row partial sums (float input)
  uint64_t* mask;     // mask words of the series being flagged
  uint64_t* cmask;    // channel mask words (17)
  uint32_t* hist;     // 256 radix bins
  double* T;          // thresholds (16)
  int64_t* G;         // integer window thresholds of one level, by count 0..64 (+pad)
  int64_t* red;       // block reduction scratch (32 x 8 B)
};

__device__ __forceinline__ IntegSm integ_carve(unsigned char* base, int Tmax) {
  IntegSm s;
  const size_t n = (size_t)(Tmax > MAXC ? Tmax : MAXC);
  unsigned char* p = base;
  s.val = (uint64_t*)p;  p += n * 8;
  s.spec = (uint64_t*)p; p += (size_t)MAXC * 8;
  s.part = (uint64_t*)p; p += (size_t)NW * 64 * 8;
  s.mask = (uint64_t*)p; p += (n / 64 + 2) * 8;
  s.cmask = (uint64_t*)p; p += 17 * 8;
  s.hist = (uint32_t*)p; p += 1024;
  s.T = (double*)p;      p += 16 * 8;
  s.G = (int64_t*)p;     p += 128 * 8;
  s.red = (int64_t*)p;
  return s;
}

// ---------------------------------------------------------------- block reductions
template <class F>
__device__ __forceinline__ int64_t block_reduce_i64(int64_t x, int64_t* red, F&& op) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = op(x, (int64_t)__shfl_xor((long long)x, d));
  __syncthreads();
  if (lane == 0) red[wv] = x;
  __syncthreads();
  int64_t r = red[0];
  for (int w = 1; w < NW; ++w) r = op(r, red[w]);
  __syncthreads();
  return r;
}

// sums of four 64-bit integers over the workgroup at once (one set of barriers)
__device__ __forceinline__ void block_sum4_i64(int64_t (&x)[4], int64_t* red) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] += (int64_t)__shfl_xor((long long)x[k], d);
  __syncthreads();
  const int64_t mine = lane == 0 ? x[0] : (lane == 1 ? x[1] : (lane == 2 ? x[2] : x[3]));
  if (lane < 4) red[4 * wv + lane] = mine;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int64_t r = 0;
    for (int w = 0; w < NW; ++w) r += red[4 * w + k];
    x[k] = r;
  }
  __syncthreads();
}

// sum of doubles in a fixed order: lanes by a shuffle tree, waves in order
__device__ __forceinline__ double block_sum_f64(double x, int64_t* red) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  __syncthreads();
  if (lane == 0) red[wv] = __double_as_longlong(x);
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < NW; ++w) r += __longlong_as_double(red[w]);
  __syncthreads();
  return r;
}

// scans over the threads of the workgroup, in thread order
__device__ __forceinline__ int64_t block_scan_incl(int64_t x, int64_t* red) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = (int64_t)__shfl_up((long long)x, d);
    if (lane >= d) x += y;
  }
  __syncthreads();
  if (lane == 63) red[wv] = x;
  __syncthreads();
  for (int w = 0; w < wv; ++w) x += red[w];
  __syncthreads();
  return x;
}

// min over the threads before this one (BIG for thread 0)
__device__ __forceinline__ int block_scan_min_excl(int x, int64_t* red) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  int incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d);
    if (lane >= d) incl = min(incl, y);
  }
  int excl = __shfl_up(incl, 1);
  if (lane == 0) excl = BIG;
  __syncthreads();
  if (lane == 63) red[wv] = incl;
  __syncthreads();
  for (int w = 0; w < wv; ++w) excl = min(excl, (int)red[w]);
  __syncthreads();
  return excl;
}

// max over the threads after this one (-BIG for the last)
__device__ __forceinline__ int block_scan_max_excl_rev(int x, int64_t* red) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  int incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_down(incl, d);
    if (lane + d < 64) incl = max(incl, y);
  }
  int excl = __shfl_down(incl, 1);
  if (lane == 63) excl = -BIG;
  __syncthreads();
  if (lane == 0) red[wv] = incl;
  __syncthreads();
  for (int w = wv + 1; w < NW; ++w) excl = max(excl, (int)red[w]);
  __syncthreads();
  return excl;
}

// ---------------------------------------------------------------- exact integer moments
// correctly rounded (round to nearest even) value of the 128-bit integer hi:lo
// divided by n (1 <= n < 2^32), as a double.  The dividend is first shifted left
// by k bits so that the integer quotient has at least 55 significant bits; the
// quotient's top 53 bits, the next bit and whether anything nonzero follows
// (lower quotient bits or a remainder) give the rounding; the result is scaled
// back by 2^-k.
__device__ __forceinline__ double u128_div_rn(uint64_t hi, uint64_t lo, uint64_t n) {
  if (hi == 0 && lo == 0) return 0.0;
  const int bl_s = hi ? 128 - __builtin_clzll(hi) : 64 - __builtin_clzll(lo);
  const int bl_n = 64 - __builtin_clzll(n);
  const int k = max(0, 56 + bl_n - bl_s);
  // (hi:lo) << k, k <= 88 and bl_s + k <= 128
  if (k >= 64) {
    hi = lo << (k - 64);
    lo = 0;
  } else if (k > 0) {
    hi = (hi << k) | (lo >> (64 - k));
    lo <<= k;
  }
  // long division by n in 32-bit digits: 128-bit quotient qhi:qlo, remainder r
  uint64_t q[4];
  uint64_t r = 0;
  const uint32_t w[4] = {(uint32_t)(hi >> 32), (uint32_t)hi, (uint32_t)(lo >> 32), (uint32_t)lo};
  for (int i = 0; i < 4; ++i) {
    const uint64_t cur = (r << 32) | w[i];
    q[i] = cur / n;
    r = cur % n;
  }
  const uint64_t qhi = (q[0] << 32) | q[1], qlo = (q[2] << 32) | q[3];
  const int nbits = qhi ? 128 - __builtin_clzll(qhi) : 64 - __builtin_clzll(qlo);   // >= 55
  const int sh = nbits - 53;                  // quotient bits below the significand (>= 2)
  uint64_t mant, rest_hi, rest_lo;            // mant = q >> sh, rest = q mod 2^sh
  if (sh >= 64) {
    mant = qhi >> (sh - 64);
    rest_hi = (sh > 64) ? (qhi & ((1ull << (sh - 64)) - 1)) : 0;
    rest_lo = qlo;
  } else {
    mant = (qlo >> sh) | (qhi << (64 - sh));
    rest_hi = 0;
    rest_lo = qlo & ((1ull << sh) - 1);
  }
  // compare rest + r/n with half = 2^(sh-1)
  bool above, equal;
  if (sh - 1 >= 64) {
    const uint64_t hb = 1ull << (sh - 1 - 64);
    above = rest_hi > hb || (rest_hi == hb && (rest_lo != 0 || r != 0));
    equal = rest_hi == hb && rest_lo == 0 && r == 0;
  } else {
    const uint64_t hb = 1ull << (sh - 1);
    above = rest_hi != 0 || rest_lo > hb || (rest_lo == hb && r != 0);
    equal = rest_hi == 0 && rest_lo == hb && r == 0;
  }
  if (above || (equal && (mant & 1))) ++mant;   // mant <= 2^53: exact in a double
  return __builtin_ldexp((double)mant, sh - k);
}

// population stddev of the n series values in vals, with the oracle's formula
template <bool INT>
__device__ __forceinline__ double integ_stddev(const IntegSm& s, const uint64_t* vals, int n) {
  const int tid = thread_id();
  if constexpr (INT) {
    unsigned __int128 s2 = 0;
    uint64_t s1 = 0;
    for (int i = tid; i < n; i += WG) {
      const uint64_t v = vals[i];
      s1 += v;
      s2 += (unsigned __int128)v * v;
    }
    // 128-bit sum: the low word in two 32-bit halves (sums of 512 of them stay
    // below 2^41) and the high word, all added exactly
    const uint64_t lo = (uint64_t)s2, hi = (uint64_t)(s2 >> 64);
    int64_t v4[4] = {(int64_t)s1, (int64_t)(lo & 0xffffffffull), (int64_t)(lo >> 32), (int64_t)hi};
    block_sum4_i64(v4, s.red);
    const int64_t S1 = v4[0], A = v4[1], B = v4[2], Hs = v4[3];
    // S2 = Hs * 2^64 + B * 2^32 + A (A, B < 2^41)
    const unsigned __int128 S2 = ((unsigned __int128)(uint64_t)Hs << 64) + ((unsigned __int128)(uint64_t)B << 32) +
                                 (unsigned __int128)(uint64_t)A;
    const double mu = (double)(uint64_t)S1 / (double)n;   // S1 < 2^53: one rounding
    const double ex2 = u128_div_rn((uint64_t)(S2 >> 64), (uint64_t)S2, (uint64_t)n);
    double var = ex2 - mu * mu;
    if (var < 0.0) var = 0.0;
    return __builtin_sqrt(var);
  } else {
    double a = 0.0, b = 0.0;
    for (int i = tid; i < n; i += WG) {
      const double v = __longlong_as_double((long long)vals[i]);
      a += v;
      b += v * v;
    }
    const double S1 = block_sum_f64(a, s.red), S2 = block_sum_f64(b, s.red);
    const double mu = S1 / (double)n, ex2 = S2 / (double)n;
    double var = ex2 - mu * mu;
    if (var < 0.0) var = 0.0;
    return __builtin_sqrt(var);
  }
}

// ---------------------------------------------------------------- median (radix select)
// order-preserving 64-bit key of a series value
template <bool INT>
__device__ __forceinline__ uint64_t integ_key(uint64_t v) {
  if constexpr (INT) return v;
  return (v & 0x8000000000000000ull) ? ~v : (v | 0x8000000000000000ull);
}
template <bool INT>
__device__ __forceinline__ double integ_key_value(uint64_t k) {
  if constexpr (INT) return (double)k;
  const uint64_t v = (k & 0x8000000000000000ull) ? (k ^ 0x8000000000000000ull) : ~k;
  return __longlong_as_double((long long)v);
}

// the key of rank r (0-based) among the n values, by 8-bit digits from the most
// significant byte in which the smallest and largest key differ (every key
// shares the bytes above it); kmin / kmax are the extreme keys
template <class KF>
__device__ __forceinline__ uint64_t integ_select(const IntegSm& s, const uint64_t* vals, int n, uint32_t r,
                                                 uint64_t kmin, uint64_t kmax, KF key) {
  const int tid = thread_id(), lane = tid & 63;
  if (kmin == kmax) return kmin;
  const int top = 63 - __builtin_clzll(kmin ^ kmax);      // highest differing bit
  int shift = (top / 8) * 8;
  // the bytes above `shift + 8` are the same in every key
  uint64_t prefix = (shift + 8 >= 64) ? 0ull : ((kmin >> (shift + 8)) << (shift + 8));
  for (; shift >= 0; shift -= 8) {
    for (int i = tid; i < 256; i += WG) s.hist[i] = 0u;
    __syncthreads();
    const uint64_t hmask = (shift + 8 >= 64) ? 0ull : (~0ull << (shift + 8));
    for (int i = tid; i < n; i += WG) {
      const uint64_t k = key(vals[i]);
      if ((k & hmask) == prefix) atomicAdd(&s.hist[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    // the digit holding rank r: the first wave scans the 256 bins (4 per lane)
    if (tid < 64) {
      uint32_t c[4], sum = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c[j] = s.hist[4 * lane + j];
        sum += c[j];
      }
      uint32_t x = sum;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
      }
      uint32_t before = x - sum;
      if (r >= before && r < x) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (r >= before && r < before + c[j]) {
            s.red[16] = 4 * lane + j;
            s.red[17] = (int64_t)(r - before);
          }
          before += c[j];
        }
      }
    }
    __syncthreads();
    prefix |= (uint64_t)s.red[16] << shift;
    r = (uint32_t)s.red[17];
    __syncthreads();
  }
  return prefix;
}

// the two middle order statistics' keys (equal for odd n): the lower by radix
// select, the upper as the same key when it occurs often enough, else the
// smallest key above it
template <class KF>
__device__ __forceinline__ void integ_middle(const IntegSm& s, const uint64_t* vals, int n, KF key, uint64_t& k0,
                                             uint64_t& k1) {
  const int tid = thread_id();
  uint64_t mn = ~0ull, mx = 0ull;
  for (int i = tid; i < n; i += WG) {
    const uint64_t k = key(vals[i]);
    mn = k < mn ? k : mn;
    mx = k > mx ? k : mx;
  }
  const uint64_t kmin = (uint64_t)block_reduce_i64((int64_t)(mn ^ 0x8000000000000000ull), s.red,
                                                   [](int64_t a, int64_t b) { return a < b ? a : b; }) ^
                        0x8000000000000000ull;
  const uint64_t kmax = (uint64_t)block_reduce_i64((int64_t)(mx ^ 0x8000000000000000ull), s.red,
                                                   [](int64_t a, int64_t b) { return a > b ? a : b; }) ^
                        0x8000000000000000ull;
  const uint32_t r0 = (uint32_t)((n - 1) / 2), r1 = (uint32_t)(n / 2);
  k0 = integ_select(s, vals, n, r0, kmin, kmax, key);
  if (r1 == r0) {
    k1 = k0;
    return;
  }
  int le = 0;
  uint64_t above = ~0ull;
  for (int i = tid; i < n; i += WG) {
    const uint64_t k = key(vals[i]);
    le += k <= k0 ? 1 : 0;
    if (k > k0 && k < above) above = k;
  }
  const int64_t cnt = block_reduce_i64((int64_t)le, s.red, [](int64_t a, int64_t b) { return a + b; });
  const uint64_t nxt = (uint64_t)block_reduce_i64((int64_t)(above ^ 0x8000000000000000ull), s.red,
                                                  [](int64_t a, int64_t b) { return a < b ? a : b; }) ^
                       0x8000000000000000ull;
  k1 = cnt > (int64_t)r1 ? k0 : nxt;
}

// ---------------------------------------------------------------- 1-D SumThreshold + SIR
// Flags the n values in vals (mask words in s.mask, which start cleared):
// median, stddev and thresholds of the series, nl SumThreshold levels with
// windows of I = 2^k <= n (level-synchronous, flagged samples out of sum and
// count), then the SIR step.  Thread t takes the positions [t*SEG, t*SEG + SEG).
template <bool INT>
__device__ __forceinline__ void integ_flag_series(const IntegSm& s, const uint64_t* vals, int n, int nl, const DevParams& P,
                                  double* med_out, double* sd_out) {
  const int tid = thread_id();
  const int nw = (n + 63) >> 6;
  for (int i = tid; i < nw; i += WG) s.mask[i] = 0ull;
  // median (numpy definition) and stddev
  uint64_t k0, k1;
  integ_middle(s, vals, n, [](uint64_t v) { return integ_key<INT>(v); }, k0, k1);
  const double v0 = integ_key_value<INT>(k0), v1 = integ_key_value<INT>(k1);
  const double med = (n & 1) ? v0 : (v0 + v1) / 2.0;
  double sd;
  if (P.robust) {
    // 1.4826 * MAD: the middle order statistics of the deviations from the
    // median (integer series: doubled deviations |2v - med2|, exact)
    uint64_t m0, m1;
    double mad;
    if (INT) {
      const uint64_t med2 = k0 + k1;
      integ_middle(s, vals, n, [med2](uint64_t v) { return 2 * v > med2 ? 2 * v - med2 : med2 - 2 * v; }, m0, m1);
      mad = ((double)m0 + (double)m1) / 4.0;
    } else {
      integ_middle(s, vals, n, [med](uint64_t v) {
        return integ_key<false>((uint64_t)__double_as_longlong(__builtin_fabs(__longlong_as_double((long long)v) - med)));
      }, m0, m1);
      mad = (integ_key_value<false>(m0) + integ_key_value<false>(m1)) / 2.0;
    }
    sd = MAD_TO_SIGMA * mad;
  } else {
    sd = integ_stddev<INT>(s, vals, n);
  }
  if (tid == 0) {
    double pk = 1.0;
    for (int k = 0; k < 16; ++k) {
      if (k < max(1, nl)) {
        const double f = P.start * pk / (double)(1 << k);
        s.T[k] = med + sd * (f * P.sens);
        pk = pk * P.p;
      } else {
        s.T[k] = 0.0;
      }
    }
  }
  *med_out = med;
  *sd_out = sd;
  __syncthreads();
  // thread t takes the positions [t*seg, t*seg + seg), seg <= 32
  const int seg = (n + WG - 1) / WG;
  const int a = tid * seg;
  for (int k = 0; k < nl && k < ST_MAX_LEVELS; ++k) {
    const int I = 1 << k;
    if (I > n) break;
    const double Tk = s.T[k];
    if (INT) {
      // exact window thresholds floor(c * T_k) for c = 0..I (FMA-exact floor)
      for (int c = tid; c <= I; c += WG) {
        const double cd = (double)c, prod = cd * Tk, err = __builtin_fma(cd, Tk, -prod);
        double fl = __builtin_floor(prod);
        if (prod == fl && err < 0.0) fl -= 1.0;
        s.G[c] = fl >= 9.0e18 ? INT64_MAX : (fl <= -9.0e18 ? INT64_MIN : (int64_t)fl);
      }
      __syncthreads();
    }
    // windows starting in this thread's positions: running sum and count
    uint32_t hits = 0;
    const int s_end = min(a + seg, n - I + 1);
    if (a < s_end) {
      int64_t Si = 0;
      double Sf = 0.0;
      int cnt = 0;
      // the first window, 8 positions at a time so their LDS reads are in flight
      // together (the sum is still taken in position order)
      int j = a;
      for (; j + 8 <= a + I; j += 8) {
        uint64_t v[8];
        bool fl[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          fl[q] = (s.mask[(j + q) >> 6] >> ((j + q) & 63)) & 1ull;
          v[q] = vals[j + q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (!fl[q]) {
            ++cnt;
            if (INT) Si += (int64_t)v[q];
            else Sf += __longlong_as_double((long long)v[q]);
          }
        }
      }
      for (; j < a + I; ++j) {
        const bool fl = (s.mask[j >> 6] >> (j & 63)) & 1ull;
        if (!fl) {
          ++cnt;
          if (INT) Si += (int64_t)vals[j];
          else Sf += __longlong_as_double((long long)vals[j]);
        }
      }
      for (int st = a; st < s_end; ++st) {
        if (st > a) {
          const int out = st - 1, in = st + I - 1;
          if (!((s.mask[out >> 6] >> (out & 63)) & 1ull)) {
            --cnt;
            if (INT) Si -= (int64_t)vals[out];
            else Sf -= __longlong_as_double((long long)vals[out]);
          }
          if (!((s.mask[in >> 6] >> (in & 63)) & 1ull)) {
            ++cnt;
            if (INT) Si += (int64_t)vals[in];
            else Sf += __longlong_as_double((long long)vals[in]);
          }
        }
        bool h;
        if (INT) h = cnt > 0 && Si > s.G[cnt];
        else h = cnt > 0 && Sf > (double)cnt * Tk;
        if (h) hits |= 1u << (st - a);
      }
    }
    __syncthreads();   // every window of the level judged on the previous mask
    while (hits) {
      const int j = __builtin_ctz(hits);
      hits &= hits - 1;
      const int st = a + j;
      // positions [st, st + I): at most two mask words
      const int w0 = st >> 6, b0 = st & 63;
      const uint64_t m0 = (b0 + I >= 64) ? (~0ull << b0) : (lowmask(I) << b0);
      uint32_t* h32 = reinterpret_cast<uint32_t*>(s.mask);
      if ((uint32_t)m0) atomicOr(&h32[2 * w0], (uint32_t)m0);
      if ((uint32_t)(m0 >> 32)) atomicOr(&h32[2 * w0 + 1], (uint32_t)(m0 >> 32));
      if (b0 + I > 64) {
        const uint64_t m1 = lowmask(b0 + I - 64);
        if ((uint32_t)m1) atomicOr(&h32[2 * w0 + 2], (uint32_t)m1);
        if ((uint32_t)(m1 >> 32)) atomicOr(&h32[2 * w0 + 3], (uint32_t)(m1 >> 32));
      }
    }
    __syncthreads();
  }
  // SIR step on the series mask
  if (P.eta_num > 0) {
    if (P.prose) {
      // forward and backward scans by one thread over the words
      if (tid == 0) {
        const FastDiv fd((uint32_t)P.eta_den);
        ProseScan f{0u, 0};
        uint64_t* out = s.part;   // forward result words (n / 64 <= 256 <= NW * 64)
        for (int w = 0; w < nw; ++w) {
          const int nb = min(64, n - 64 * w);
          out[w] = prose_fwd_word(s.mask[w] & lowmask(nb), 64 * w, nb, f, (uint32_t)P.eta_num, fd);
        }
        ProseScan r{0u, n};
        for (int w = nw - 1; w >= 0; --w) {
          const int nb = min(64, n - 64 * w);
          const uint64_t x = s.mask[w] & lowmask(nb);
          s.mask[w] = out[w] | prose_bwd_word(x, 64 * w, nb, r, (uint32_t)P.eta_num, fd);
        }
      }
      __syncthreads();
    } else {
      // linear form, the thread's seg positions in a lane summary (up to 32),
      // block scans between threads
      const int num = P.eta_num, den = P.eta_den;
      const int nval = clampi(n - a, 0, seg);
      uint64_t bits = 0;
      if (nval > 0) {
        const int w0 = a >> 6, o = a & 63;
        bits = s.mask[w0] >> o;
        if (o + nval > 64) bits |= s.mask[w0 + 1] << (64 - o);
        bits &= lowmask(nval);
      }
      const SirSum ss = sir_lane_summary<INTEG_SEG>(bits, nval, num, den);
      // exclusive prefix sum of the totals, prefix min of base + mn, suffix max of base + mx
      const int64_t tot_incl = block_scan_incl(ss.tot, s.red);
      const int base = (int)(tot_incl - ss.tot);
      const int pm = block_scan_min_excl(nval > 0 ? base + ss.mn : BIG, s.red);
      const int sx = block_scan_max_excl_rev(nval > 0 ? base + ss.mx : -BIG, s.red);
      const uint64_t out = sir_lane_apply<INTEG_SEG>(bits, nval, num, den, base, pm, sx);
      __syncthreads();
      if (nval > 0) {
        // the segment's bits may straddle two mask words
        uint32_t* h32 = reinterpret_cast<uint32_t*>(s.mask);
        const int w0 = a >> 6, o = a & 63;
        const uint64_t lo = out << o, hi = o ? (out >> (64 - o)) : 0ull;
        if ((uint32_t)lo) atomicOr(&h32[2 * w0], (uint32_t)lo);
        if ((uint32_t)(lo >> 32)) atomicOr(&h32[2 * w0 + 1], (uint32_t)(lo >> 32));
        if ((uint32_t)hi) atomicOr(&h32[2 * w0 + 2], (uint32_t)hi);
        if ((uint32_t)(hi >> 32)) atomicOr(&h32[2 * w0 + 3], (uint32_t)(hi >> 32));
      }
      __syncthreads();
    }
  }
}

// lane q's 64-bit value (q wave-uniform), each half zero-extended
__device__ __forceinline__ uint64_t lane_u64(uint64_t x, int q) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, q);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), q);
  return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// the key of rank r among the first n lanes' keys (ties by lane), wave-uniform
__device__ __forceinline__ uint64_t wave_rank_key(uint64_t key, int n, int r, int lane) {
  int rank = 0;
  for (int q = 0; q < n; ++q) {
    const uint64_t kq = lane_u64(key, q);
    rank += (kq < key || (kq == key && q < lane)) ? 1 : 0;
  }
  const unsigned long long b = __ballot(lane < n && rank == r);
  return lane_u64(key, __ffsll(b) - 1);
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  return x;
}

// The series of at most 64 values (the spectrum of a block of at most 64
// channels) flagged by wave 0 alone, value i in lane i: the statistics, the
// thresholds, SumThreshold and the SIR step of integ_flag_series, with wave
// shuffles in place of block barriers.  Writes s.mask[0] and s.T; every thread
// returns the median and stddev.
template <bool INT>
__device__ __forceinline__ void integ_flag_series_wave(const IntegSm& s, const uint64_t* vals, int n, int nl,
                                                       const DevParams& P, double* med_out, double* sd_out) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  if (wv == 0) {
    const bool live = lane < n;
    const uint64_t v = live ? vals[lane] : 0ull;
    const uint64_t key = integ_key<INT>(v);
    const int r0 = (n - 1) / 2, r1 = n / 2;
    const uint64_t k0 = wave_rank_key(key, n, r0, lane);
    const uint64_t k1 = (r1 == r0) ? k0 : wave_rank_key(key, n, r1, lane);
    const double v0 = integ_key_value<INT>(k0), v1 = integ_key_value<INT>(k1);
    const double med = (n & 1) ? v0 : (v0 + v1) / 2.0;
    double sd;
    if (P.robust) {
      // 1.4826 * MAD (integer series: doubled deviations |2v - med2|, exact)
      uint64_t dk;
      if (INT) {
        const uint64_t med2 = k0 + k1;
        dk = 2 * v > med2 ? 2 * v - med2 : med2 - 2 * v;
      } else {
        dk = integ_key<false>((uint64_t)__double_as_longlong(__builtin_fabs(__longlong_as_double((long long)v) - med)));
      }
      const uint64_t m0 = wave_rank_key(dk, n, r0, lane);
      const uint64_t m1 = (r1 == r0) ? m0 : wave_rank_key(dk, n, r1, lane);
      const double mad = INT ? ((double)m0 + (double)m1) / 4.0
                             : (integ_key_value<false>(m0) + integ_key_value<false>(m1)) / 2.0;
      sd = MAD_TO_SIGMA * mad;
    } else if constexpr (INT) {
      // exact moments: S1 < 2^53; S2 from the 32-bit halves of the squares' low
      // words and their high words (sums of 64 stay exact)
      const unsigned __int128 sq = (unsigned __int128)v * v;
      const uint64_t lo = (uint64_t)sq, hi = (uint64_t)(sq >> 64);
      const uint64_t S1 = wave_sum<unsigned long long>(v);
      const uint64_t A = wave_sum<unsigned long long>(lo & 0xffffffffull);
      const uint64_t B = wave_sum<unsigned long long>(lo >> 32);
      const uint64_t Hs = wave_sum<unsigned long long>(hi);
      const unsigned __int128 S2 = ((unsigned __int128)Hs << 64) + ((unsigned __int128)B << 32) + (unsigned __int128)A;
      const double mu = (double)S1 / (double)n;
      const double ex2 = u128_div_rn((uint64_t)(S2 >> 64), (uint64_t)S2, (uint64_t)n);
      double var = ex2 - mu * mu;
      if (var < 0.0) var = 0.0;
      sd = __builtin_sqrt(var);
    } else {
      const double x = __longlong_as_double((long long)v);
      const double S1 = wave_sum<double>(x), S2 = wave_sum<double>(x * x);
      const double mu = S1 / (double)n, ex2 = S2 / (double)n;
      double var = ex2 - mu * mu;
      if (var < 0.0) var = 0.0;
      sd = __builtin_sqrt(var);
    }
    // lane k < max(1, nl) holds the level-k threshold (p^k by k products, as
    // integ_flag_series forms it)
    double Tl = 0.0;
    if (lane < max(1, nl)) {
      double pk = 1.0;
      for (int j = 0; j < lane; ++j) pk = pk * P.p;
      Tl = med + sd * ((P.start * pk / (double)(1 << lane)) * P.sens);
    }
    // SumThreshold, level-synchronous, on the prefix sums of the unflagged values
    uint64_t M = 0;
    for (int k = 0; k < nl && k < ST_MAX_LEVELS; ++k) {
      const int I = 1 << k;
      if (I > n) break;
      const double Tk = lane_double(Tl, k);
      const bool keep = live && !((M >> lane) & 1ull);
      uint64_t Pi = (INT && keep) ? v : 0ull;
      double Pf = (!INT && keep) ? __longlong_as_double((long long)v) : 0.0;
      int Pc = keep ? 1 : 0;
      for (int d = 1; d < 64; d <<= 1) {
        const uint64_t yi = __shfl_up(Pi, d);
        const double yf = __shfl_up(Pf, d);
        const int yc = __shfl_up(Pc, d);
        if (lane >= d) {
          Pi += yi;
          Pf += yf;
          Pc += yc;
        }
      }
      uint64_t Ei = __shfl_up(Pi, 1);
      double Ef = __shfl_up(Pf, 1);
      int Ec = __shfl_up(Pc, 1);
      if (lane == 0) {
        Ei = 0ull;
        Ef = 0.0;
        Ec = 0;
      }
      const int e = min(lane + I - 1, 63);
      const int c = __shfl(Pc, e) - Ec;
      bool hit;
      if (INT) {
        const int64_t S = (int64_t)(__shfl(Pi, e) - Ei);
        // floor(c * T_k), FMA-exact, for this window's count
        const double cd = (double)c, prod = cd * Tk, err = __builtin_fma(cd, Tk, -prod);
        double fl = __builtin_floor(prod);
        if (prod == fl && err < 0.0) fl -= 1.0;
        const int64_t g = fl >= 9.0e18 ? INT64_MAX : (fl <= -9.0e18 ? INT64_MIN : (int64_t)fl);
        hit = c > 0 && S > g;
      } else {
        const double S = __shfl(Pf, e) - Ef;
        hit = c > 0 && S > (double)c * Tk;
      }
      const unsigned long long H = __ballot(hit && lane <= n - I);
      if (H == 0) continue;
      uint64_t Wm = H;
      for (int d = 1; d < I; d <<= 1) Wm |= Wm << d;
      M |= Wm & lowmask(n);
    }
    // SIR step on the series mask
    if (P.eta_num > 0) {
      if (P.prose) {
        const FastDiv fd((uint32_t)P.eta_den);
        ProseScan f{0u, 0};
        const uint64_t fw = prose_fwd_word(M, 0, n, f, (uint32_t)P.eta_num, fd);
        ProseScan r{0u, n};
        M = fw | prose_bwd_word(M, 0, n, r, (uint32_t)P.eta_num, fd);
      } else if (P.eta_num >= P.eta_den) {
        M = lowmask(n);   // eta = 1: every interval qualifies
      } else if (M != 0) {
        const int cw = P.eta_den - P.eta_num;
        const FastDiv fc((uint32_t)cw);
        M = sir_runs_lane(M, n, P.eta_num, cw, fc);
      }
    }
    if (lane == 0) {
      s.mask[0] = M;
      s.red[0] = __double_as_longlong(med);
      s.red[1] = __double_as_longlong(sd);
    }
    if (lane < 16) s.T[lane] = Tl;
  }
  __syncthreads();
  *med_out = __longlong_as_double(s.red[0]);
  *sd_out = __longlong_as_double(s.red[1]);
  __syncthreads();
}

// ---------------------------------------------------------------- the block
// powers of 8 consecutive samples of a row from t0 (zero past the row's end)
template <bool INT>
__device__ __forceinline__ void integ_load8(const DevBlock& b, int row, int t0, typename PowT<INT>::T (&v)[8]) {
  if (b.aligned && t0 + 8 <= b.T) load8v<INT>(b, row, t0, v);
  else load8<INT>(b, row, t0, v);
}

template <bool INT>
__device__ __forceinline__ void phase_integrated(const DevBlock& b, const DevParams& P, const IntegSm& s) {
  typedef typename PowT<INT>::T VT;
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int C = b.C, T = b.T, W = (T + 63) >> 6;
  const int nq = (T + 8 * WG - 1) / (8 * WG);   // chunks of 8 columns per thread (<= 4)
  for (int i = tid; i < C; i += WG) s.spec[i] = 0ull;
  for (int i = tid; i < 17; i += WG) s.cmask[i] = 0ull;
  __syncthreads();
  // one pass: column sums in registers (each thread owns its columns; integer
  // column sums stay below 2^25), row sums by wave reductions, RB rows at a time
  // so that their loads are in flight together (exact integer atomics, or
  // per-wave partials added in wave order for float input)
  constexpr int RB = 4;
  uint32_t ci[4][8];
  double cf[4][8];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ci[q][j] = 0u;
      cf[q][j] = 0.0;
    }
  for (int r0 = 0; r0 < C; r0 += 64) {
    const int r1 = min(C, r0 + 64);
    for (int rb = r0; rb < r1; rb += RB) {
      uint32_t rsi[RB];
      double rsf[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        rsi[u] = 0u;
        rsf[u] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t0 = (tid + q * WG) * 8;
        if (q < nq && t0 < T) {
          VT v[RB][8];
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            if (rb + u < r1) {
              integ_load8<INT>(b, rb + u, t0, v[u]);
            } else {
#pragma unroll
              for (int j = 0; j < 8; ++j) v[u][j] = (VT)0;
            }
          }
#pragma unroll
          for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              if (INT) {
                ci[q][j] += (uint32_t)v[u][j];
                rsi[u] += (uint32_t)v[u][j];
              } else {
                cf[q][j] += (double)v[u][j];
                rsf[u] += (double)v[u][j];
              }
            }
        }
        // one chunk's RB loads in flight at a time: hoisting all chunks' loads
        // would hold 4 x RB x 8 values
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          if (INT) rsi[u] += __shfl_xor(rsi[u], d);
          else rsf[u] += __shfl_xor(rsf[u], d);
        }
      if (lane == 0) {
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          if (rb + u >= r1) continue;
          if (INT) {
            if (rsi[u]) atomicAdd((unsigned long long*)&s.spec[rb + u], (unsigned long long)rsi[u]);
          } else {
            s.part[wv * 64 + (rb + u - r0)] = (uint64_t)__double_as_longlong(rsf[u]);
          }
        }
      }
    }
    if (!INT) {
      __syncthreads();
      for (int row = r0 + tid; row < r1; row += WG) {
        double acc = 0.0;
        for (int w = 0; w < NW; ++w) acc += __longlong_as_double((long long)s.part[w * 64 + (row - r0)]);
        s.spec[row] = (uint64_t)__double_as_longlong(acc);
      }
      __syncthreads();
    }
  }
  // the all-channel time series into LDS (each thread writes only its columns)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t0 = (tid + q * WG) * 8;
    if (q < nq && t0 < T) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (t0 + j < T) s.val[t0 + j] = INT ? (uint64_t)ci[q][j] : (uint64_t)__double_as_longlong(cf[q][j]);
    }
  }
  __syncthreads();
  // spectrum: flag along frequency first
  double med, sd;
  if (C <= 64) integ_flag_series_wave<INT>(s, s.spec, C, min(P.nl_f, ST_MAX_LEVELS), P, &med, &sd);
  else integ_flag_series<INT>(s, s.spec, C, min(P.nl_f, ST_MAX_LEVELS), P, &med, &sd);
  for (int i = tid; i < (C + 63) / 64; i += WG) s.cmask[i] = s.mask[i];
  if (INT) {
    // the rows' exact power sums, for the history flagger
    for (int i = tid; i < C; i += WG) gp<uint64_t>(P.rowsum)[(int64_t)b.sidx * P.maxC + i] = s.spec[i];
  }
  __syncthreads();
  // the time series of the unflagged channels
  int nflag = 0;
  for (int i = 0; i < (C + 63) / 64; ++i) nflag += __popcll(s.cmask[i]);
  if (INT) {
    // subtract the flagged rows from the all-channel column sums (exact)
    for (int w = 0; w < (C + 63) / 64; ++w) {
      uint64_t m = s.cmask[w];
      while (m) {
        const int row = 64 * w + __builtin_ctzll(m);
        m &= m - 1;
        for (int q = 0; q < nq; ++q) {
          const int t0 = (tid + q * WG) * 8;
          if (t0 < T) {
            VT v[8];
            integ_load8<INT>(b, row, t0, v);
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if (t0 + j < T) s.val[t0 + j] -= (uint64_t)v[j];
          }
        }
      }
    }
  } else if (nflag > 0) {
    // float input: the sums over the unflagged channels again, in row order
    for (int q = 0; q < nq; ++q) {
      const int t0 = (tid + q * WG) * 8;
      if (t0 >= T) continue;
      double acc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = 0.0;
      for (int row = 0; row < C; ++row) {
        if ((s.cmask[row >> 6] >> (row & 63)) & 1ull) continue;
        VT v[8];
        integ_load8<INT>(b, row, t0, v);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += (double)v[j];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (t0 + j < T) s.val[t0 + j] = (uint64_t)__double_as_longlong(acc[j]);
    }
  }
  __syncthreads();
  integ_flag_series<INT>(s, s.val, T, min(P.nl_t, ST_MAX_LEVELS), P, &med, &sd);
  // the block's mask words: a flagged channel's whole row, else the time flags
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  for (int i = tid; i < C * W; i += WG) {
    const int row = i / W, w = i - row * W;
    const uint64_t valid = lowmask(min(64, T - 64 * w));
    const bool chan = (s.cmask[row >> 6] >> (row & 63)) & 1ull;
    m0[(int64_t)row * W + w] = chan ? valid : (s.mask[w] & valid);
  }
  // statistics entry: the time series' median, stddev and thresholds; the flag
  // totals are accumulated by the final kernel
  if (P.stats && tid < STATS_BYTES / 8) {
    GLB double* st = (GLB double*)(gp<char>(P.stats) + (int64_t)b.out_idx * STATS_BYTES);
    if (tid == 0) st[0] = med;
    else if (tid == 1) st[1] = sd;
    else if (tid < 2 + LOF_MAX_LEVELS) st[tid] = s.T[tid - 2];
    else *(GLB long long*)(st + tid) = 0;
  }
}

}  // namespace lofk
