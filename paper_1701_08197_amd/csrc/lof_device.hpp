// lof_device.hpp -- device-side building blocks of the LOF flagging kernel (gfx950).
//
// Method: van Nieuwpoort, "Towards exascale real-time RFI mitigation" (arXiv
// 1701.08197).  The kernel runs one workgroup per time-frequency block:
//   phase A  power (Sec. 4), block moments and an exact radix-select median
//            (Sec. 2.1 threshold, Sec. 4.2 O(N) median), thresholds (Sec. 2.1)
//   phase B  SumThreshold along time, then along frequency (Sec. 2.1)
//   phase C  SIR operator along time, then frequency (Sec. 2.2)
//   phase D  history flagger (Sec. 4.1) and the flag-byte write.
//
// Layouts.  A "row" (one channel of the block, along time) is held by a group of
// G consecutive lanes of a wave64, each lane owning L consecutive samples; a
// "column" (one time sample, along frequency) is held the same way with channels
// as positions.  Window sums for I = 2^k are built by doubling,
// S_2I(s) = S_I(s) + S_I(s + I), which needs at most the neighbouring lane's
// registers (I/2 <= L), fetched with DPP wave shifts.  Masks are per-lane u64 bit
// vectors (bit i <-> position lane_in_group*L + i).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lofk {

constexpr int WG = 512;            // threads per workgroup
constexpr int NW = WG / 64;        // waves per workgroup
constexpr int ST_MAX_LEVELS = 7;   // I <= 64: the dependency radius 120 and the packed
                                   // integer sums below rely on it
constexpr int SEG_CORE = 3840;     // time positions finished per segment of a long row
constexpr int SEG_HALO = 128;      // >= 1+3+7+15+31+63 = 120, the 7-level radius
constexpr int SIR_SEG = 4096;      // SIR positions per segment of a long row
constexpr int SIR_MAX_SEGS = 64;
constexpr int HBINS = 4096;        // radix-select digit: 12 bits
constexpr int MAXC = 1024;
constexpr int BIG = 1 << 30;

struct DevBlock {
  const void* data;
  uint8_t* flags;
  int64_t dstride;      // elements
  int64_t fstride;      // bytes
  int32_t C, T, dtype, stream_id;
  int64_t mask_off;     // u64 words into the mask scratch
  int32_t out_idx;      // index of the caller's stats entry
  int32_t aligned;      // data rows 16-byte aligned
  int32_t faligned;     // flag rows 16-byte aligned
  int32_t pad;
};

struct DevParams {
  double start, p, sens, hs;
  int32_t nl_t, nl_f, eta_num, eta_den, H, Hmin, maxC, literal;
  double* ring;          // [streams][maxC][H]
  int32_t* rcount;       // [streams][maxC]
  int32_t* rhead;        // [streams][maxC]
  double* pend;          // [streams][maxC]
  uint8_t* pvalid;       // [streams][maxC]
  uint64_t* maskw;       // mask scratch of this call
  void* stats;           // lof_block_stats* or null
};

// ---------------------------------------------------------------- cross-lane
// wave_shl:1 -> lane i reads lane i+1 (lane 63 reads 0); wave_shr:1 -> lane i reads i-1.
__device__ __forceinline__ uint32_t shl1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float shl1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ uint32_t shr1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint64_t shr1_64(uint64_t v) {
  return (uint64_t)shr1((uint32_t)v) | ((uint64_t)shr1((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ uint64_t shl1_64(uint64_t v) {
  return (uint64_t)shl1((uint32_t)v) | ((uint64_t)shl1((uint32_t)(v >> 32)) << 32);
}
// quad_perm [1,2,3,3]: lane j of a quad reads lane j+1 (lane 3 reads itself)
__device__ __forceinline__ uint64_t quad_next_64(uint64_t v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0xF9, 0xf, 0xf, false);
  uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0xF9, 0xf, 0xf, false);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t lowmask(int n) {
  return n <= 0 ? 0ull : (n >= 64 ? ~0ull : ((1ull << n) - 1ull));
}
__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Loads of mask words written earlier in the kernel by other waves (possibly with
// atomics, which complete in L2): read at agent scope so the vector L1 is bypassed.
__device__ __forceinline__ uint64_t ld_mask(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void or_mask(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- power (Sec. 4)
// complex int8 sample packed in 16 bits (re low byte, im high byte): exact power.
__device__ __forceinline__ uint32_t ci8_power(uint32_t w16) {
  int re = (int)(int8_t)(w16 & 0xffu);
  int im = (int)(int8_t)((w16 >> 8) & 0xffu);
  return (uint32_t)(re * re + im * im);
}
__device__ __forceinline__ float c64_power(float re, float im) { return re * re + im * im; }
__device__ __forceinline__ float c64_amp(float re, float im) { return __builtin_sqrtf(re * re + im * im); }

// power of one sample of a float-typed block (dtype 1, 2, 3)
__device__ __forceinline__ float fpower_at(const DevBlock& b, int row, int t) {
  if (b.dtype == 2) {
    return ((const float*)b.data)[(int64_t)row * b.dstride + t];
  }
  const float2 z = ((const float2*)b.data)[(int64_t)row * b.dstride + t];
  return b.dtype == 1 ? c64_power(z.x, z.y) : c64_amp(z.x, z.y);
}
__device__ __forceinline__ uint32_t ipower_at(const DevBlock& b, int row, int t) {
  return ci8_power(((const uint16_t*)b.data)[(int64_t)row * b.dstride + t]);
}

// 8 consecutive samples of a row starting at t0 (vector loads when aligned and full)
template <bool INT>
struct PowT;
template <>
struct PowT<true> { typedef uint32_t T; };
template <>
struct PowT<false> { typedef float T; };

template <bool INT>
__device__ __forceinline__ int load8(const DevBlock& b, int row, int t0, typename PowT<INT>::T (&v)[8]) {
  const int nv = min(8, b.T - t0);
  if (INT) {
    const uint8_t* rb = (const uint8_t*)b.data + (int64_t)row * b.dstride * 2;
    if (b.aligned && nv == 8) {
      const uint4 q = *(const uint4*)(rb + (int64_t)t0 * 2);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[2 * j] = (typename PowT<INT>::T)ci8_power(w[j] & 0xffffu);
        v[2 * j + 1] = (typename PowT<INT>::T)ci8_power(w[j] >> 16);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        v[j] = (typename PowT<INT>::T)(j < nv ? ci8_power(*(const uint16_t*)(rb + (int64_t)(t0 + j) * 2)) : 0u);
    }
  } else {
    if (b.dtype == 2) {
      const float* rb = (const float*)b.data + (int64_t)row * b.dstride;
      if (b.aligned && nv == 8) {
        const float4 a = *(const float4*)(rb + t0);
        const float4 c = *(const float4*)(rb + t0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = j < nv ? rb[t0 + j] : 0.0f;
      }
    } else {
      const float2* rb = (const float2*)b.data + (int64_t)row * b.dstride;
      const bool amp = b.dtype == 3;
      if (b.aligned && nv == 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float4 a = *(const float4*)(rb + t0 + 2 * j);
          v[2 * j] = amp ? c64_amp(a.x, a.y) : c64_power(a.x, a.y);
          v[2 * j + 1] = amp ? c64_amp(a.z, a.w) : c64_power(a.z, a.w);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float r = 0.0f;
          if (j < nv) {
            const float2 z = rb[t0 + j];
            r = amp ? c64_amp(z.x, z.y) : c64_power(z.x, z.y);
          }
          v[j] = r;
        }
      }
    }
  }
  return nv;
}

// ---------------------------------------------------------------- shared memory
struct Smem {
  union {
    uint32_t hist[2][HBINS];                 // phase A
    struct {
      double rsum[MAXC];                     // history: per-row unflagged sum
      int32_t rcnt[MAXC];                    // history: per-row unflagged count
      int32_t seg[NW][SIR_MAX_SEGS][3];      // SIR: per-segment summaries / carries
    } c;
  } u;
  double T[16];
  float Tf[16];
  int32_t G[ST_MAX_LEVELS][128];   // index: window count c (<= 64); padded to any 7-bit value
  uint32_t rowflag[MAXC / 32];
  double red_d[2][NW];
  unsigned long long red_u[2][NW];
  uint32_t scan[NW];
  uint32_t sel[4];
  double median, sigma;
  unsigned long long nflag;
};

}  // namespace lofk
