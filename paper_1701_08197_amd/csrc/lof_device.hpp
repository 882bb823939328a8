// lof_device.hpp -- device-side building blocks of the LOF flagging kernels (gfx950).
//
// Method: van Nieuwpoort, "Towards exascale real-time RFI mitigation" (arXiv
// 1701.08197).  One kernel per phase, each over (block, chunk) work items:
//   phase A  power (Sec. 4), block moments and an exact median (Sec. 2.1
//            threshold, Sec. 4.2 O(N) median), thresholds (Sec. 2.1); per block
//   phase B  SumThreshold along time (row chunks), then along frequency (column
//            slabs) (Sec. 2.1)
//   phase C  SIR operator along time (row chunks), then frequency (slabs) (Sec. 2.2)
//   phase D  history flagger (Sec. 4.1) and the flag-byte write (row chunks).
// The phases hand over a per-block statistics record and the mask bits in a
// global scratch area (one u64 word per 64 samples of a row).
//
// Layouts.  A "row" (one channel of the block, along time) is held by a group of
// G consecutive lanes of a wave64, each lane owning L consecutive samples; a
// "column" (one time sample, along frequency) is held the same way with channels
// as positions.  Integer rows keep inclusive prefix sums of the packed samples,
// so a window is one difference of two prefixes, the far one read from the next
// lane(s) by DPP wave shifts; float rows and columns build window sums by
// doubling, S_2I(s) = S_I(s) + S_I(s + I).  Masks are per-lane u64 bit vectors
// (bit i <-> position lane_in_group*L + i).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lof.h"

namespace lofk {

// Pointers held in descriptors are plain addresses; dereference them through the
// global address space so the compiler emits global (not flat) memory
// instructions, which do not share a wait counter with LDS traffic.
#define GLB __attribute__((address_space(1)))
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ GLB T* gp(const void* p) {
  return (GLB T*)(uintptr_t)p;
}


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

// the caller's per-block statistics entry (struct lof_block_stats of lof.h)
constexpr int STATS_BYTES = (int)sizeof(lof_block_stats);
constexpr int STATS_NFLAG = (int)offsetof(lof_block_stats, n_flagged);
constexpr int STATS_HROWS = (int)offsetof(lof_block_stats, history_flagged_rows);
static_assert(offsetof(lof_block_stats, threshold) == 2 * sizeof(double), "stats layout");

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
  int32_t sidx;         // index of the block's BlockState in this call
};

// Per-block results of the statistics kernel, read by the later kernels.
struct BlockState {
  double median, sigma;
  double T[16];          // T_k of level k (window 2^k)
};

// ---------------------------------------------------------------- work split
// Each kernel after the statistics one takes a block in chunks: rows for the
// time-direction kernels, column slabs for the frequency-direction kernels.  The
// host sizes the grid with the same functions.
__host__ __device__ inline int time_groups(int T, int L) {   // lanes per row (T <= 64 L)
  int G = 1;
  while (G * L < T) G <<= 1;
  return G;
}
__host__ __device__ inline int time_rows_per_chunk(int T, int L) {
  return T <= 64 * L ? NW * (64 / time_groups(T, L)) : NW;
}
__host__ __device__ inline int time_chunks(int C, int T, int L) {
  const int r = time_rows_per_chunk(T, L);
  return (C + r - 1) / r;
}
__host__ __device__ inline bool freq_colpath(bool integer, int C) {
  return integer && (C == 16 || C == 32 || C == 64);
}
// columns of one frequency slab: LF channels per lane, G lanes per column
__host__ __device__ inline int freq_cols(int C, int LF_min16) {
  const int LF = (C <= 16 && LF_min16) ? 16 : 32;
  int G = 1;
  while (G * LF < C) G <<= 1;
  return NW * (64 / G);
}
// a chunk covers whole 64-column mask words, so no two workgroups share a word
__host__ __device__ inline int freq_span(bool integer, int C) {
  if (freq_colpath(integer, C)) return NW * 64;
  const int cols = freq_cols(C, 1);
  return cols < 64 ? 64 : cols;
}
__host__ __device__ inline int freq_chunks(bool integer, int C, int T) {
  const int span = freq_span(integer, C);
  return (T + span - 1) / span;
}
// SIR along frequency: up to 64 channels one lane per column, 64 columns per wave
__host__ __device__ inline bool sirf_colpath(int C) { return C <= 64; }
__host__ __device__ inline int sirf_chunks(int C, int T) {
  const int span = sirf_colpath(C) ? NW * 64 : freq_span(false, C);
  return (T + span - 1) / span;
}
__host__ __device__ inline int final_chunks(int C) { return (C + NW - 1) / NW; }
// prose SIR reading: one lane per row (64 rows a wave), one wave per 64-column word
__host__ __device__ inline int prose_time_chunks(int C) { return (C + NW * 64 - 1) / (NW * 64); }
__host__ __device__ inline int prose_freq_chunks(int T) { return (((T + 63) >> 6) + NW - 1) / NW; }

struct DevParams {
  double start, p, sens, hs;
  int32_t nl_t, nl_f, eta_num, eta_den, H, Hmin, maxC, literal;
  int32_t prose;         // the range-extension reading of the SIR step
  int32_t integrated;    // integrated pre-correlation mode
  int32_t integ_tmax;    // longest block of the call (integrated mode: LDS layout)
  int32_t robust;        // stddev from the MAD
  int32_t winsor;        // history: committed means winsorized k per side (0: off)
  int32_t _pad;
  double* ring;          // [streams][maxC][H]
  int32_t* rcount;       // [streams][maxC]
  int32_t* rhead;        // [streams][maxC]
  double* pend;          // [streams][maxC]
  uint8_t* pvalid;       // [streams][maxC]
  uint64_t* maskw;       // mask scratch of this call
  uint64_t* maskw2;      // second mask buffer (prose SIR reading only)
  BlockState* bstate;    // per-block statistics of this call
  uint64_t* rowsum;      // integer input: [block sidx][maxC] power sum of each row
  void* stats;           // lof_block_stats* or null
  uint32_t* cand;        // float statistics: CAND_PER_WORD keys per mask word (null: none)
};

// float statistics: candidate keys of the last radix pass kept per mask word of
// the block (a block's list holds up to CAND_PER_WORD * C * ceil(T / 64) keys,
// about N / 8)
constexpr int CAND_PER_WORD = 8;

// ---------------------------------------------------------------- cross-lane
// DPP moves with bound_ctrl: a lane whose source is outside the wave reads 0.
// wave_shl:1 -> lane i reads lane i+1; wave_shr:1 -> lane i reads lane i-1.
__device__ __forceinline__ uint32_t shl1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ float shl1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ uint32_t shr1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ uint64_t shr1_64(uint64_t v) {
  return (uint64_t)shr1((uint32_t)v) | ((uint64_t)shr1((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ uint64_t shl1_64(uint64_t v) {
  return (uint64_t)shl1((uint32_t)v) | ((uint64_t)shl1((uint32_t)(v >> 32)) << 32);
}
// quad_perm [1,2,3,3]: lane j of a quad reads lane j+1 (lane 3 reads itself)
__device__ __forceinline__ uint64_t quad_next_64(uint64_t v) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, 0xF9, 0xf, 0xf, true);
  uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), 0xF9, 0xf, 0xf, true);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// The thread index as a value the compiler cannot move.  The phases run inside a
// work-item loop; values derived from a plain threadIdx.x would be hoisted out
// of it and held, spilled to scratch, across every item.
__device__ __forceinline__ int thread_id() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// lane q's double (q wave-uniform), read without memory
__device__ __forceinline__ double lane_double(double x, int q) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, q);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), q);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ uint64_t lowmask(int n) {
  return n <= 0 ? 0ull : (n >= 64 ? ~0ull : ((1ull << n) - 1ull));
}
__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Mask words are written with plain stores and read back by other waves of the
// same workgroup after a barrier (same CU, so the same write-through L1).
__device__ __forceinline__ uint64_t ld_mask(const GLB uint64_t* p) { return *p; }

// ---------------------------------------------------------------- power (Sec. 4)
// complex int8 sample packed in the low 16 bits of w16 (re low byte, im high
// byte, upper bytes zero): exact power re^2 + im^2 as one 4-way int8 dot product
// of the word with itself
__device__ __forceinline__ uint32_t ci8_power(uint32_t w16) {
  return (uint32_t)__builtin_amdgcn_sdot4((int)w16, (int)w16, 0, false);
}
__device__ __forceinline__ float c64_power(float re, float im) { return re * re + im * im; }
__device__ __forceinline__ float c64_amp(float re, float im) { return __builtin_sqrtf(re * re + im * im); }

// power of one sample of a float-typed block (dtype 1, 2, 3)
__device__ __forceinline__ float fpower_at(const DevBlock& b, int row, int t) {
  if (b.dtype == 2) {
    return gp<const float>(b.data)[(int64_t)row * b.dstride + t];
  }
  const f32x2 z = gp<const f32x2>(b.data)[(int64_t)row * b.dstride + t];
  return b.dtype == 1 ? c64_power(z.x, z.y) : c64_amp(z.x, z.y);
}
__device__ __forceinline__ uint32_t ipower_at(const DevBlock& b, int row, int t) {
  return ci8_power(gp<const uint16_t>(b.data)[(int64_t)row * b.dstride + t]);
}

// 8 consecutive samples of a row starting at t0 (vector loads when aligned and full)
template <bool INT>
struct TileOf;
template <>
struct TileOf<true> { typedef uint16_t T; };
template <>
struct TileOf<false> { typedef float T; };

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
    const GLB uint8_t* rb = gp<const uint8_t>(b.data) + (int64_t)row * b.dstride * 2;
    if (b.aligned && nv == 8) {
      const u32x4 q = *(const GLB u32x4*)(rb + (int64_t)t0 * 2);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[2 * j] = (typename PowT<INT>::T)ci8_power(w[j] & 0xffffu);
        v[2 * j + 1] = (typename PowT<INT>::T)ci8_power(w[j] >> 16);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        v[j] = (typename PowT<INT>::T)(j < nv ? ci8_power(*(const GLB uint16_t*)(rb + (int64_t)(t0 + j) * 2)) : 0u);
    }
  } else {
    if (b.dtype == 2) {
      const GLB float* rb = gp<const float>(b.data) + (int64_t)row * b.dstride;
      if (b.aligned && nv == 8) {
        const f32x4 a = *(const GLB f32x4*)(rb + t0);
        const f32x4 c = *(const GLB f32x4*)(rb + t0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = j < nv ? rb[t0 + j] : 0.0f;
      }
    } else {
      const GLB f32x2* rb = gp<const f32x2>(b.data) + (int64_t)row * b.dstride;
      const bool amp = b.dtype == 3;
      if (b.aligned && nv == 8) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const f32x4 a = *(const GLB f32x4*)(rb + t0 + 2 * j);
          v[2 * j] = amp ? c64_amp(a.x, a.y) : c64_power(a.x, a.y);
          v[2 * j + 1] = amp ? c64_amp(a.z, a.w) : c64_power(a.z, a.w);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float r = 0.0f;
          if (j < nv) {
            const f32x2 z = rb[t0 + j];
            r = amp ? c64_amp(z.x, z.y) : c64_power(z.x, z.y);
          }
          v[j] = r;
        }
      }
    }
  }
  return nv;
}

// 8 samples from element offset eoff (row * dstride + t0) with unconditional
// vector loads: rows 16-byte aligned and t0 + 8 <= T
template <bool INT>
__device__ __forceinline__ void load8v_off(const DevBlock& b, int64_t eoff, typename PowT<INT>::T (&v)[8]) {
  if (INT) {
    const GLB uint8_t* rb = gp<const uint8_t>(b.data) + eoff * 2;
    const u32x4 q = *(const GLB u32x4*)rb;
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[2 * j] = (typename PowT<INT>::T)ci8_power(w[j] & 0xffffu);
      v[2 * j + 1] = (typename PowT<INT>::T)ci8_power(w[j] >> 16);
    }
  } else if (b.dtype == 2) {
    const GLB float* rb = gp<const float>(b.data) + eoff;
    const f32x4 a = *(const GLB f32x4*)rb;
    const f32x4 c = *(const GLB f32x4*)(rb + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
  } else {
    const GLB f32x2* rb = gp<const f32x2>(b.data) + eoff;
    const bool amp = b.dtype == 3;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 a = *(const GLB f32x4*)(rb + 2 * j);
      v[2 * j] = amp ? c64_amp(a.x, a.y) : c64_power(a.x, a.y);
      v[2 * j + 1] = amp ? c64_amp(a.z, a.w) : c64_power(a.z, a.w);
    }
  }
}
template <bool INT>
__device__ __forceinline__ void load8v(const DevBlock& b, int row, int t0, typename PowT<INT>::T (&v)[8]) {
  load8v_off<INT>(b, (int64_t)row * b.dstride + t0, v);
}

// ---------------------------------------------------------------- shared memory
constexpr int IHIST_WORDS = 16385;   // 32769 integer-power bins, two 16-bit counters per word
constexpr int TILE_ELEMS = NW * 64 * 32;   // frequency slab: (G*32 channels) x (NW*64/G columns)
constexpr int TILE_PAD = 1024;             // one padding element per slab row (<= 1024 rows)
constexpr int TILE_WORDS = 1024;           // mask words of one frequency slab

// caller-supplied pre-flags (LOF_OPT_PREFLAGGED) of the nv <= 8 samples of a row
// from t0: bit j set when the flag byte of t0 + j is nonzero
template <bool PRE>
__device__ __forceinline__ uint32_t pre8(const DevBlock& b, int row, int t0, int nv) {
  if constexpr (!PRE) {
    return 0u;
  } else {
    const GLB uint8_t* fb = gp<const uint8_t>(b.flags) + (int64_t)row * b.fstride + t0;
    uint32_t m = 0;
    if (b.faligned && nv == 8 && (t0 & 7) == 0) {
      const uint64_t w = *(const GLB uint64_t*)fb;
#pragma unroll
      for (int j = 0; j < 8; ++j) m |= ((w >> (8 * j)) & 0xffull) ? (1u << j) : 0u;
    } else {
      for (int j = 0; j < nv; ++j) m |= fb[j] ? (1u << j) : 0u;
    }
    return m;
  }
}

// Shared memory of each kernel: only what that kernel's phase uses.
template <bool INT>
struct SmStats {
  union {
    uint32_t ihist[INT ? IHIST_WORDS : 1];   // integer input: full-resolution histogram
    uint32_t hist[2][HBINS];                 // 12-bit digit histograms (radix select)
  } u;
  double T[16];
  float Tf[16];
  double red_d[2][NW];
  unsigned long long red_u[2][NW];
  uint32_t scan[NW];
  uint32_t sel[4];
  uint32_t nlive;                            // samples not pre-flagged
  uint32_t ncand;                            // candidate keys of the last radix pass
  double median, sigma;
};

// thresholds of the block as the SumThreshold passes use them
struct SmThr {
  double T[16];
  float Tf[16];
  int32_t G[ST_MAX_LEVELS][128];   // index: window count c (<= 64); padded to any 7-bit value
};

template <bool INT>
struct SmFreq {
  typedef typename TileOf<INT>::T TileT;
  // integer slabs hold 64 columns per wave (one lane per column, up to 64
  // channels): 64 x 513 u16; float slabs the generic (G*32) x (NW*64/G + 1)
  static constexpr int TE = INT ? (64 * (NW * 64 + 1)) : (TILE_ELEMS + TILE_PAD);
  // the threshold table first: its LDS address then fits the 16-bit offset field
  // of ds_read, so a table read costs no address add
  int32_t G[ST_MAX_LEVELS][128];
  double T[16];
  float Tf[16];
  union {
    struct {
      TileT t[TE];                 // frequency slab of powers (u16 values / float)
      uint64_t w[TILE_WORDS];      // mask words of the slab
    } f;
  } u;
};

// float slabs of blocks of at most 16 channels: 16 x (NW*64 + 1) powers and the
// slab's mask words (at most 9 per channel), a third of the generic slab
struct SmFreqS {
  int32_t G[ST_MAX_LEVELS][128];
  double T[16];
  float Tf[16];
  union {
    struct {
      float t[16 * (NW * 64 + 1)];
      uint64_t w[16 * 16];
    } f;
  } u;
};

struct SmSirT {
  union {
    struct {
      int32_t seg[NW][SIR_MAX_SEGS][3];   // per-segment summaries / carries of long rows
    } c;
  } u;
};

struct SmSirF {
  union {
    struct {
      uint64_t w[TILE_WORDS];
    } f;
  } u;
};

struct SmFinal {
  uint32_t rowflag[MAXC / 32];
  unsigned long long red_u[2][NW];
};

}  // namespace lofk
