// lof_partial.hpp -- 2-D flagging with partial integration (gfx950).
//
// Method: van Nieuwpoort, "Towards exascale real-time RFI mitigation", arXiv
// 1701.08197, Sec. 4 (integration paragraph: the alternative to full
// integration, 2-D flagging on data partially integrated in one or both
// dimensions).
//
// Each block is integrated into tiles of ff channels x ft times (tiles at the
// block's end hold fewer samples): a tile's value is the sum of its powers over
// its sample count, rounded once to float32 (integer input: an exact integer sum
// divided in float64).  The whole path then runs on the grid of tile means as
// float32 input, writing one flag byte per tile, and the spread kernel gives
// every sample of the block its tile's flag.
//
// Integration kernel: a work item is one row of tiles and a segment of up to
// PART_SEG times holding whole tiles.  Each thread adds 8 consecutive times over
// the tile's channels (vector loads, one 1 KB span per wave instruction for
// complex int8) into column sums in LDS; then each tile's columns are added, by
// one thread (ft <= 64) or by one wave (ft > 64).
#pragma once
#include "lof_kernels.hpp"

namespace lofk {

constexpr int PART_SEG = 4096;        // times per integration work item (whole tiles)
constexpr int PART_MAX_TIME = 4096;   // largest tile along time

// one block of a partial-integration call: the caller's block and its grid of
// tile means (float32 [Cc][cstride]) and tile flags (bytes [Cc][cstride])
struct PartialBlock {
  DevBlock fine;
  float* coarse;
  uint8_t* cflags;
  int64_t cstride;
  int32_t Cc, Tc;      // tiles along frequency and time
  int32_t ff, ft;      // channels and times per tile
};

__host__ __device__ inline int part_tiles_per_seg(int ft) { return ft >= PART_SEG ? 1 : PART_SEG / ft; }
__host__ __device__ inline int part_items(int Cc, int Tc, int ft) {
  const int k = part_tiles_per_seg(ft);
  return Cc * ((Tc + k - 1) / k);
}
__host__ __device__ inline int part_spread_chunks(int C) { return (C + NW - 1) / NW; }

template <bool INT>
struct PartSum;
template <>
struct PartSum<true> { typedef uint64_t T; };
template <>
struct PartSum<false> { typedef double T; };

template <bool INT>
struct SmPartial {
  typename PartSum<INT>::T col[PART_SEG];
};

// tile means of one (row of tiles, segment) work item
template <bool INT>
__device__ __forceinline__ void phase_partial_integrate(const PartialBlock& pb, int item, SmPartial<INT>& sm) {
  typedef typename PartSum<INT>::T ST;
  typedef typename PowT<INT>::T VT;
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const DevBlock& b = pb.fine;
  const int k = part_tiles_per_seg(pb.ft);
  const int nseg = (pb.Tc + k - 1) / k;
  const int ti = item / nseg, seg = item - ti * nseg;
  const int r0 = ti * pb.ff, r1 = min(b.C, r0 + pb.ff);
  const int j0 = seg * k, j1 = min(pb.Tc, j0 + k);       // tiles of this item
  const int t0 = j0 * pb.ft, t1 = min(b.T, j1 * pb.ft);  // its times
  const int span = t1 - t0;
  // column sums over the tile's channels, 8 consecutive times per thread
  for (int x = 8 * tid; x < span; x += 8 * WG) {
    ST acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0;
    const int t = t0 + x;
    const bool full = t + 8 <= t1 && b.aligned && (t & 7) == 0;
    for (int r = r0; r < r1; ++r) {
      VT v[8];
      if (full) {
        load8v<INT>(b, r, t, v);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (INT) v[q] = (VT)(t + q < t1 ? ipower_at(b, r, t + q) : 0u);
          else v[q] = (VT)(t + q < t1 ? fpower_at(b, r, t + q) : 0.0f);
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += (ST)v[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (x + q < span) sm.col[x + q] = acc[q];
  }
  __syncthreads();
  const int ntile = j1 - j0;
  const double rows = (double)(r1 - r0);
  GLB float* out = gp<float>(pb.coarse) + (int64_t)ti * pb.cstride;
  if (pb.ft <= 64) {
    for (int j = tid; j < ntile; j += WG) {
      const int a = j * pb.ft, e = min(span, a + pb.ft);
      ST s = 0;
      for (int x = a; x < e; ++x) s += sm.col[x];
      out[j0 + j] = (float)((double)s / (rows * (double)(e - a)));
    }
  } else {
    for (int j = wv; j < ntile; j += NW) {
      const int a = j * pb.ft, e = min(span, a + pb.ft);
      ST s = 0;
      for (int x = a + lane; x < e; x += 64) s += sm.col[x];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
      if (lane == 0) out[j0 + j] = (float)((double)s / (rows * (double)(e - a)));
    }
  }
  __syncthreads();
}

// flag bytes of the caller's rows from the tile flags (one wave per row), the
// block's flagged-sample count, and the grid's statistics copied to the caller
__device__ __forceinline__ void phase_partial_spread(const PartialBlock& pb, int chunk, int out_idx,
                                                     const lof_block_stats* cstats, lof_block_stats* stats) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const DevBlock& b = pb.fine;
  const FastDiv fdt((uint32_t)pb.ft);
  const FastDiv fdf((uint32_t)pb.ff);
  const int row = chunk * NW + wv;
  unsigned long long nfl = 0;
  if (row < b.C) {
    const GLB uint8_t* cf = gp<const uint8_t>(pb.cflags) + (int64_t)fdf.div((uint32_t)row) * pb.cstride;
    GLB uint8_t* f = gp<uint8_t>(b.flags) + (int64_t)row * b.fstride;
    for (int t = 16 * lane; t < b.T; t += 16 * 64) {
      uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const uint32_t v = (t + q < b.T) ? (uint32_t)(cf[fdt.div((uint32_t)(t + q))] != 0) : 0u;
        w[q >> 2] |= v << (8 * (q & 3));
      }
      nfl += (unsigned long long)(__popc(w[0]) + __popc(w[1]) + __popc(w[2]) + __popc(w[3]));
      if (b.faligned && t + 16 <= b.T) {
        u32x4 o;
        o.x = w[0];
        o.y = w[1];
        o.z = w[2];
        o.w = w[3];
        *(GLB u32x4*)(f + t) = o;
      } else {
        for (int q = 0; q < 16 && t + q < b.T; ++q) f[t + q] = (uint8_t)((w[q >> 2] >> (8 * (q & 3))) & 0xffu);
      }
    }
  }
  if (!stats) return;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) nfl += __shfl_xor(nfl, d);
  char* st = (char*)stats + (int64_t)out_idx * STATS_BYTES;
  if (lane == 0 && nfl) atomicAdd((unsigned long long*)(st + STATS_NFLAG), nfl);
  if (chunk == 0) {
    const char* cs = (const char*)cstats + (int64_t)out_idx * STATS_BYTES;
    if (tid < 2 + LOF_MAX_LEVELS) ((double*)st)[tid] = ((const double*)cs)[tid];
    if (tid == 0) *(int32_t*)(st + STATS_HROWS) = *(const int32_t*)(cs + STATS_HROWS);
  }
}

}  // namespace lofk
