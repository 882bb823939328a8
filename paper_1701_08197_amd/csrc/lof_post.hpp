// lof_post.hpp -- SIR operator, history flagger and flag bytes of one block in
// one workgroup, with the block's mask in LDS (gfx950).
//
// Citations are to van Nieuwpoort, "Towards exascale real-time RFI mitigation",
// arXiv 1701.08197: SIR operator Sec. 2.2, history flagger Sec. 4.1.
//
// For blocks of at most 64 channels and 4096 times (mask words <= 4096) the
// three mask passes after SumThreshold run as one kernel per block: the mask
// words are read once into LDS, SIR runs along time and then along frequency
// there, the history flagger reads them per row, and the flag bytes are written
// from them.
//
// SIR (linear form: weights +a flagged, -c unflagged, W the running sum; y is
// flagged iff max_{b > y} W[b] >= min_{a <= y} W[a]) runs in lanes, one 64-position
// sequence (a row word, or a column of up to 64 channels) per lane: a sequence
// with no flag, or with every position flagged, has a closed form; the others are
// walked run by run.  Along time a row's words are chained by composing each
// word's effect on the best interval sums crossing it (the lane maps of the row
// kernels).
#pragma once
#include "lof_kernels.hpp"

namespace lofk {

constexpr int POST_MAX_WORDS = 4096;   // C <= 64 and T <= 4096

__host__ __device__ inline bool post_eligible(int C, int T) { return C <= 64 && T <= 64 * 64; }

struct SmPost {
  uint64_t w[POST_MAX_WORDS];          // mask words [C][W]
  uint32_t rowflag[2];                 // rows flagged by the history flagger
  unsigned long long nfl;              // flagged samples of the block
};

// positions of an unflagged stretch of n that alpha / beta flag (closed form of
// the linear definition: j < alpha/c, j >= n - beta/c, or everything when
// alpha + beta >= n c)
__device__ __forceinline__ uint64_t sir_empty_word(int n, int c, int alpha, int beta, const FastDiv& fc) {
  if (alpha + beta >= n * c) return lowmask(n);
  const int f = min(n, (int)fc.div((uint32_t)alpha));
  const int g = min(n, (int)fc.div((uint32_t)beta));
  return lowmask(f) | (lowmask(n) & ~lowmask(n - g));
}

// SIR along time of one row of W <= 64 words in LDS (lane = word), in place.
// Each word's effect on the best interval sums crossing it is composed along
// the row (lane maps); a word with no flag, or flagged throughout, has a closed
// form, the others are walked run by run in their lane.
__device__ __forceinline__ void post_sir_row(uint64_t* row, int W, int T, int a, int c, const FastDiv& fc, int lane) {
  const int n = lane < W ? min(64, T - 64 * lane) : 0;
  const uint64_t full = lowmask(n);
  const uint64_t x = lane < W ? (row[lane] & full) : 0ull;
  if (__ballot(x != 0) == 0) return;   // nothing flagged: nothing to add
  const bool mixed = x != 0 && x != full;
  int Pf = x ? a * n : 0, Pb = Pf, Q = x ? a * n : -c * n;
  if (mixed) sir_lane_maps(x, n, a, c, Pf, Pb, Q);
  int ain, bin;
  sir_map_scans(Pf, Pb, Q, lane, 64, ain, bin);
  uint64_t out = x;
  if (x == 0 && n > 0) out = sir_empty_word(n, c, ain, bin, fc);
  if (mixed) out = sir_runs_lane(x, n, a, c, fc, ain, bin);
  if (lane < W) row[lane] = out;
}

// SIR along frequency of the 64 columns of word w (C <= 64 channels): lane c
// reads channel c's word, a bit transpose gives each lane its column, the column
// is walked run by run in the lane (columns with no flag, or flagged throughout,
// are left), and the new flags go back by a transpose
__device__ __forceinline__ void post_sir_cols(uint64_t* m, int C, int W, int w, int T, int a, int c, const FastDiv& fc,
                              int lane) {
  const uint64_t vcols = lowmask(min(64, T - 64 * w));
  const uint64_t x = lane < C ? (m[lane * W + w] & vcols) : 0ull;
  if (__ballot(x != 0) == 0) return;
  // the transpose takes every lane (it shuffles across the wave); columns past
  // the block's end are cleared afterwards
  const uint64_t tr = wave_transpose64(x, lane);
  const bool ok = (vcols >> lane) & 1ull;
  const uint64_t col = ok ? (tr & lowmask(C)) : 0ull;
  const bool mixed = col != 0 && col != lowmask(C);
  uint64_t ext = 0;
  if (mixed) ext = sir_runs_lane(col, C, a, c, fc) & ~col;
  if (__ballot(ext != 0) == 0) return;
  const uint64_t rows = wave_transpose64(ext, lane);   // every lane, as above
  if (lane < C && rows) m[lane * W + w] = x | rows;
}

template <bool INT>
__device__ __forceinline__ void phase_post(const DevBlock& b, const DevParams& P, SmPost& sm) {
  const int tid = thread_id(), lane = tid & 63, wv = tid >> 6;
  const int C = b.C, T = b.T, W = (T + 63) >> 6;
  GLB uint64_t* m0 = gp<uint64_t>(P.maskw) + b.mask_off;
  for (int i = tid; i < C * W; i += WG) sm.w[i] = m0[i];
  if (tid < 2) sm.rowflag[tid] = 0u;
  if (tid == 0) sm.nfl = 0ull;
  __syncthreads();
  const int num = P.eta_num, den = P.eta_den;
  if (num > 0 && num >= den) {
    // eta = 1: every interval qualifies, every position is flagged
    for (int i = tid; i < C * W; i += WG) sm.w[i] = lowmask(min(64, T - 64 * (i % W)));
    __syncthreads();
  } else if (num > 0) {
    const int a = num, c = den - num;
    const FastDiv fc((uint32_t)c);
    for (int row = wv; row < C; row += NW) post_sir_row(sm.w + row * W, W, T, a, c, fc, lane);
    __syncthreads();
    if (C > 1) {
      for (int w = wv; w < W; w += NW) post_sir_cols(sm.w, C, W, w, T, a, c, fc, lane);
      __syncthreads();
    }
  }
  // history flagger per row (one wave per row), then the flag bytes
  const int s = b.stream_id;
  if (s >= 0) {
    // a wave's rows in turn; the next row's ring count, head, ring and row sum
    // are loaded while the current row is judged
    const bool small_ring = P.H <= 64;
    auto fetch = [&](int row, int& L, int& head, double& xs, uint64_t& rs) {
      const int64_t idx = (int64_t)s * P.maxC + row;
      L = gp<const int32_t>(P.rcount)[idx];
      head = gp<const int32_t>(P.rhead)[idx];
      xs = (small_ring && lane < P.H) ? gp<const double>(P.ring)[idx * P.H + lane] : 0.0;
      rs = INT ? gp<const uint64_t>(P.rowsum)[(int64_t)b.sidx * P.maxC + row] : 0ull;
    };
    int L = 0, head = 0;
    double xs = 0.0;
    uint64_t rowsum = 0;
    if (wv < C) fetch(wv, L, head, xs, rowsum);
    for (int row = wv; row < C; row += NW) {
      int L2 = 0, head2 = 0;
      double xs2 = 0.0;
      uint64_t rs2 = 0;
      if (row + NW < C) fetch(row + NW, L2, head2, xs2, rs2);
      const int64_t idx = (int64_t)s * P.maxC + row;
      const GLB double* ring = gp<const double>(P.ring) + idx * P.H;
      double usum;
      int cnt;
      row_unflagged<INT>(b, (const uint64_t*)(sm.w + row * W), row, lane, rowsum, usum, cnt);
      history_judge(P, idx, L, head, ring, xs, small_ring, usum, cnt, lane, sm.rowflag, row);
      L = L2;
      head = head2;
      xs = xs2;
      rowsum = rs2;
    }
    __syncthreads();
  }
  unsigned long long nfl = 0;
  for (int i = tid; i < C * W; i += WG) {
    const int row = i / W, w = i - row * W;
    const int nv = min(64, T - 64 * w);
    uint64_t fw = sm.w[i] & lowmask(nv);
    if ((sm.rowflag[row >> 5] >> (row & 31)) & 1u) fw = lowmask(nv);
    nfl += (unsigned long long)__popcll(fw);
    write_word_bytes(b, row, 64 * w, nv, fw);
  }
  if (!P.stats) return;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) nfl += __shfl_xor(nfl, d);
  char* st = (char*)P.stats + (int64_t)b.out_idx * STATS_BYTES;
  if (lane == 0 && nfl) atomicAdd((unsigned long long*)(st + STATS_NFLAG), nfl);
  if (tid == 0 && s >= 0) {
    const int hr = __popc(sm.rowflag[0]) + __popc(sm.rowflag[1]);
    if (hr) atomicAdd((int*)(st + STATS_HROWS), hr);
  }
}

}  // namespace lofk
