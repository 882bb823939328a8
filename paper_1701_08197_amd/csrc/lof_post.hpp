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
// flagged iff max_{b > y} W[b] >= min_{a <= y} W[a]) exploits that masks after
// SumThreshold are sparse.  A 64-position sequence (a row word, or a column of
// up to 64 channels) with no flag, or with every position flagged, has a closed
// form; only "mixed" sequences are computed position by position, with the
// whole wave on one sequence (lane = position) and wave scans for the running
// sum, its prefix minimum and its suffix maximum.  Along time a row's words are
// chained by composing each word's effect on the best interval sums crossing it
// (the lane maps of the row kernels).
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

// ---------------------------------------------------------------- wave scans
// inclusive scans over the 64 lanes in lane order (DPP row shifts, then row
// broadcasts); id is the operation's identity
template <int CTRL>
__device__ __forceinline__ int dpp_shr(int x, int id) {
  return __builtin_amdgcn_update_dpp(id, x, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ int wave_scan_add(int x) {
  x += dpp_shr<0x111>(x, 0);
  x += dpp_shr<0x112>(x, 0);
  x += dpp_shr<0x114>(x, 0);
  x += dpp_shr<0x118>(x, 0);
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
  return x;
}
__device__ __forceinline__ int wave_scan_min(int x) {
  x = min(x, dpp_shr<0x111>(x, BIG));
  x = min(x, dpp_shr<0x112>(x, BIG));
  x = min(x, dpp_shr<0x114>(x, BIG));
  x = min(x, dpp_shr<0x118>(x, BIG));
  x = min(x, __builtin_amdgcn_update_dpp(BIG, x, 0x142, 0xa, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(BIG, x, 0x143, 0xc, 0xf, false));
  return x;
}
__device__ __forceinline__ int wave_scan_max(int x) {
  x = max(x, dpp_shr<0x111>(x, -BIG));
  x = max(x, dpp_shr<0x112>(x, -BIG));
  x = max(x, dpp_shr<0x114>(x, -BIG));
  x = max(x, dpp_shr<0x118>(x, -BIG));
  x = max(x, __builtin_amdgcn_update_dpp(-BIG, x, 0x142, 0xa, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(-BIG, x, 0x143, 0xc, 0xf, false));
  return x;
}
// the value of lane 63 (wave-uniform)
__device__ __forceinline__ int wave_last(int x) { return __builtin_amdgcn_readlane(x, 63); }
// lane k's 64-bit value (k wave-uniform); each half zero-extended
__device__ __forceinline__ uint64_t lane_u64(uint64_t x, int k) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), k);
  return ((uint64_t)hi << 32) | lo;
}

// SIR of one sequence of n <= 64 positions held one per lane (lane i <->
// position i, flagged f), with alpha / beta (>= 0) the best interval sums
// ending just before position 0 / starting just after position n-1.  Returns
// the ballot of the positions the operator flags.
__device__ __forceinline__ uint64_t sir_coop(bool f, int n, int a, int c, int alpha, int beta, int lane) {
  const bool valid = lane < n;
  const int w = valid ? (f ? a : -c) : 0;
  const int Wi = wave_scan_add(w);              // running sum after position i
  const int Ei = Wi - w;                        // before position i
  const int Q = wave_last(Wi);
  const int pm = min(-alpha, wave_scan_min(valid ? Ei : BIG));
  // suffix maximum of Wi: a prefix maximum over the lanes in reverse order
  const int rev = __shfl(valid ? Wi : -BIG, 63 - lane);
  const int sx = max(Q + beta, __shfl(wave_scan_max(rev), 63 - lane));
  return __ballot(valid && sx >= pm);
}

// the map of one such sequence (alpha0 = beta0 = 0): total Q, best suffix sum
// Pf and best prefix sum Pb (both >= 0), wave-uniform
__device__ __forceinline__ void sir_coop_map(bool f, int n, int a, int c, int lane, int& Pf, int& Pb, int& Q) {
  const bool valid = lane < n;
  const int w = valid ? (f ? a : -c) : 0;
  const int Wi = wave_scan_add(w);
  const int Ei = Wi - w;
  Q = wave_last(Wi);
  const int emin = wave_last(wave_scan_min(valid ? Ei : BIG));
  const int wmax = wave_last(wave_scan_max(valid ? Wi : -BIG));
  Pf = max(0, Q - emin);
  Pb = max(0, wmax);
}

// positions of an unflagged stretch of n that alpha / beta flag (closed form of
// the linear definition: j < alpha/c, j >= n - beta/c, or everything when
// alpha + beta >= n c)
__device__ __forceinline__ uint64_t sir_empty_word(int n, int c, int alpha, int beta, const FastDiv& fc) {
  if (alpha + beta >= n * c) return lowmask(n);
  const int f = min(n, (int)fc.div((uint32_t)alpha));
  const int g = min(n, (int)fc.div((uint32_t)beta));
  return lowmask(f) | (lowmask(n) & ~lowmask(n - g));
}

// SIR along time of one row of W <= 64 words in LDS (lane = word), in place
__device__ void post_sir_row(uint64_t* row, int W, int T, int a, int c, const FastDiv& fc, int lane) {
  const int n = lane < W ? min(64, T - 64 * lane) : 0;
  const uint64_t full = lowmask(n);
  const uint64_t x = lane < W ? (row[lane] & full) : 0ull;
  const bool mixed = x != 0 && x != full;
  if (__ballot(x != 0) == 0) return;   // nothing flagged: nothing to add
  // each word's map; mixed words by the whole wave, one after the other
  int Pf = x ? a * n : 0, Pb = Pf, Q = x ? a * n : -c * n;
  uint64_t todo = __ballot(mixed);
  while (todo) {
    const int k = __builtin_ctzll(todo);
    todo &= todo - 1;
    const uint64_t xk = lane_u64(x, k);
    const int nk = __builtin_amdgcn_readlane(n, k);
    int pf, pb, q;
    sir_coop_map((xk >> lane) & 1ull, nk, a, c, lane, pf, pb, q);
    if (lane == k) {
      Pf = pf;
      Pb = pb;
      Q = q;
    }
  }
  int ain, bin;
  sir_map_scans(Pf, Pb, Q, lane, 64, ain, bin);
  // apply: full words stay, empty words by the closed form, mixed words by the wave
  uint64_t out = x;
  if (x == 0 && n > 0) out = sir_empty_word(n, c, ain, bin, fc);
  todo = __ballot(mixed);
  while (todo) {
    const int k = __builtin_ctzll(todo);
    todo &= todo - 1;
    const uint64_t xk = lane_u64(x, k);
    const int nk = __builtin_amdgcn_readlane(n, k);
    const int ak = __builtin_amdgcn_readlane(ain, k), bk = __builtin_amdgcn_readlane(bin, k);
    const uint64_t o = sir_coop((xk >> lane) & 1ull, nk, a, c, ak, bk, lane);
    if (lane == k) out = o;
  }
  if (lane < W) row[lane] = out;
}

// SIR along frequency of the 64 columns of word w (C <= 64 channels, lane =
// channel): empty and full columns are left, mixed columns are computed by the
// wave one after the other; the new flags return to the row words by a transpose
__device__ void post_sir_cols(uint64_t* m, int C, int W, int w, int T, int a, int c, int lane) {
  const uint64_t vcols = lowmask(min(64, T - 64 * w));
  const uint64_t x = lane < C ? (m[lane * W + w] & vcols) : 0ull;
  // columns with some flag, and columns flagged in every channel
  uint32_t olo = (uint32_t)x, ohi = (uint32_t)(x >> 32);
  uint32_t alo = lane < C ? (uint32_t)x : ~0u, ahi = lane < C ? (uint32_t)(x >> 32) : ~0u;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    olo |= __shfl_xor(olo, d);
    ohi |= __shfl_xor(ohi, d);
    alo &= __shfl_xor(alo, d);
    ahi &= __shfl_xor(ahi, d);
  }
  const uint64_t any = ((uint64_t)ohi << 32) | olo, all = ((uint64_t)ahi << 32) | alo;
  uint64_t todo = lane_u64(any & ~all & vcols, 0);   // the same in every lane
  if (todo == 0) return;
  // lane t collects the channels newly flagged in column t
  uint32_t elo = 0, ehi = 0;
  while (todo) {
    const int t = __builtin_ctzll(todo);
    todo &= todo - 1;
    const bool f = (x >> t) & 1ull;
    const uint64_t o = sir_coop(f, C, a, c, 0, 0, lane);
    const uint64_t col = __ballot(f);
    const uint64_t ext = o & ~col;
    if (lane == t) {
      elo = (uint32_t)ext;
      ehi = (uint32_t)(ext >> 32);
    }
  }
  const uint64_t rows = wave_transpose64(((uint64_t)ehi << 32) | elo, lane);
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
      for (int w = wv; w < W; w += NW) post_sir_cols(sm.w, C, W, w, T, a, c, lane);
      __syncthreads();
    }
  }
  // history flagger per row (one wave per row), then the flag bytes
  const int s = b.stream_id;
  if (s >= 0) {
    for (int row = wv; row < C; row += NW) {
      const int64_t idx = (int64_t)s * P.maxC + row;
      const int L = gp<const int32_t>(P.rcount)[idx];
      const int head = gp<const int32_t>(P.rhead)[idx];
      const GLB double* ring = gp<const double>(P.ring) + idx * P.H;
      const bool small_ring = P.H <= 64;
      const double xs = (small_ring && lane < P.H) ? ring[lane] : 0.0;
      const uint64_t rowsum = INT ? gp<const uint64_t>(P.rowsum)[(int64_t)b.sidx * P.maxC + row] : 0ull;
      double usum;
      int cnt;
      row_unflagged<INT>(b, (const uint64_t*)(sm.w + row * W), row, lane, rowsum, usum, cnt);
      history_judge(P, idx, L, head, ring, xs, small_ring, usum, cnt, lane, sm.rowflag, row);
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
