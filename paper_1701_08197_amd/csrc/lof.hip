// lof.hip -- host side of the C ABI declared in include/lof.h, and the kernel
// instantiations.  Method: van Nieuwpoort, "Towards exascale real-time RFI
// mitigation", arXiv 1701.08197 (SumThreshold Sec. 2.1, SIR Sec. 2.2, history
// flagger Sec. 4.1; one independent block per station, polarisation and subband,
// Sec. 4.1 domain decomposition).
//
// The host validates every block (all-or-nothing), groups blocks by input kind
// and by the time layout their length needs, orders each group by decreasing
// size so the largest blocks start first, uploads one descriptor table and
// launches one kernel per phase on the caller's stream: statistics per block,
// then SumThreshold time / frequency, SIR time / frequency and the history + flag
// write, each over (block, chunk) work items.  No allocation happens after
// lof_create: descriptor tables, per-block statistics and mask scratch live in a
// small ring of slots, each slot guarded by an event so that calls on different
// streams can overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lof.h"
#include "lof_kernel_table.hpp"
#include "lof_integrated.hpp"
#include "lof_partial.hpp"
#include "lof_post.hpp"
#include "lof_stats_split.hpp"
#include "lof_kernels.hpp"

namespace lofk {
// zero a few device ints (work counters) without a memset node
__global__ void lof_zero_kernel(int* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Commit staged history values (Sec. 4.1 addToHistory) of a list of streams.
__global__ void lof_commit_kernel(IdList ids, int all_streams, DevParams P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nsel = all_streams ? (int64_t)all_streams : (int64_t)ids.n;
  if (i >= nsel * P.maxC) return;
  const int si = (int)(i / P.maxC), c = (int)(i - (int64_t)si * P.maxC);
  const int s = all_streams ? si : ids.ids[si];
  const int64_t idx = (int64_t)s * P.maxC + c;
  if (!P.pvalid[idx]) return;
  const int h = P.rhead[idx];
  P.ring[idx * P.H + h] = P.pend[idx];
  P.rhead[idx] = (h + 1 == P.H) ? 0 : h + 1;
  const int n = P.rcount[idx];
  P.rcount[idx] = n < P.H ? n + 1 : P.H;
  P.pvalid[idx] = 0;
}

// commit for the streams of a descriptor table (automatic commit)
__global__ void lof_commit_desc_kernel(const DevBlock* __restrict__ blocks, int nb, DevParams P) {
  const int bi = blockIdx.x;
  if (bi >= nb) return;
  const int s = blocks[bi].stream_id;
  if (s < 0) return;
  for (int c = threadIdx.x; c < P.maxC; c += blockDim.x) {
    const int64_t idx = (int64_t)s * P.maxC + c;
    if (!P.pvalid[idx]) continue;
    const int h = P.rhead[idx];
    P.ring[idx * P.H + h] = P.pend[idx];
    P.rhead[idx] = (h + 1 == P.H) ? 0 : h + 1;
    const int n = P.rcount[idx];
    P.rcount[idx] = n < P.H ? n + 1 : P.H;
    P.pvalid[idx] = 0;
  }
}

// Allocation-free entry point (lof_flag_blocks_static): the per-call scratch of
// the phase kernels (descriptor table, per-block statistics, integer row sums,
// mask words) lives in this one file-scope array, one copy per GPU, held until
// the process ends.  Host code uses its device address from hipGetSymbolAddress.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

// descriptors travel as kernel arguments (no host staging buffer, no copy)
constexpr int DESC_CHUNK = 32;
struct DescChunk {
  int32_t n, first;
  DevBlock d[DESC_CHUNK];
};
__global__ void lof_put_desc_kernel(DevBlock* dst, DescChunk ch) {
  const int i = (int)threadIdx.x;
  if (i < ch.n) dst[ch.first + i] = ch.d[i];
}
}  // namespace lofk

using lofk::BlockState;
using lofk::DevBlock;
using lofk::DevParams;

namespace {

constexpr int NSLOT = 4;            // call slots when lof_params.call_slots is 0
constexpr int MAX_SLOTS = 65536;
constexpr int MAX_TIMES = lofk::SIR_SEG * lofk::SIR_MAX_SEGS;   // 262144

thread_local const char* g_create_err = "no error";

constexpr int NCOUNTER = 32;      // persistent-launch work counters per call (<= 20 launches)
constexpr int NTEV = NCOUNTER + 1;   // phase-timing events per call

struct Slot {
  int ncx = 0;                    // blocks of complex float input at the head of the 32-lane float group
  DevBlock* d_desc = nullptr;
  DevBlock* h_desc = nullptr;     // pinned
  uint64_t* d_mask = nullptr;
  uint64_t* d_mask2 = nullptr;    // second mask buffer (LOF_OPT_SIR_PROSE only)
  BlockState* d_state = nullptr;
  uint64_t* d_rowsum = nullptr;   // integer rows' power sums [block][max_channels]
  int* d_counter = nullptr;       // persistent-launch work counters, one per launch
  uint32_t* d_cand = nullptr;     // float statistics: candidate keys, CAND_PER_WORD per mask word
  lofk::SplitState* d_split = nullptr;   // split statistics of up to nsplit float blocks
  int nsplit = 0;
  hipEvent_t ev = nullptr;
  bool used = false;
  // LOF_OPT_PHASE_TIMING: event 0 before the first phase kernel, event k after
  // launch k, whose phase is tph[k]
  hipEvent_t tev[NTEV] = {};
  int tph[NTEV] = {};
  int ntev = 0;
  bool timed = false;             // events of a call not yet added to the totals
};

// partial integration (lof_params.partial_time / partial_freq): per call slot, the
// grid of tile means and tile flags of every block, their descriptor tables and
// the statistics of the grids
struct PSlot {
  Slot s;                                  // the grids' call: descriptor table and scratch
  lofk::PartialBlock* d_part = nullptr;    // per caller block: block and its grid
  lofk::PartialBlock* h_part = nullptr;    // pinned
  float* d_coarse = nullptr;
  uint8_t* d_cflags = nullptr;
  lof_block_stats* d_cstats = nullptr;
};

int time_bucket(int T) { return T <= 1024 ? 0 : (T <= 2048 ? 1 : (T <= 3072 ? 2 : (T <= 4096 ? 3 : 4))); }
int lanes_index(int L) { return L == 32 ? 0 : (L == 48 ? 1 : 2); }
bool lanes_allowed(int L, int bucket) {
  static const int maxT[LOF_TUNE_BUCKETS] = {1024, 2048, 3072, 4096, 1 << 30};
  if (L != 32 && L != 48 && L != 64) return false;
  return L == 64 || 64 * L >= maxT[bucket];
}
constexpr int NVAR = 6;   // time layouts: (integer, float) x (32, 48, 64 lanes)

// kernels, for occupancy lookups
enum KernId {
  K_STATS = 0, K_TIME = 2, K_FREQ = 8, K_SIRT = 10, K_SIRF = 13, K_FINAL = 14, K_PROSE = 16, K_INTEG = 18, K_POST = 20,
  K_STATS_PRE = 22, K_TIME_PRE = 24, K_TIMECX = 30, K_SPLIT = 31, K_FREQS = 33, NKERN = 34
};
int variant_lanes(int v) { return v % 3 == 0 ? 32 : (v % 3 == 1 ? 48 : 64); }

size_t elem_size(int dtype) { return dtype == LOF_CI8 ? 2 : (dtype == LOF_F32 ? 4 : 8); }

}  // namespace

struct lof_ctx {
  lof_params prm;
  int dev = 0;
  double* ring = nullptr;
  int32_t* rcount = nullptr;
  int32_t* rhead = nullptr;
  double* pend = nullptr;
  uint8_t* pvalid = nullptr;
  std::vector<Slot> slot;         // call slots (descriptor table, scratch, event), used in turn
  int next = 0;
  lof_tuning tune;
  int occ[NKERN] = {};   // resident workgroups per CU of each kernel
  int n_cu = 0;
  // hipGraph cache (LOF_OPT_GRAPH): the last block table, its graph and its slot
  Slot gslot;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<lof_block> gsig;
  void* gstats = nullptr;
  bool gvalid = false;
  size_t mask_words = 0;
  std::vector<int32_t> seen;     // per stream: last call that named it
  int32_t call_no = 0;
  std::vector<DevBlock> tmp;
  std::vector<int> order;
  double phase_ms[LOF_N_PHASES] = {};   // LOF_OPT_PHASE_TIMING totals since the last read
  // partial integration: tile shape, grid capacity per call, slots, grid blocks
  bool partial = false;
  int pt = 1, pf = 1;
  size_t coarse_cap = 0;
  std::vector<PSlot> pslot;
  std::vector<lof_block> ctmp;
  int32_t phase_calls = 0;
  const char* err = "no error";
};

namespace {

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != d) (void)hipSetDevice(d);
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

DevParams dev_params(const lof_ctx* c, uint64_t* mask, uint64_t* mask2, BlockState* state, uint64_t* rowsum,
                     void* stats) {
  DevParams P;
  P.start = c->prm.start_threshold;
  P.p = c->prm.p;
  P.sens = c->prm.sensitivity;
  P.hs = c->prm.history_sensitivity;
  P.nl_t = c->prm.n_levels;
  P.nl_f = c->prm.n_levels_freq < 0 ? c->prm.n_levels : c->prm.n_levels_freq;
  P.eta_num = c->prm.sir_eta_num;
  P.eta_den = c->prm.sir_eta_den;
  P.H = c->prm.history_len;
  P.Hmin = c->prm.history_min;
  P.maxC = c->prm.max_channels;
  P.literal = (c->prm.options & LOF_OPT_LITERAL_HISTORY_TIE) ? 1 : 0;
  P.prose = (c->prm.options & LOF_OPT_SIR_PROSE) ? 1 : 0;
  P.integrated = (c->prm.options & LOF_OPT_INTEGRATED) ? 1 : 0;
  P.integ_tmax = 0;
  P.robust = (c->prm.options & LOF_OPT_ROBUST_SIGMA) ? 1 : 0;
  P.winsor = c->prm.history_winsor;
  P._pad = 0;
  P.ring = c->ring;
  P.rcount = c->rcount;
  P.rhead = c->rhead;
  P.pend = c->pend;
  P.pvalid = c->pvalid;
  P.maskw = mask;
  P.maskw2 = mask2;
  P.bstate = state;
  P.rowsum = rowsum;
  P.stats = stats;
  P.cand = nullptr;
  return P;
}

const char* check_params(const lof_params* p) {
  if (!p) return "params is NULL";
  if (!(p->start_threshold == p->start_threshold) || !(p->p == p->p) || !(p->sensitivity == p->sensitivity) ||
      !(p->history_sensitivity == p->history_sensitivity))
    return "NaN parameter";
  if (p->n_levels < 1 || p->n_levels > lofk::ST_MAX_LEVELS) return "n_levels must be in 1..7 (windows up to 64)";
  if (p->n_levels_freq < -1 || p->n_levels_freq > lofk::ST_MAX_LEVELS) return "n_levels_freq must be -1 or 0..7";
  if (p->sir_eta_den < 1 || p->sir_eta_den > 1024 || p->sir_eta_num < 0 || p->sir_eta_num > p->sir_eta_den)
    return "SIR eta must be num/den with 0 <= num <= den <= 1024";
  if (p->history_len < 1 || p->history_len > 4096) return "history_len must be in 1..4096";
  if (p->history_min < 0) return "history_min must be >= 0";
  if (p->history_winsor < 0 || (p->history_winsor > 0 && p->history_len > 64))
    return "history_winsor must be >= 0, and 0 unless history_len <= 64";
  if (p->max_streams < 1) return "max_streams must be >= 1";
  if (p->max_channels < 1 || p->max_channels > LOF_MAX_CHANNELS) return "max_channels must be in 1..1024";
  if (p->max_blocks_per_call < 1) return "max_blocks_per_call must be >= 1";
  if (p->max_samples_per_call < 1) return "max_samples_per_call must be >= 1";
  if (p->call_slots < 0 || p->call_slots > MAX_SLOTS) return "call_slots must be in 0..65536";
  if (p->partial_time < 0 || p->partial_time > lofk::PART_MAX_TIME) return "partial_time must be in 0..4096";
  if (p->partial_freq < 0 || p->partial_freq > LOF_MAX_CHANNELS) return "partial_freq must be in 0..1024";
  if ((p->partial_time > 1 || p->partial_freq > 1) &&
      (p->options & (LOF_OPT_INTEGRATED | LOF_OPT_GRAPH | LOF_OPT_PREFLAGGED)))
    return "partial integration does not combine with LOF_OPT_INTEGRATED, LOF_OPT_GRAPH or LOF_OPT_PREFLAGGED";
  if ((p->options & LOF_OPT_PREFLAGGED) && (p->options & LOF_OPT_INTEGRATED))
    return "LOF_OPT_PREFLAGGED does not combine with LOF_OPT_INTEGRATED";
  return nullptr;
}

lof_status fail(lof_ctx* c, lof_status s, const char* msg) {
  if (c) c->err = msg;
  return s;
}

}  // namespace


namespace {

const void* kernel_of(int k) {
  if (k == K_STATS || k == K_STATS + 1) return lofk::kernel_stats(k == K_STATS);
  if (k >= K_TIME && k < K_TIME + 6) return lofk::kernel_time(k < K_TIME + 3, variant_lanes(k - K_TIME));
  if (k == K_FREQ || k == K_FREQ + 1) return lofk::kernel_freq(k == K_FREQ);
  if (k >= K_SIRT && k < K_SIRT + 3) return lofk::kernel_sir_time(variant_lanes(k - K_SIRT));
  if (k == K_SIRF) return lofk::kernel_sir_freq();
  if (k == K_PROSE || k == K_PROSE + 1) return lofk::kernel_prose(k == K_PROSE + 1);
  if (k == K_INTEG || k == K_INTEG + 1) return lofk::kernel_integrated(k == K_INTEG);
  if (k == K_POST || k == K_POST + 1) return lofk::kernel_post(k == K_POST);
  if (k == K_STATS_PRE || k == K_STATS_PRE + 1) return lofk::kernel_stats_pre(k == K_STATS_PRE);
  if (k >= K_TIME_PRE && k < K_TIME_PRE + 6)
    return lofk::kernel_time_pre(k < K_TIME_PRE + 3, variant_lanes(k - K_TIME_PRE));
  if (k == K_TIMECX) return lofk::kernel_time_cx();
  if (k == K_FREQS) return lofk::kernel_freq_small();
  if (k == K_SPLIT || k == K_SPLIT + 1) return lofk::kernel_stats_split(k == K_SPLIT + 1);
  return lofk::kernel_final(k == K_FINAL);
}

void free_slot(Slot& s) {
  if (s.d_desc) (void)hipFree(s.d_desc);
  if (s.h_desc) (void)hipHostFree(s.h_desc);
  if (s.d_mask) (void)hipFree(s.d_mask);
  if (s.d_mask2) (void)hipFree(s.d_mask2);
  if (s.d_state) (void)hipFree(s.d_state);
  if (s.d_rowsum) (void)hipFree(s.d_rowsum);
  if (s.d_counter) (void)hipFree(s.d_counter);
  if (s.d_split) (void)hipFree(s.d_split);
  if (s.d_cand) (void)hipFree(s.d_cand);
  if (s.ev) (void)hipEventDestroy(s.ev);
  for (hipEvent_t& e : s.tev)
    if (e) (void)hipEventDestroy(e);
  s = Slot();
}

void free_pslot(PSlot& p) {
  free_slot(p.s);
  if (p.d_part) (void)hipFree(p.d_part);
  if (p.h_part) (void)hipHostFree(p.h_part);
  if (p.d_coarse) (void)hipFree(p.d_coarse);
  if (p.d_cflags) (void)hipFree(p.d_cflags);
  if (p.d_cstats) (void)hipFree(p.d_cstats);
  p = PSlot();
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }
int64_t round16(int64_t x) { return (x + 15) & ~(int64_t)15; }

bool alloc_slot(Slot& s, int max_blocks, int max_channels, size_t mask_words, bool timing, bool prose) {
  if (timing)
    for (hipEvent_t& e : s.tev)
      if (hipEventCreate(&e) != hipSuccess) return false;
  if (prose && hipMalloc(&s.d_mask2, sizeof(uint64_t) * mask_words) != hipSuccess) return false;
  // split statistics: their histograms and pass counters start at zero, and each
  // call leaves them so
  s.nsplit = std::min(max_blocks, lofk::SPLIT_MAX_BLOCKS);
  const size_t split_bytes = sizeof(lofk::SplitState) * (size_t)s.nsplit;
  if (hipMalloc(&s.d_split, split_bytes) != hipSuccess || hipMemset(s.d_split, 0, split_bytes) != hipSuccess)
    return false;
  if (hipMalloc(&s.d_cand, sizeof(uint32_t) * lofk::CAND_PER_WORD * mask_words) != hipSuccess) return false;
  return hipMalloc(&s.d_desc, sizeof(DevBlock) * max_blocks) == hipSuccess &&
         hipHostMalloc(&s.h_desc, sizeof(DevBlock) * max_blocks, hipHostMallocDefault) == hipSuccess &&
         hipMalloc(&s.d_mask, sizeof(uint64_t) * mask_words) == hipSuccess &&
         hipMalloc(&s.d_state, sizeof(BlockState) * max_blocks) == hipSuccess &&
         hipMalloc(&s.d_rowsum, sizeof(uint64_t) * (size_t)max_blocks * (size_t)max_channels) == hipSuccess &&
         hipMalloc(&s.d_counter, sizeof(int) * NCOUNTER) == hipSuccess &&
         hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) == hipSuccess;
}

void default_tuning(lof_tuning* t) {
  std::memset(t, 0, sizeof(*t));
  for (int k = 0; k < 2; ++k) {
    t->time_lanes[k][0] = 32;
    t->time_lanes[k][1] = 32;
    t->time_lanes[k][2] = 48;
    t->time_lanes[k][3] = 64;
    t->time_lanes[k][4] = 64;
  }
  t->persistent = 0;
}

bool tuning_ok(const lof_tuning* t) {
  if (!t || (t->persistent != 0 && t->persistent != 1) || t->fuse_post < 0 || t->fuse_post > 2) return false;
  for (int k = 0; k < 2; ++k)
    for (int b = 0; b < LOF_TUNE_BUCKETS; ++b)
      if (!lanes_allowed(t->time_lanes[k][b], b)) return false;
  return true;
}

int variant_of(const lof_tuning& t, const lof_block& b) {
  const int kind = b.dtype == LOF_CI8 ? 0 : 1;
  return kind * 3 + lanes_index(t.time_lanes[kind][time_bucket(b.n_times)]);
}

// shape, stride, dtype and stream-id range of one block; nullptr when valid
const char* check_block(const lof_block& b, int max_channels, int max_streams, lof_status* code) {
  *code = LOF_ERR_INVALID;
  if (!b.data || !b.flags) return "block data or flags pointer is NULL";
  if (b.n_channels < 1 || b.n_times < 1) return "block shape must be >= 1 x 1";
  if (b.n_channels > LOF_MAX_CHANNELS) return "more than 1024 channels";
  if (b.n_times > MAX_TIMES) return "more than 262144 times";
  if ((int64_t)b.n_channels * b.n_times > LOF_MAX_BLOCK_SAMPLES) return "block larger than 2^23 samples";
  if (b.data_row_stride < b.n_times || b.flag_row_stride < b.n_times) return "row stride smaller than n_times";
  if (b.dtype < LOF_CI8 || b.dtype > LOF_C64_AMP) return "unknown dtype";
  if (b.stream_id < -1 || b.stream_id >= max_streams) return "stream_id out of range";
  if (b.n_channels > max_channels) {
    *code = LOF_ERR_CAPACITY;
    return "n_channels > max_channels";
  }
  return nullptr;
}

size_t block_mask_words(const lof_block& b) { return (size_t)b.n_channels * (size_t)((b.n_times + 63) / 64); }

// validation of one call (all-or-nothing)
lof_status validate(lof_ctx* c, const lof_block* blocks, int32_t n, bool check_ids) {
  if (n > c->prm.max_blocks_per_call) return fail(c, LOF_ERR_CAPACITY, "more blocks than max_blocks_per_call");
  c->call_no++;
  if (c->call_no == 0x7fffffff) {
    std::fill(c->seen.begin(), c->seen.end(), -1);
    c->call_no = 1;
  }
  int64_t samples = 0;
  size_t words = 0;
  for (int i = 0; i < n; ++i) {
    const lof_block& b = blocks[i];
    lof_status code;
    if (const char* m = check_block(b, c->prm.max_channels, c->prm.max_streams, &code)) return fail(c, code, m);
    if (check_ids && b.stream_id >= 0) {
      if (c->seen[b.stream_id] == c->call_no) return fail(c, LOF_ERR_INVALID, "stream_id repeated in one call");
      c->seen[b.stream_id] = c->call_no;
    }
    samples += (int64_t)b.n_channels * b.n_times;
    words += block_mask_words(b);
  }
  if (samples > c->prm.max_samples_per_call)
    return fail(c, LOF_ERR_CAPACITY, "more samples than max_samples_per_call");
  if (c->prm.options & LOF_OPT_INTEGRATED)
    for (int i = 0; i < n; ++i)
      if (blocks[i].n_times > lofk::INTEG_MAX_T) return fail(c, LOF_ERR_INVALID, "integrated mode: n_times > 16384");
  if (words > c->mask_words) return fail(c, LOF_ERR_CAPACITY, "mask scratch too small");
  if (c->partial) {
    size_t cells = 0;
    for (int i = 0; i < n; ++i)
      cells += (size_t)ceil_div(blocks[i].n_channels, c->pf) * (size_t)round16(ceil_div(blocks[i].n_times, c->pt));
    if (cells > c->coarse_cap) return fail(c, LOF_ERR_CAPACITY, "partial integration: tile grids too large");
  }
  return LOF_OK;
}

// descriptor table in s.h_desc: variant groups, largest block first; counts[v]
void build_table(int* order, const lof_tuning& t, const lof_block* blocks, int32_t n, Slot& s, int* counts,
                 bool history) {
  for (int i = 0; i < n; ++i) order[i] = i;
  // within a variant, float blocks of complex input first (their 32-lane time
  // kernel keeps the formed powers), then by decreasing size
  auto cx = [&](const lof_block& b) { return b.dtype == LOF_C64 || b.dtype == LOF_C64_AMP; };
  std::sort(order, order + n, [&](int a, int bb) {
    const int va = variant_of(t, blocks[a]), vb = variant_of(t, blocks[bb]);
    if (va != vb) return va < vb;
    if (cx(blocks[a]) != cx(blocks[bb])) return cx(blocks[a]);
    const int64_t sa = (int64_t)blocks[a].n_channels * blocks[a].n_times;
    const int64_t sb = (int64_t)blocks[bb].n_channels * blocks[bb].n_times;
    if (sa != sb) return sa > sb;
    return a < bb;
  });
  int64_t moff = 0;
  for (int v = 0; v < NVAR; ++v) counts[v] = 0;
  for (int j = 0; j < n; ++j) {
    const int i = order[j];
    const lof_block& b = blocks[i];
    DevBlock& d = s.h_desc[j];
    d.data = b.data;
    d.flags = b.flags;
    d.dstride = b.data_row_stride;
    d.fstride = b.flag_row_stride;
    d.C = b.n_channels;
    d.T = b.n_times;
    d.dtype = b.dtype;
    d.stream_id = history ? b.stream_id : -1;
    d.mask_off = moff;
    d.out_idx = i;
    const size_t es = elem_size(b.dtype);
    d.aligned = (((uintptr_t)b.data % 16) == 0 && ((size_t)b.data_row_stride * es) % 16 == 0) ? 1 : 0;
    d.faligned = (((uintptr_t)b.flags % 16) == 0 && (b.flag_row_stride % 16) == 0) ? 1 : 0;
    d.sidx = j;
    moff += (int64_t)b.n_channels * ((b.n_times + 63) / 64);
    counts[variant_of(t, b)]++;
  }
  s.ncx = 0;
  for (int j = 0; j < n; ++j)
    if (variant_of(t, blocks[order[j]]) == 3 && cx(blocks[order[j]])) s.ncx++;
}

// one kernel launch over nb blocks (maxch > 0: chunked kernel, nb * maxch items)
void launch(lof_ctx* c, const lof_tuning& t, int kid, int phase, const DevBlock* dd, int nb, int maxch, Slot& s,
            int& ncounter, hipStream_t st, const DevParams& P, size_t lds = 0) {
  const int items = maxch > 0 ? nb * maxch : nb;
  if (items <= 0) return;
  int* counter = nullptr;
  int grid = items;
  if (t.persistent && ncounter < NCOUNTER) {
    counter = s.d_counter + ncounter++;
    grid = std::min(items, std::max(1, c->occ[kid]) * std::max(1, c->n_cu));
  }
  const DevBlock* a_blocks = dd;
  int a_nb = nb, a_maxch = maxch;
  int* a_counter = counter;
  DevParams a_p = P;
  if (maxch > 0) {
    void* args[] = {&a_blocks, &a_nb, &a_maxch, &a_counter, &a_p};
    (void)hipLaunchKernel(kernel_of(kid), dim3(grid), dim3(lofk::WG), args, lds, st);
  } else {
    void* args[] = {&a_blocks, &a_nb, &a_counter, &a_p};
    (void)hipLaunchKernel(kernel_of(kid), dim3(grid), dim3(lofk::WG), args, 0, st);
  }
  if (s.tev[0] && s.ntev > 0 && s.ntev < NTEV) {
    s.tph[s.ntev] = phase;
    (void)hipEventRecord(s.tev[s.ntev++], st);
  }
}

template <class F>
int max_chunks(const DevBlock* h, int n, F&& f) {
  int m = 0;
  for (int i = 0; i < n; ++i) m = std::max(m, f(h[i]));
  return m;
}

// kernels of one call on stream st (descriptors already on the device in s and
// still in s.h_desc, which sizes the chunked launches)
void enqueue(lof_ctx* c, const lof_tuning& t, Slot& s, const int* counts, int n, void* stats, hipStream_t st,
             bool autocommit, bool timing = false) {
  DevParams P = dev_params(c, s.d_mask, s.d_mask2, s.d_state, s.d_rowsum, stats);
  P.cand = s.d_cand;
  if (t.persistent) hipLaunchKernelGGL(lofk::lof_zero_kernel, dim3(1), dim3(64), 0, st, s.d_counter, NCOUNTER);
  s.ntev = 0;
  if (timing && s.tev[0] && hipEventRecord(s.tev[0], st) == hipSuccess) s.ntev = 1;
  int nc = 0;
  int off = 0;
  for (int kind = 0; kind < 2; ++kind) {
    const int kcnt = counts[3 * kind] + counts[3 * kind + 1] + counts[3 * kind + 2];
    if (!kcnt) continue;
    const bool integer = kind == 0;
    const DevBlock* dk = s.d_desc + off;
    const DevBlock* hk = s.h_desc + off;
    if (P.integrated) {
      // spectrum and time series flagging per block, then history and flag bytes
      DevParams Pi = P;
      Pi.integ_tmax = max_chunks(hk, kcnt, [&](const DevBlock& b) { return b.T; });
      launch(c, t, K_INTEG + kind, LOF_PHASE_STATS, dk, kcnt, 1, s, nc, st, Pi, lofk::integ_lds_bytes(Pi.integ_tmax));
      const int mw = max_chunks(hk, kcnt, [&](const DevBlock& b) { return lofk::final_chunks(b.C); });
      launch(c, t, K_FINAL + kind, LOF_PHASE_FINAL, dk, kcnt, mw, s, nc, st, P);
      off += kcnt;
      continue;
    }
    const bool pre = (c->prm.options & LOF_OPT_PREFLAGGED) != 0;
    // a few float blocks with a large one among them: each block's statistics
    // split over workgroups (one launch per radix pass), else one workgroup per block
    const int64_t big = max_chunks(hk, kcnt, [&](const DevBlock& b) { return (int)std::min<int64_t>(
                                                   (int64_t)b.C * b.T, INT32_MAX); });
    if (!integer && s.d_split && kcnt <= s.nsplit && lofk::split_chosen(kcnt, big)) {
      const int mp = max_chunks(hk, kcnt, [&](const DevBlock& b) { return lofk::split_parts(b.C, b.T); });
      const int np = lofk::split_passes(P.robust != 0);
      lofk::SplitState* ss = s.d_split;
      const int kid = K_SPLIT + (pre ? 1 : 0);
      for (int pass = 0; pass < np; ++pass) {
        const DevBlock* a_blocks = dk;
        int a_nb = kcnt, a_mp = mp, a_pass = pass;
        lofk::SplitState* a_ss = ss;
        DevParams a_p = P;
        void* args[] = {&a_blocks, &a_nb, &a_mp, &a_pass, &a_ss, &a_p};
        (void)hipLaunchKernel(kernel_of(kid), dim3(kcnt * mp), dim3(lofk::WG), args, 0, st);
      }
      if (s.tev[0] && s.ntev > 0 && s.ntev < NTEV) {
        s.tph[s.ntev] = LOF_PHASE_STATS;
        (void)hipEventRecord(s.tev[s.ntev++], st);
      }
    } else {
      launch(c, t, (pre ? K_STATS_PRE : K_STATS) + kind, LOF_PHASE_STATS, dk, kcnt, 0, s, nc, st, P);
    }
    int mt[3] = {0, 0, 0};
    for (int j = 0, voff = 0; j < 3; voff += counts[3 * kind + j], ++j) {
      const int cnt = counts[3 * kind + j];
      if (!cnt) continue;
      const int L = variant_lanes(j);
      mt[j] = max_chunks(hk + voff, cnt, [&](const DevBlock& b) { return lofk::time_chunks(b.C, b.T, L); });
      // float rows of complex input at 32 lanes (the group's head) keep their powers
      const int ncx = (!pre && kind == 1 && j == 0) ? s.ncx : 0;
      if (ncx > 0) {
        const int mx = max_chunks(hk + voff, ncx, [&](const DevBlock& b) { return lofk::time_chunks(b.C, b.T, L); });
        launch(c, t, K_TIMECX, LOF_PHASE_ST_TIME, dk + voff, ncx, mx, s, nc, st, P);
      }
      if (cnt > ncx) {
        const int mr = max_chunks(hk + voff + ncx, cnt - ncx,
                                  [&](const DevBlock& b) { return lofk::time_chunks(b.C, b.T, L); });
        launch(c, t, (pre ? K_TIME_PRE : K_TIME) + 3 * kind + j, LOF_PHASE_ST_TIME, dk + voff + ncx, cnt - ncx, mr, s,
               nc, st, P);
      }
    }
    const int mf = max_chunks(hk, kcnt, [&](const DevBlock& b) { return lofk::freq_chunks(integer, b.C, b.T); });
    // float blocks of at most 16 channels only: the small-slab kernel
    const bool small = !integer && max_chunks(hk, kcnt, [&](const DevBlock& b) { return b.C; }) <= 16;
    launch(c, t, small ? K_FREQS : K_FREQ + kind, LOF_PHASE_ST_FREQ, dk, kcnt, mf, s, nc, st, P);
    // blocks of at most 64 channels and 4096 times: SIR, history and flag bytes in
    // one kernel per block with the mask in LDS, when the blocks fill the chip
    // (fewer blocks than CUs: the row- and column-chunked kernels spread them)
    bool post = !P.prose && (t.fuse_post == 1 || (t.fuse_post == 0 && kcnt >= c->n_cu));
    for (int i = 0; post && i < kcnt; ++i) post = lofk::post_eligible(hk[i].C, hk[i].T);
    if (post) {
      launch(c, t, K_POST + kind, LOF_PHASE_FINAL, dk, kcnt, 1, s, nc, st, P);
      off += kcnt;
      continue;
    }
    if (c->prm.sir_eta_num > 0 && P.prose) {
      const int mr = max_chunks(hk, kcnt, [&](const DevBlock& b) { return lofk::prose_time_chunks(b.C); });
      launch(c, t, K_PROSE, LOF_PHASE_SIR_TIME, dk, kcnt, mr, s, nc, st, P);
      const int mc = max_chunks(hk, kcnt, [&](const DevBlock& b) { return lofk::prose_freq_chunks(b.T); });
      launch(c, t, K_PROSE + 1, LOF_PHASE_SIR_FREQ, dk, kcnt, mc, s, nc, st, P);
    } else if (c->prm.sir_eta_num > 0) {
      for (int j = 0, voff = 0; j < 3; voff += counts[3 * kind + j], ++j) {
        const int cnt = counts[3 * kind + j];
        if (cnt) launch(c, t, K_SIRT + j, LOF_PHASE_SIR_TIME, dk + voff, cnt, mt[j], s, nc, st, P);
      }
      const int ms = max_chunks(hk, kcnt, [&](const DevBlock& b) { return lofk::sirf_chunks(b.C, b.T); });
      launch(c, t, K_SIRF, LOF_PHASE_SIR_FREQ, dk, kcnt, ms, s, nc, st, P);
    }
    const int mw = max_chunks(hk, kcnt, [&](const DevBlock& b) { return lofk::final_chunks(b.C); });
    launch(c, t, K_FINAL + kind, LOF_PHASE_FINAL, dk, kcnt, mw, s, nc, st, P);
    off += kcnt;
  }
  if (autocommit) hipLaunchKernelGGL(lofk::lof_commit_desc_kernel, dim3(n), dim3(256), 0, st, s.d_desc, n, P);
}

// add a finished call's phase times (events of slot s) to the totals of ctx
bool harvest_timing(lof_ctx* c, Slot& s) {
  if (!s.timed || s.ntev < 2) {
    s.timed = false;
    return true;
  }
  s.timed = false;
  if (hipEventSynchronize(s.tev[s.ntev - 1]) != hipSuccess) return false;
  for (int k = 1; k < s.ntev; ++k) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, s.tev[k - 1], s.tev[k]) != hipSuccess) return false;
    c->phase_ms[s.tph[k]] += t;
  }
  c->phase_calls++;
  return true;
}

// one lof_flag_blocks call with partial integration: tile means of every block,
// the whole path on the grids (as float32 blocks, history keyed by row of tiles),
// then every sample of a block takes its tile's flag
lof_status flag_partial(lof_ctx* c, const lof_block* blocks, int32_t n, hipStream_t st, lof_block_stats* stats,
                        bool autocommit) {
  Slot& s = c->slot[c->next];
  PSlot& ps = c->pslot[c->next];
  c->next = (c->next + 1) % (int)c->slot.size();
  if (s.used) {
    // the slot's previous call must be done before its tables and grids are reused
    if (hipEventSynchronize(s.ev) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "hipEventSynchronize failed");
    if (!harvest_timing(c, ps.s)) return fail(c, LOF_ERR_DEVICE, "event timing failed");
  }
  int64_t off = 0;
  int max_items = 1, max_rows = 1;
  bool kinds[2] = {false, false};
  for (int i = 0; i < n; ++i) {
    const lof_block& b = blocks[i];
    lofk::PartialBlock& pb = ps.h_part[i];
    DevBlock& d = pb.fine;
    d = DevBlock();
    d.data = b.data;
    d.flags = b.flags;
    d.dstride = b.data_row_stride;
    d.fstride = b.flag_row_stride;
    d.C = b.n_channels;
    d.T = b.n_times;
    d.dtype = b.dtype;
    d.stream_id = b.stream_id;
    d.out_idx = i;
    const size_t es = elem_size(b.dtype);
    d.aligned = (((uintptr_t)b.data % 16) == 0 && ((size_t)b.data_row_stride * es) % 16 == 0) ? 1 : 0;
    d.faligned = (((uintptr_t)b.flags % 16) == 0 && (b.flag_row_stride % 16) == 0) ? 1 : 0;
    pb.Cc = ceil_div(b.n_channels, c->pf);
    pb.Tc = ceil_div(b.n_times, c->pt);
    pb.cstride = round16(pb.Tc);
    pb.coarse = ps.d_coarse + off;
    pb.cflags = ps.d_cflags + off;
    pb.ff = c->pf;
    pb.ft = c->pt;
    lof_block& cb = c->ctmp[i];
    cb.data = pb.coarse;
    cb.flags = pb.cflags;
    cb.data_row_stride = pb.cstride;
    cb.flag_row_stride = pb.cstride;
    cb.n_channels = pb.Cc;
    cb.n_times = pb.Tc;
    cb.dtype = LOF_F32;
    cb.stream_id = b.stream_id;
    off += (int64_t)pb.Cc * pb.cstride;
    max_items = std::max(max_items, lofk::part_items(pb.Cc, pb.Tc, pb.ft));
    max_rows = std::max(max_rows, lofk::part_spread_chunks(b.n_channels));
    kinds[b.dtype == LOF_CI8 ? 0 : 1] = true;
  }
  if (hipMemcpyAsync(ps.d_part, ps.h_part, sizeof(lofk::PartialBlock) * n, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(c, LOF_ERR_DEVICE, "descriptor upload failed");
  const lofk::PartialBlock* dpart = ps.d_part;
  int a_n = n, a_items = max_items, a_rows = max_rows;
  lof_block_stats* a_stats = stats;
  const lof_block_stats* a_cstats = ps.d_cstats;
  for (int kind = 0; kind < 2; ++kind) {
    if (!kinds[kind]) continue;
    void* args[] = {&dpart, &a_n, &a_items, &a_stats};
    (void)hipLaunchKernel(lofk::kernel_partial_integrate(kind == 0), dim3(n * max_items), dim3(lofk::WG), args, 0, st);
  }
  int counts[NVAR];
  build_table(c->order.data(), c->tune, c->ctmp.data(), n, ps.s, counts, true);
  if (hipMemcpyAsync(ps.s.d_desc, ps.s.h_desc, sizeof(DevBlock) * n, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(c, LOF_ERR_DEVICE, "descriptor upload failed");
  const bool timing = (c->prm.options & LOF_OPT_PHASE_TIMING) != 0;
  enqueue(c, c->tune, ps.s, counts, n, ps.d_cstats, st, autocommit, timing);
  {
    void* args[] = {&dpart, &a_n, &a_rows, &a_cstats, &a_stats};
    (void)hipLaunchKernel(lofk::kernel_partial_spread(), dim3(n * max_rows), dim3(lofk::WG), args, 0, st);
  }
  if (hipGetLastError() != hipSuccess) return fail(c, LOF_ERR_DEVICE, "kernel launch failed");
  ps.s.timed = timing && ps.s.ntev >= 2;
  if (hipEventRecord(s.ev, st) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "hipEventRecord failed");
  s.used = true;
  return LOF_OK;
}

}  // namespace

extern "C" {
lof_status lof_default_params(lof_params* p) {
  if (!p) return LOF_ERR_INVALID;
  std::memset(p, 0, sizeof(*p));
  p->start_threshold = 6.0;
  p->p = 1.5;
  p->sensitivity = 1.0;
  p->n_levels = 7;
  p->n_levels_freq = -1;
  p->sir_eta_num = 1;
  p->sir_eta_den = 5;
  p->history_sensitivity = 6.0;
  p->history_len = 32;
  p->history_min = 4;
  p->max_streams = 1;
  p->max_channels = 64;
  p->max_blocks_per_call = 1;
  p->max_samples_per_call = LOF_MAX_BLOCK_SAMPLES;
  p->options = 0;
  return LOF_OK;
}


lof_status lof_destroy(lof_ctx* c) {
  if (!c) return LOF_OK;
  DevGuard g(c->dev);
  for (auto& s : c->slot) free_slot(s);
  for (auto& p : c->pslot) free_pslot(p);
  free_slot(c->gslot);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->ring) (void)hipFree(c->ring);
  if (c->rcount) (void)hipFree(c->rcount);
  if (c->rhead) (void)hipFree(c->rhead);
  if (c->pend) (void)hipFree(c->pend);
  if (c->pvalid) (void)hipFree(c->pvalid);
  delete c;
  return LOF_OK;
}

lof_status lof_create(const lof_params* params, int hip_device, lof_ctx** out) {
  if (!out) {
    g_create_err = "out is NULL";
    return LOF_ERR_INVALID;
  }
  *out = nullptr;
  if (const char* m = check_params(params)) {
    g_create_err = m;
    return LOF_ERR_INVALID;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
    g_create_err = "no such HIP device";
    return LOF_ERR_INVALID;
  }
  lof_ctx* c = new (std::nothrow) lof_ctx();
  if (!c) {
    g_create_err = "host allocation failed";
    return LOF_ERR_NOMEM;
  }
  c->prm = *params;
  c->dev = hip_device;
  default_tuning(&c->tune);
  DevGuard g(hip_device);
  const int64_t SC = (int64_t)params->max_streams * params->max_channels;
  bool ok = hipMalloc(&c->ring, sizeof(double) * SC * params->history_len) == hipSuccess &&
            hipMalloc(&c->rcount, sizeof(int32_t) * SC) == hipSuccess &&
            hipMalloc(&c->rhead, sizeof(int32_t) * SC) == hipSuccess &&
            hipMalloc(&c->pend, sizeof(double) * SC) == hipSuccess &&
            hipMalloc(&c->pvalid, SC) == hipSuccess;
  if (ok) {
    ok = hipMemset(c->ring, 0, sizeof(double) * SC * params->history_len) == hipSuccess &&
         hipMemset(c->rcount, 0, sizeof(int32_t) * SC) == hipSuccess &&
         hipMemset(c->rhead, 0, sizeof(int32_t) * SC) == hipSuccess &&
         hipMemset(c->pend, 0, sizeof(double) * SC) == hipSuccess &&
         hipMemset(c->pvalid, 0, SC) == hipSuccess;
  }
  // mask scratch: one u64 word per 64 samples of a row, rows rounded up
  c->mask_words = (size_t)(params->max_samples_per_call / 64) +
                  (size_t)params->max_blocks_per_call * (size_t)params->max_channels + 64;
  const bool timing = (params->options & LOF_OPT_PHASE_TIMING) && !(params->options & LOF_OPT_GRAPH);
  const bool prose = (params->options & LOF_OPT_SIR_PROSE) != 0;
  c->slot.resize(params->call_slots > 0 ? params->call_slots : NSLOT);
  for (size_t i = 0; ok && i < c->slot.size(); ++i)
    ok = alloc_slot(c->slot[i], params->max_blocks_per_call, params->max_channels, c->mask_words, timing, prose);
  c->partial = params->partial_time > 1 || params->partial_freq > 1;
  if (ok && c->partial) {
    c->pt = std::max(1, params->partial_time);
    c->pf = std::max(1, params->partial_freq);
    // tile cells of one call, rows padded to 16: per block at most
    // C (T + 15) and (C/pf + 1) (T/pt + 16); the sum of T is at most the samples
    const size_t S = (size_t)params->max_samples_per_call, B = (size_t)params->max_blocks_per_call;
    const size_t M = (size_t)params->max_channels;
    const size_t cap1 = S + 15 * B * M;
    const size_t cap2 = S / ((size_t)c->pf * c->pt) + 16 * B * (M / c->pf + 1) + S / c->pt + 16 * B + 64;
    c->coarse_cap = std::min(cap1, cap2);
    c->pslot.resize(c->slot.size());
    for (size_t i = 0; ok && i < c->pslot.size(); ++i) {
      PSlot& p = c->pslot[i];
      ok = alloc_slot(p.s, params->max_blocks_per_call, params->max_channels, c->mask_words, timing, prose) &&
           hipMalloc(&p.d_part, sizeof(lofk::PartialBlock) * B) == hipSuccess &&
           hipHostMalloc(&p.h_part, sizeof(lofk::PartialBlock) * B, hipHostMallocDefault) == hipSuccess &&
           hipMalloc(&p.d_coarse, sizeof(float) * c->coarse_cap) == hipSuccess &&
           hipMalloc(&p.d_cflags, c->coarse_cap) == hipSuccess &&
           hipMalloc(&p.d_cstats, sizeof(lof_block_stats) * B) == hipSuccess;
    }
  }
  if (ok && (params->options & LOF_OPT_GRAPH)) {
    ok = alloc_slot(c->gslot, params->max_blocks_per_call, params->max_channels, c->mask_words, false, prose) &&
         hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
  }
  if (ok) {
    hipDeviceProp_t prop;
    ok = hipGetDeviceProperties(&prop, hip_device) == hipSuccess;
    c->n_cu = ok ? prop.multiProcessorCount : 0;
    const int integ_lds = (int)lofk::integ_lds_bytes(lofk::INTEG_MAX_T);
    for (int k = K_INTEG; ok && k < K_INTEG + 2; ++k)
      ok = hipFuncSetAttribute(kernel_of(k), hipFuncAttributeMaxDynamicSharedMemorySize, integ_lds) == hipSuccess;
    for (int k = 0; ok && k < NKERN; ++k)
      ok = hipOccupancyMaxActiveBlocksPerMultiprocessor(&c->occ[k], kernel_of(k), lofk::WG,
                                                        (k == K_INTEG || k == K_INTEG + 1) ? 3072 * 8 : 0) ==
           hipSuccess;
  }
  if (ok) ok = hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    lof_destroy(c);
    g_create_err = "device allocation failed";
    return LOF_ERR_NOMEM;
  }
  c->seen.assign(params->max_streams, -1);
  c->tmp.resize(params->max_blocks_per_call);
  c->order.resize(params->max_blocks_per_call);
  if (c->partial) c->ctmp.resize(params->max_blocks_per_call);
  *out = c;
  return LOF_OK;
}

lof_status lof_flag_blocks(lof_ctx* c, const lof_block* blocks, int32_t n, void* hip_stream,
                           lof_block_stats* stats) {
  if (!c) return LOF_ERR_INVALID;
  if (n < 0) return fail(c, LOF_ERR_INVALID, "n_blocks < 0");
  if (n == 0) return LOF_OK;
  if (!blocks) return fail(c, LOF_ERR_INVALID, "blocks is NULL");
  const lof_status vs = validate(c, blocks, n, true);
  if (vs != LOF_OK) return vs;
  DevGuard g(c->dev);
  hipStream_t st = (hipStream_t)hip_stream;
  const bool autocommit = (c->prm.options & LOF_OPT_AUTOCOMMIT) != 0;
  int counts[NVAR];

  if (c->prm.options & LOF_OPT_GRAPH) {
    Slot& s = c->gslot;
    const bool same = c->gvalid && (int32_t)c->gsig.size() == n && c->gstats == (void*)stats &&
                      std::memcmp(c->gsig.data(), blocks, sizeof(lof_block) * n) == 0;
    if (!same) {
      // rebuild: the previous replay must be done before its table is replaced
      if (s.used && hipEventSynchronize(s.ev) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "graph wait failed");
      if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
      if (c->graph) (void)hipGraphDestroy(c->graph);
      c->gexec = nullptr;
      c->graph = nullptr;
      c->gvalid = false;
      build_table(c->order.data(), c->tune, blocks, n, s, counts, true);
      if (hipMemcpy(s.d_desc, s.h_desc, sizeof(DevBlock) * n, hipMemcpyHostToDevice) != hipSuccess)
        return fail(c, LOF_ERR_DEVICE, "descriptor upload failed");
      if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(c, LOF_ERR_DEVICE, "graph capture failed");
      enqueue(c, c->tune, s, counts, n, stats, c->cap_stream, autocommit);
      if (hipStreamEndCapture(c->cap_stream, &c->graph) != hipSuccess ||
          hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, LOF_ERR_DEVICE, "graph instantiation failed");
      }
      c->gsig.assign(blocks, blocks + n);
      c->gstats = (void*)stats;
      c->gvalid = true;
    } else if (s.used) {
      // replays share the graph's scratch: order them on the device
      if (hipStreamWaitEvent(st, s.ev, 0) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "stream wait failed");
    }
    if (hipGraphLaunch(c->gexec, st) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "graph launch failed");
    if (hipEventRecord(s.ev, st) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "hipEventRecord failed");
    s.used = true;
    return LOF_OK;
  }

  if (c->partial) return flag_partial(c, blocks, n, st, stats, autocommit);
  Slot& s = c->slot[c->next];
  c->next = (c->next + 1) % (int)c->slot.size();
  if (s.used) {
    // the slot's previous call must be done before its table and scratch are reused
    if (hipEventSynchronize(s.ev) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "hipEventSynchronize failed");
    if (!harvest_timing(c, s)) return fail(c, LOF_ERR_DEVICE, "event timing failed");
  }
  build_table(c->order.data(), c->tune, blocks, n, s, counts, true);
  if (hipMemcpyAsync(s.d_desc, s.h_desc, sizeof(DevBlock) * n, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(c, LOF_ERR_DEVICE, "descriptor upload failed");
  const bool timing = (c->prm.options & LOF_OPT_PHASE_TIMING) != 0;
  enqueue(c, c->tune, s, counts, n, stats, st, autocommit, timing);
  if (hipGetLastError() != hipSuccess) return fail(c, LOF_ERR_DEVICE, "kernel launch failed");
  s.timed = timing && s.ntev >= 2;
  if (hipEventRecord(s.ev, st) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "hipEventRecord failed");
  s.used = true;
  return LOF_OK;
}

lof_status lof_get_tuning(const lof_ctx* c, lof_tuning* out) {
  if (!c || !out) return LOF_ERR_INVALID;
  *out = c->tune;
  return LOF_OK;
}

lof_status lof_set_tuning(lof_ctx* c, const lof_tuning* t) {
  if (!c) return LOF_ERR_INVALID;
  if (!tuning_ok(t)) return fail(c, LOF_ERR_INVALID, "tuning values outside the allowed set");
  c->tune = *t;
  c->gvalid = false;   // a cached graph was built with the old tuning
  return LOF_OK;
}

lof_status lof_autotune(lof_ctx* c, const lof_block* blocks, int32_t n, void* hip_stream, int32_t reps,
                        lof_tuning* out) {
  if (!c) return LOF_ERR_INVALID;
  if (n < 0 || reps < 1) return fail(c, LOF_ERR_INVALID, "n < 0 or reps < 1");
  if (c->partial) return fail(c, LOF_ERR_INVALID, "lof_autotune does not run with partial integration");
  if (c->prm.options & LOF_OPT_PREFLAGGED)
    return fail(c, LOF_ERR_INVALID, "lof_autotune does not run with LOF_OPT_PREFLAGGED (tuning runs overwrite flags)");
  if (n > 0 && !blocks) return fail(c, LOF_ERR_INVALID, "blocks is NULL");
  if (n > 0) {
    const lof_status vs = validate(c, blocks, n, false);
    if (vs != LOF_OK) return vs;
  }
  DevGuard g(c->dev);
  hipStream_t st = (hipStream_t)hip_stream;
  // wait for every slot: tuning uses slot 0 synchronously
  for (auto& s : c->slot) {
    if (s.used && hipEventSynchronize(s.ev) != hipSuccess) return fail(c, LOF_ERR_DEVICE, "slot wait failed");
    if (!harvest_timing(c, s)) return fail(c, LOF_ERR_DEVICE, "event timing failed");
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(c, LOF_ERR_DEVICE, "event creation failed");
  Slot& s = c->slot[0];
  lof_tuning best = c->tune;
  auto time_run = [&](const lof_tuning& t, const std::vector<lof_block>& sub, float* ms) -> bool {
    int counts[NVAR];
    const int m = (int)sub.size();
    build_table(c->order.data(), t, sub.data(), m, s, counts, false);
    if (hipMemcpy(s.d_desc, s.h_desc, sizeof(DevBlock) * m, hipMemcpyHostToDevice) != hipSuccess) return false;
    enqueue(c, t, s, counts, m, nullptr, st, false);   // warm-up
    if (hipEventRecord(e0, st) != hipSuccess) return false;
    for (int r = 0; r < reps; ++r) enqueue(c, t, s, counts, m, nullptr, st, false);
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
    return hipEventElapsedTime(ms, e0, e1) == hipSuccess;
  };
  bool ok = true;
  // 1) time layout per (kind, bucket) present in the table, one-workgroup-per-block launches
  for (int kind = 0; ok && kind < 2; ++kind) {
    for (int b = 0; ok && b < LOF_TUNE_BUCKETS; ++b) {
      std::vector<lof_block> sub;
      for (int i = 0; i < n; ++i)
        if ((blocks[i].dtype == LOF_CI8 ? 0 : 1) == kind && time_bucket(blocks[i].n_times) == b)
          sub.push_back(blocks[i]);
      if (sub.empty()) continue;
      float best_ms = 1e30f;
      for (int L : {32, 48, 64}) {
        if (!lanes_allowed(L, b)) continue;
        lof_tuning t = best;
        t.time_lanes[kind][b] = L;
        t.persistent = 0;
        float ms = 0.0f;
        ok = time_run(t, sub, &ms);
        if (ok && ms < best_ms) {
          best_ms = ms;
          best.time_lanes[kind][b] = L;
        }
      }
    }
  }
  // 2) launch mode on the whole table
  if (ok && n > 0) {
    std::vector<lof_block> all(blocks, blocks + n);
    float ms0 = 0.0f, ms1 = 0.0f;
    lof_tuning t = best;
    t.persistent = 0;
    ok = time_run(t, all, &ms0);
    t.persistent = 1;
    if (ok) ok = time_run(t, all, &ms1);
    if (ok) best.persistent = ms1 < ms0 ? 1 : 0;
    // 3) blocks of at most 64 channels and 4096 times: the fused SIR/history
    //    pass or the row- and column-chunked kernels
    bool any_post = false;
    for (int i = 0; i < n && !any_post; ++i) any_post = lofk::post_eligible(blocks[i].n_channels, blocks[i].n_times);
    if (ok && any_post && !(c->prm.options & LOF_OPT_SIR_PROSE)) {
      t = best;
      t.fuse_post = 1;
      ok = time_run(t, all, &ms0);
      t.fuse_post = 2;
      if (ok) ok = time_run(t, all, &ms1);
      if (ok) best.fuse_post = ms1 < ms0 ? 2 : 1;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) {
    (void)hipGetLastError();
    return fail(c, LOF_ERR_DEVICE, "autotune run failed");
  }
  c->tune = best;
  c->gvalid = false;
  if (out) *out = best;
  return LOF_OK;
}

lof_status lof_history_update(lof_ctx* c, const int32_t* ids, int32_t n, void* hip_stream) {
  if (!c) return LOF_ERR_INVALID;
  if (n < 0) return fail(c, LOF_ERR_INVALID, "n < 0");
  std::vector<int32_t> list;
  if (ids) {
    list.assign(ids, ids + n);
    for (int32_t s : list)
      if (s < 0 || s >= c->prm.max_streams) return fail(c, LOF_ERR_INVALID, "stream id out of range");
    std::sort(list.begin(), list.end());
    list.erase(std::unique(list.begin(), list.end()), list.end());
    if (list.empty()) return LOF_OK;
  }
  DevGuard g(c->dev);
  hipStream_t st = (hipStream_t)hip_stream;
  const DevParams P = dev_params(c, nullptr, nullptr, nullptr, nullptr, nullptr);
  const int TPB = 256;
  if (!ids) {
    lofk::IdList none;
    none.n = 0;
    const int64_t tot = (int64_t)c->prm.max_streams * c->prm.max_channels;
    hipLaunchKernelGGL(lofk::lof_commit_kernel, dim3((unsigned)((tot + TPB - 1) / TPB)), dim3(TPB), 0, st, none,
                       c->prm.max_streams, P);
  } else {
    for (size_t i = 0; i < list.size(); i += 255) {
      lofk::IdList L;
      L.n = (int32_t)std::min<size_t>(255, list.size() - i);
      for (int j = 0; j < L.n; ++j) L.ids[j] = list[i + j];
      const int64_t tot = (int64_t)L.n * c->prm.max_channels;
      hipLaunchKernelGGL(lofk::lof_commit_kernel, dim3((unsigned)((tot + TPB - 1) / TPB)), dim3(TPB), 0, st, L, 0,
                         P);
    }
  }
  if (hipGetLastError() != hipSuccess) return fail(c, LOF_ERR_DEVICE, "commit launch failed");
  return LOF_OK;
}

lof_status lof_history_export(lof_ctx* c, double* values, int32_t* counts, double* staged, uint8_t* staged_valid,
                              void* hip_stream) {
  if (!c) return LOF_ERR_INVALID;
  DevGuard g(c->dev);
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t SC = (int64_t)c->prm.max_streams * c->prm.max_channels;
  const int H = c->prm.history_len;
  std::vector<double> ring((size_t)SC * H);
  std::vector<int32_t> cnt(SC), head(SC);
  bool ok = hipMemcpyAsync(ring.data(), c->ring, sizeof(double) * SC * H, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipMemcpyAsync(cnt.data(), c->rcount, sizeof(int32_t) * SC, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipMemcpyAsync(head.data(), c->rhead, sizeof(int32_t) * SC, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (ok && staged) ok = hipMemcpyAsync(staged, c->pend, sizeof(double) * SC, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (ok && staged_valid)
    ok = hipMemcpyAsync(staged_valid, c->pvalid, SC, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(st) == hipSuccess;
  if (!ok) return fail(c, LOF_ERR_DEVICE, "history export copy failed");
  for (int64_t i = 0; i < SC; ++i) {
    if (counts) counts[i] = cnt[i];
    if (values) {
      for (int j = 0; j < H; ++j) {
        double v = 0.0;
        if (j < cnt[i]) {
          int k = head[i] - cnt[i] + j;
          if (k < 0) k += H;
          v = ring[(size_t)i * H + k];
        }
        values[(size_t)i * H + j] = v;
      }
    }
  }
  return LOF_OK;
}

lof_status lof_phase_times(lof_ctx* c, double* ms, int32_t* n_calls) {
  if (!c) return LOF_ERR_INVALID;
  if (!ms || !n_calls) return fail(c, LOF_ERR_INVALID, "ms or n_calls is NULL");
  if (!(c->prm.options & LOF_OPT_PHASE_TIMING) || (c->prm.options & LOF_OPT_GRAPH))
    return fail(c, LOF_ERR_INVALID, "phase timing needs LOF_OPT_PHASE_TIMING without LOF_OPT_GRAPH");
  DevGuard g(c->dev);
  for (auto& s : c->slot)
    if (!harvest_timing(c, s)) return fail(c, LOF_ERR_DEVICE, "event timing failed");
  for (auto& p : c->pslot)
    if (!harvest_timing(c, p.s)) return fail(c, LOF_ERR_DEVICE, "event timing failed");
  for (int p = 0; p < LOF_N_PHASES; ++p) {
    ms[p] = c->phase_ms[p];
    c->phase_ms[p] = 0.0;
  }
  *n_calls = c->phase_calls;
  c->phase_calls = 0;
  return LOF_OK;
}

const char* lof_last_error(const lof_ctx* c) { return c ? c->err : g_create_err; }

// ---------------------------------------------------------------- allocation-free entry point
namespace {
constexpr int STATIC_MAX_DEVICES = 64;
constexpr int STATIC_MAX_BLOCKS = 4096;
std::atomic<void*> g_static_scratch[STATIC_MAX_DEVICES];
// host-side descriptor staging, in static storage; one call at a time builds it
std::mutex g_static_mu;
int g_static_order[STATIC_MAX_BLOCKS];
DevBlock g_static_desc[STATIC_MAX_BLOCKS];

lof_status static_fail(lof_status s, const char* m) {
  g_create_err = m;
  return s;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

lof_status lof_flag_blocks_static(const lof_params* params, int hip_device, const lof_block* blocks,
                                  int32_t n_blocks, void* hip_stream, lof_block_stats* stats) {
  if (const char* m = check_params(params)) return static_fail(LOF_ERR_INVALID, m);
  if (params->partial_time > 1 || params->partial_freq > 1)
    return static_fail(LOF_ERR_INVALID, "no partial integration here");
  if (n_blocks < 0) return static_fail(LOF_ERR_INVALID, "n_blocks < 0");
  if (n_blocks == 0) return LOF_OK;
  if (!blocks) return static_fail(LOF_ERR_INVALID, "blocks is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev ||
      hip_device >= STATIC_MAX_DEVICES)
    return static_fail(LOF_ERR_INVALID, "no such HIP device");
  if (n_blocks > STATIC_MAX_BLOCKS) return static_fail(LOF_ERR_CAPACITY, "more than 4096 blocks");
  int maxC = 1;
  size_t words = 0;
  for (int i = 0; i < n_blocks; ++i) {
    lof_status code;
    if (const char* m = check_block(blocks[i], LOF_MAX_CHANNELS, 1, &code)) return static_fail(code, m);
    if (blocks[i].stream_id != -1) return static_fail(LOF_ERR_INVALID, "no history here: stream_id must be -1");
    if ((params->options & LOF_OPT_INTEGRATED) && blocks[i].n_times > lofk::INTEG_MAX_T)
      return static_fail(LOF_ERR_INVALID, "integrated mode: n_times > 16384");
    maxC = std::max(maxC, blocks[i].n_channels);
    words += block_mask_words(blocks[i]);
  }
  // carve the scratch array: descriptors, block statistics, row sums, work counters, mask words
  const size_t o_desc = 0;
  const size_t o_state = align256(o_desc + sizeof(DevBlock) * n_blocks);
  const size_t o_rowsum = align256(o_state + sizeof(BlockState) * n_blocks);
  const size_t o_counter = align256(o_rowsum + sizeof(uint64_t) * (size_t)n_blocks * maxC);
  const size_t o_mask = align256(o_counter + sizeof(int) * NCOUNTER);
  const bool prose = (params->options & LOF_OPT_SIR_PROSE) != 0 && params->sir_eta_num > 0;
  const size_t o_mask2 = align256(o_mask + sizeof(uint64_t) * words);
  const size_t need = prose ? o_mask2 + sizeof(uint64_t) * words : o_mask + sizeof(uint64_t) * words;
  if (need > lofk::STATIC_SCRATCH_BYTES) return static_fail(LOF_ERR_CAPACITY, "call needs more than the 32 MiB static scratch");

  std::lock_guard<std::mutex> lock(g_static_mu);
  DevGuard g(hip_device);
  void* base = g_static_scratch[hip_device].load();
  if (!base) {
    if (hipGetSymbolAddress(&base, HIP_SYMBOL(lofk::scratch)) != hipSuccess || !base) {
      (void)hipGetLastError();
      return static_fail(LOF_ERR_DEVICE, "hipGetSymbolAddress of the static scratch failed");
    }
    g_static_scratch[hip_device].store(base);
  }
  unsigned char* sp = (unsigned char*)base;
  hipStream_t st = (hipStream_t)hip_stream;

  lof_ctx c;                     // launch configuration only: owns no memory
  c.prm = *params;
  c.prm.max_channels = maxC;     // row sums are indexed [block][maxC]
  c.prm.options &= ~(uint32_t)(LOF_OPT_AUTOCOMMIT | LOF_OPT_GRAPH | LOF_OPT_PHASE_TIMING);
  default_tuning(&c.tune);
  Slot s;
  s.d_desc = (DevBlock*)(sp + o_desc);
  s.h_desc = g_static_desc;
  s.d_state = (BlockState*)(sp + o_state);
  s.d_rowsum = (uint64_t*)(sp + o_rowsum);
  s.d_counter = (int*)(sp + o_counter);
  s.d_mask = (uint64_t*)(sp + o_mask);
  s.d_mask2 = prose ? (uint64_t*)(sp + o_mask2) : nullptr;
  int counts[NVAR];
  build_table(g_static_order, c.tune, blocks, n_blocks, s, counts, false);
  for (int i = 0; i < n_blocks; i += lofk::DESC_CHUNK) {
    lofk::DescChunk ch;
    ch.n = std::min(lofk::DESC_CHUNK, n_blocks - i);
    ch.first = i;
    std::memcpy(ch.d, s.h_desc + i, sizeof(DevBlock) * ch.n);
    hipLaunchKernelGGL(lofk::lof_put_desc_kernel, dim3(1), dim3(lofk::DESC_CHUNK), 0, st, s.d_desc, ch);
  }
  enqueue(&c, c.tune, s, counts, n_blocks, stats, st, false);
  if (hipGetLastError() != hipSuccess) return static_fail(LOF_ERR_DEVICE, "kernel launch failed");
  return LOF_OK;
}


}  // extern "C"
