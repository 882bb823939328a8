/*
 * lof.h -- C ABI of the MI355X (gfx950) LOFAR Online Flagger hot path.
 *
 * Method: van Nieuwpoort, "Towards exascale real-time RFI mitigation",
 * arXiv 1701.08197.  Per time-frequency block the library computes
 *   power |x|^2 (or amplitude, or takes power as given)           -- Sec. 4
 *   block median and population standard deviation                 -- Sec. 2.1, 4.2
 *   threshold_I = median + stddev * factor_I * sensitivity,
 *   factor_I = startThreshold * p^log2(I) / I, I = 1, 2, 4, ...    -- Sec. 2.1
 *   SumThreshold along time, then along frequency                  -- Sec. 2.1
 *   the scale-invariant rank (SIR) operator, time then frequency   -- Sec. 2.2
 *   the history flagger against per-channel statistics of earlier
 *   blocks of the same stream                                      -- Sec. 4.1
 * and writes one flag byte per sample.  All work runs in HIP kernels on the
 * device; the host side only validates, lays out descriptors and enqueues.
 *
 * Conventions shared by every call:
 *  - All calls are asynchronous with respect to the host: they validate their
 *    arguments synchronously (all-or-nothing: an invalid call enqueues nothing
 *    and changes no state) and then enqueue work on `hip_stream` (a hipStream_t
 *    passed as void*, NULL = the legacy default stream).
 *  - Pointers inside lof_block and the `stats` array are DEVICE pointers owned
 *    by the caller; they must stay valid until the work enqueued on the stream
 *    has completed.  Host arrays (the lof_block array, stream id lists) are
 *    read during the call only.
 *  - A lof_ctx is not thread-safe.  Calls on different HIP streams may overlap
 *    on the device as long as they do not name the same history stream id while
 *    both are in flight (the history ring of that id would race).
 *  - Device faults surface as LOF_ERR_DEVICE on a later call.
 *  - lof_last_error() returns a static description of the last failure.
 */
#ifndef LOF_H
#define LOF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lof_ctx lof_ctx;

typedef enum {
  LOF_OK = 0,
  LOF_ERR_INVALID = -1,   /* bad argument (nothing enqueued, no state change)   */
  LOF_ERR_NOMEM = -2,     /* device or pinned-host allocation failed (create)   */
  LOF_ERR_DEVICE = -3,    /* a HIP runtime call failed                           */
  LOF_ERR_CAPACITY = -4   /* request exceeds the capacities given to lof_create */
} lof_status;

/* Sample types (Sec. 4: voltages need power first; visibilities are flagged on
 * amplitude; beam-formed data is Stokes I as given). */
typedef enum {
  LOF_CI8 = 0,     /* complex int8, interleaved (re, im) bytes; power re^2+im^2 is an
                      exact integer, so flags are exact                              */
  LOF_C64 = 1,     /* complex64 (float re, float im); power in float32                */
  LOF_F32 = 2,     /* float32 power / Stokes I, flagged as given                      */
  LOF_C64_AMP = 3  /* complex64 visibilities; amplitude sqrt(re^2+im^2) in float32    */
} lof_dtype;

/* Option bits for lof_params.options */
#define LOF_OPT_AUTOCOMMIT 0x1u          /* lof_flag_blocks also commits the history
                                            values it staged (same enqueue)          */
#define LOF_OPT_LITERAL_HISTORY_TIE 0x2u /* history flags when cur >= thr (the Sec. 4.1
                                            listing's else-branch) instead of cur > thr */
#define LOF_OPT_GRAPH 0x4u               /* keep the launches of the last block table in
                                            a hipGraph and replay it when lof_flag_blocks
                                            is called again with the identical table and
                                            stats pointer (no descriptor upload, one
                                            graph launch)                                 */
#define LOF_OPT_PHASE_TIMING 0x8u        /* record a HIP event after every phase kernel
                                            of each lof_flag_blocks call, for
                                            lof_phase_times (ignored with LOF_OPT_GRAPH) */
#define LOF_OPT_SIR_PROSE 0x10u          /* the SIR step takes the Sec. 2.2 prose reading:
                                            every maximal range of L consecutive flagged
                                            samples gains floor(eta*L) samples before and
                                            after it (eta = sir_eta_num/sir_eta_den),
                                            along time, then along frequency on the time
                                            result; default: the scale-invariant rank
                                            operator the section cites                 */
#define LOF_OPT_INTEGRATED 0x20u         /* integrated pre-correlation mode (Sec. 4): per
                                            block, integrate time fully and flag the
                                            spectrum along frequency (n_levels_freq
                                            levels), then integrate the unflagged channels
                                            fully and flag the time series along time
                                            (n_levels levels); each series has its own
                                            median, stddev and thresholds and gets the SIR
                                            step; a flagged channel flags its row, a
                                            flagged time its column; then the history
                                            flagger as usual.  Blocks must have
                                            n_times <= 16384 (LOF_ERR_INVALID).  The stats
                                            entry holds the time series' median, stddev
                                            and thresholds.  Complex int8 input stays
                                            exact (64-bit sums, 128-bit moments).      */
#define LOF_OPT_ROBUST_SIGMA 0x40u       /* robust statistics (Sec. 4.2 lists the MAD):
                                            stddev := 1.4826 * median(|x - median(x)|)
                                            in the thresholds, for full-rate blocks and
                                            for the integrated mode's series; complex int8
                                            input stays exact (the deviations are
                                            integers or half-integers)                 */

#define LOF_OPT_PREFLAGGED 0x80u         /* caller-supplied pre-flags: on entry each block's
                                            flag bytes hold a mask (nonzero = flagged, e.g.
                                            known-bad samples or an earlier flagger's
                                            output); those samples leave the median and
                                            stddev (Sec. 4.2: statistics of the unflagged
                                            samples; none left: median and stddev 0),
                                            start flagged in SumThreshold, so they leave
                                            every window's sum and count (Sec. 2.1), and
                                            stay flagged; the flag bytes are then
                                            overwritten with the result.  Not with
                                            LOF_OPT_INTEGRATED or partial integration, nor
                                            in lof_autotune (LOF_ERR_INVALID).          */

/* Phases of the path, in launch order (lof_phase_times) */
#define LOF_PHASE_STATS 0        /* power, median, stddev, thresholds (Sec. 2.1, 4.2)   */
#define LOF_PHASE_ST_TIME 1      /* SumThreshold along time (Sec. 2.1)                  */
#define LOF_PHASE_ST_FREQ 2      /* SumThreshold along frequency (Sec. 2.1)             */
#define LOF_PHASE_SIR_TIME 3     /* SIR operator along time (Sec. 2.2)                  */
#define LOF_PHASE_SIR_FREQ 4     /* SIR operator along frequency (Sec. 2.2)             */
#define LOF_PHASE_FINAL 5        /* history flagger (Sec. 4.1) and flag bytes; for blocks
                                    of at most 64 channels and 4096 times (all blocks of
                                    one input kind in the call) it also holds the SIR
                                    operator, which then runs in the same kernel       */
#define LOF_N_PHASES 6

#define LOF_MAX_LEVELS 16
#define LOF_MAX_CHANNELS 1024
#define LOF_MAX_BLOCK_SAMPLES (1LL << 23)

typedef struct {
  double start_threshold;      /* startThreshold of factor_I (Sec. 2.1); 6.0 gives the
                                  6 sigma first iteration                            */
  double p;                    /* factor base (Sec. 2.1), 1.5                         */
  double sensitivity;          /* Sec. 2.1, 1.0                                       */
  int32_t n_levels;            /* SumThreshold iterations along time, I = 1..2^(n-1)
                                  (Sec. 2.1: 7-10 typical); 1..7 (windows up to 64 are
                                  supported); a level with I > extent is skipped      */
  int32_t n_levels_freq;       /* iterations along frequency; -1 = same as n_levels  */
  int32_t sir_eta_num;         /* SIR eta = num/den (Sec. 2.2: 20 % -> 1/5);          */
  int32_t sir_eta_den;         /* num = 0 disables SIR; 0 <= num <= den, den <= 1024  */
  double history_sensitivity;  /* history threshold = mean + this * stddev of the
                                  committed means (Sec. 4.1)                          */
  int32_t history_len;         /* H, committed means kept per (stream, channel)      */
  int32_t history_min;         /* no history flagging until this many are committed  */
  int32_t max_streams;         /* history stream ids are 0..max_streams-1             */
  int32_t max_channels;        /* ring capacity per stream; also the block C limit   */
  int32_t max_blocks_per_call;
  int32_t call_slots;          /* lof_flag_blocks calls that can be in flight before a
                                  call waits on the host for the oldest: each slot
                                  holds one call's descriptor table and scratch
                                  (sized by the maxima above); 0 = 4              */
  int64_t max_samples_per_call;/* sum of C*T over one lof_flag_blocks call            */
  uint32_t options;            /* LOF_OPT_* bits                                      */
  int32_t partial_time;        /* 2-D flagging with partial integration (Sec. 4, the
                                  alternative to the integrated mode): times per tile,
                                  0 or 1 = none; 1..65536                            */
  int32_t partial_freq;        /* channels per tile, 0 or 1 = none; 1..1024.  With
                                  either above 1 every block is integrated into tile
                                  means (sum of the tile's powers / its sample count,
                                  rounded once to float32; tiles at the block's end
                                  hold fewer samples), the whole path of this header
                                  runs on the grid of means as float32 input (history
                                  keyed by (stream, row of tiles)), and every sample
                                  takes its tile's flag.  The stats entry then holds
                                  the grid's median, stddev and thresholds, n_flagged
                                  counts samples of the block, history_flagged_rows
                                  rows of tiles.  Not with LOF_OPT_INTEGRATED or
                                  LOF_OPT_GRAPH, nor in lof_autotune or
                                  lof_flag_blocks_static (LOF_ERR_INVALID).        */
  int32_t history_winsor;      /* k > 0: the history flagger takes the mean and stddev
                                  of its committed means after winsorizing them (Sec. 4.2
                                  lists winsorized means): the k smallest become the
                                  (k+1)-th smallest and the k largest the (k+1)-th
                                  largest (k at most (L-1)/2 for L committed values);
                                  0 = plain statistics.  Needs history_len <= 64.   */
} lof_params;

typedef struct {
  const void* data;            /* device pointer: row c starts at element c*data_row_stride;
                                  element size 2 (CI8), 8 (C64, C64_AMP) or 4 (F32) bytes */
  uint8_t* flags;              /* device pointer: output, byte 0/1 per sample; row c
                                  starts at byte c*flag_row_stride                    */
  int64_t data_row_stride;     /* elements between channel rows, >= n_times           */
  int64_t flag_row_stride;     /* bytes between channel rows, >= n_times              */
  int32_t n_channels;          /* C: 1..max_channels (and <= LOF_MAX_CHANNELS)        */
  int32_t n_times;             /* T: >= 1; C*T <= LOF_MAX_BLOCK_SAMPLES               */
  int32_t dtype;               /* lof_dtype                                          */
  int32_t stream_id;           /* history key (e.g. station, pol, subband) in
                                  [0, max_streams), or -1 for no history; an id may
                                  appear at most once per call                       */
} lof_block;

/* Launch tuning.  Blocks are grouped by input kind (0 = complex int8, 1 = float
 * types) and time-length bucket (T <= 1024, <= 2048, <= 3072, <= 4096, larger);
 * time_lanes[kind][bucket] is the number of consecutive time samples each GPU
 * lane holds (32, 48 or 64; a row must fit 64 lanes unless the value is 64).
 * persistent = 1 launches each phase kernel as a chip-sized grid whose
 * workgroups take (block, chunk) items from a work counter (largest block
 * first) instead of one workgroup per item.  fuse_post selects, for blocks of
 * at most 64 channels and 4096 times, the one-kernel-per-block pass that runs
 * SIR, the history flagger and the flag bytes with the block's mask in LDS:
 * 0 = when a call holds at least as many such blocks of a kind as the GPU has
 * compute units (fewer blocks spread better over row and column chunks),
 * 1 = always, 2 = never. */
#define LOF_TUNE_BUCKETS 5
typedef struct {
  int32_t time_lanes[2][LOF_TUNE_BUCKETS];
  int32_t persistent;
  int32_t fuse_post;
} lof_tuning;

typedef struct {
  double median;               /* block median (Sec. 2.1)                            */
  double stddev;               /* block population stddev                            */
  double threshold[LOF_MAX_LEVELS]; /* threshold_I for I = 2^k, k < n_levels          */
  int64_t n_flagged;           /* flagged samples in the final output                */
  int32_t history_flagged_rows;/* channels flagged by the history flagger            */
  int32_t _pad;
} lof_block_stats;

/* Fills *params with the defaults: startThreshold 6, p 1.5, sensitivity 1,
 * 7 levels both ways, SIR eta 1/5, history sensitivity 6, H 32, warm-up 4,
 * capacities 1 stream x 64 channels, 1 block, 2^23 samples.  Sec. 2.1, 2.2, 4.1. */
lof_status lof_default_params(lof_params* params);

/* Creates a flagger on HIP device `hip_device`.  Allocates every device buffer
 * the later calls need (history rings sized max_streams*max_channels*history_len
 * float64, descriptor and scratch slots sized by the per-call maxima); later
 * calls never allocate.  Returns LOF_ERR_INVALID for bad parameters (no device
 * work done), LOF_ERR_NOMEM / LOF_ERR_DEVICE on allocation or HIP failures.
 * *out receives the context (NULL on failure). */
lof_status lof_create(const lof_params* params, int hip_device, lof_ctx** out);

/* Flags `n_blocks` independent blocks (Sec. 4.1: one block per station,
 * polarisation and subband per time chunk), writing each block's flags.
 * `blocks` is a HOST array.  `stats` is a DEVICE array of n_blocks entries or
 * NULL; entry i describes blocks[i].  For blocks with stream_id >= 0 the history
 * flagger reads only the committed history of that id and stages one value per
 * channel for lof_history_update (a fully flagged channel stages nothing); a
 * second flag call for the same id before the commit replaces the staged values.
 * n_blocks = 0 is a no-op.  A call with at most 4 float blocks whose largest
 * has 65536 samples or more, or at most 16 whose largest has 2^20, computes
 * their statistics over many workgroups (a few more launches; the float64
 * moment sums are added in another order, so the stddev may differ in its last
 * bits from a call that takes one workgroup per block).
 * Errors: LOF_ERR_INVALID (null ctx/blocks, bad shape,
 * stride, dtype, stream id out of range or repeated), LOF_ERR_CAPACITY (more
 * blocks or samples than the create-time maxima, C > max_channels). */
lof_status lof_flag_blocks(lof_ctx* ctx, const lof_block* blocks, int32_t n_blocks,
                           void* hip_stream, lof_block_stats* stats);

/* Commits the staged history values (Sec. 4.1 addToHistory) of the listed stream
 * ids (HOST array of n ids), or of every stream when stream_ids is NULL.  Ids
 * with nothing staged are a no-op.  Each (stream, channel) ring keeps its last
 * history_len values.  Errors: LOF_ERR_INVALID for ids out of range or n < 0. */
lof_status lof_history_update(lof_ctx* ctx, const int32_t* stream_ids, int32_t n,
                              void* hip_stream);

/* Copies the committed history to HOST arrays (synchronous: waits for the
 * stream): values[s][c][j] oldest-first for j < counts[s][c] (rest 0),
 * counts[s][c], staged[s][c] and staged_valid[s][c], for s < max_streams,
 * c < max_channels, j < history_len.  Any output may be NULL.  Checkpointing
 * and tests. */
lof_status lof_history_export(lof_ctx* ctx, double* values, int32_t* counts,
                              double* staged, uint8_t* staged_valid, void* hip_stream);

/* Reads / replaces the launch tuning of ctx (see lof_tuning).  Results never
 * depend on it.  Errors: LOF_ERR_INVALID for NULL pointers or values outside
 * the allowed set. */
lof_status lof_get_tuning(const lof_ctx* ctx, lof_tuning* out);
lof_status lof_set_tuning(lof_ctx* ctx, const lof_tuning* tuning);

/* Autotuner: times every allowed time_lanes value for each (kind, bucket) that
 * occurs in `blocks`, the two launch modes, and (for blocks of at most 64
 * channels and 4096 times) the fused or chunked SIR/history pass, on these
 * blocks, and keeps the fastest in ctx (synchronous; `reps` timed launches
 * per candidate).  It writes the blocks' flag outputs but stages no history
 * (tuning runs ignore stream ids).  *out (host, nullable) receives the chosen
 * tuning. */
lof_status lof_autotune(lof_ctx* ctx, const lof_block* blocks, int32_t n_blocks, void* hip_stream,
                        int32_t reps, lof_tuning* out);

/* Kernel time of each phase (LOF_PHASE_*), in milliseconds, summed over the
 * lof_flag_blocks calls of ctx since the previous lof_phase_times (or since
 * lof_create), into the HOST array ms[LOF_N_PHASES]; *n_calls receives the
 * number of calls summed.  A phase launched for several block kinds or time
 * layouts counts all its launches.  Each figure is the span between HIP events
 * recorded on the call's stream around that phase's kernels.  Waits for the
 * outstanding calls; resets the totals.  Needs LOF_OPT_PHASE_TIMING (calls made
 * by lof_autotune are not counted).  Errors: LOF_ERR_INVALID when the option is
 * off, ctx uses LOF_OPT_GRAPH or a pointer is NULL; LOF_ERR_DEVICE when an
 * event query fails. */
lof_status lof_phase_times(lof_ctx* ctx, double* ms, int32_t* n_calls);

/* Frees the context.  The caller must have synchronised every stream used with
 * it.  NULL is a no-op. */
lof_status lof_destroy(lof_ctx* ctx);

/* Allocation-free variant of lof_flag_blocks, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): it needs no lof_ctx, and it neither allocates nor
 * frees anything.  Its scratch (descriptor table, per-block statistics, row
 * sums and mask words) is one file-scope device array of 32 MiB per GPU, which
 * stays allocated until the process ends.  The blocks are flagged exactly as
 * lof_flag_blocks flags them with the same `params`, except that there is no
 * history flagger: every stream_id must be -1.  Capacity: at most 4096 blocks
 * and at most what fits the 32 MiB: 256-byte-aligned areas of 72 B per block
 * (descriptors), 144 B per block (statistics), 8 B x n_blocks x (largest C) (row
 * sums), 128 B (counters), and 8 B per 64 samples of every row (mask words), e.g.
 * 160 blocks of 64 x 3072 or 3.9e6 words of rows whose length is a multiple of 64.
 * `params` is read during the call (its capacity and option fields are not used);
 * `blocks`, `stats`, `hip_stream` are as in lof_flag_blocks, on device
 * `hip_device`.  Every call on one GPU shares that GPU's scratch array: calls
 * whose work overlaps on one GPU (different host threads, or different HIP
 * streams) race and give wrong flags; the caller serialises them (the host side
 * also serialises concurrent calls).  Errors (nothing enqueued):
 * LOF_ERR_INVALID (bad params, blocks, device, or a stream_id other than -1),
 * LOF_ERR_CAPACITY (over the limits above), LOF_ERR_DEVICE (HIP failure);
 * lof_last_error(NULL) describes the failure. */
lof_status lof_flag_blocks_static(const lof_params* params, int hip_device, const lof_block* blocks,
                                  int32_t n_blocks, void* hip_stream, lof_block_stats* stats);

/* Static, NUL-terminated description of the last error on ctx (or, when ctx is
 * NULL, of the last failed lof_create or lof_flag_blocks_static on this host
 * thread). */
const char* lof_last_error(const lof_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LOF_H */
