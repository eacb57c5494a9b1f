/*
 * exsum.h -- exact binary64 summation on AMD Instinct MI355X (gfx950).
 *
 * The problem (Neal 2015, "Fast Exact Summation Using Small and Large
 * Superaccumulators", abstract): sum a set of floating-point numbers exactly
 * and round the exact sum once to the nearest binary64 value, ties to even.
 * The result depends only on the multiset of terms: it is bit-identical for
 * every order, launch geometry, tuning choice and batching.
 *
 * Conventions where the paper is silent (the same in every entry point):
 *   - an exact-zero sum, including an empty one, is +0.0;
 *   - any NaN term makes the result a NaN: the largest (bits & ~sign) over
 *     the NaN terms, with the quiet bit set;
 *   - +Inf and -Inf together (no NaN) give the quiet NaN 0x7FF8000000000000;
 *   - an infinite term dominates the finite terms;
 *   - the finite part is exact over the whole exponent range, so a sum whose
 *     partial sums overflow still rounds to the finite exact result
 *     (section "Exact summation using a small superaccumulator", on the
 *     range of the small superaccumulator); |exact sum| >= 2^1024 - 2^970
 *     rounds to an infinity.
 *
 * Memory and streams.  Unless stated otherwise every pointer is a DEVICE
 * pointer owned by the caller, terms are read with no alignment requirement
 * beyond 8 bytes, and every call is asynchronous on `stream` (a hipStream_t
 * passed as void*; NULL is the null stream): results are valid once the
 * stream reaches the call.  The library keeps a small per-(device, stream)
 * workspace (merge accumulators, tickets and segment slots, about 5 MiB)
 * that it allocates on the first call on that stream, zero-initialises
 * synchronously, and keeps clean itself
 * (each call leaves it zeroed); exsum_release() frees it.  Calls on the same
 * stream are ordered; calls on different streams use different workspaces
 * and may overlap.
 *
 * Errors.  Every function returns an exsum_status.  Arguments are checked on
 * the host; nothing is written when a check fails.  EXSUM_EDEVICE reports a
 * HIP error from an allocation or launch (the HIP error state is cleared).
 */
#ifndef EXSUM_H
#define EXSUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EXSUM_OK = 0,
    EXSUM_EINVAL = 1,   /* bad argument: n < 0, nseg < 0, NULL pointer with work to do, bad config */
    EXSUM_ENOMEM = 2,   /* workspace allocation failed */
    EXSUM_EDEVICE = 3   /* a HIP runtime error (launch or device query) */
} exsum_status;

/* Human-readable text for a status code (static storage, never NULL). */
const char *exsum_status_string(int status);

/*
 * exsum_f64 -- out[0] = the correctly rounded exact sum of x[0..n).
 *
 * The exact sum of the terms (abstract; "Exact summation using a small
 * superaccumulator"; "Faster exact summation of many terms with a large
 * superaccumulator").  Short inputs use only a small superaccumulator (67
 * overlapping 64-bit chunks); long inputs stream through a per-workgroup
 * large superaccumulator (4096 chunks, one per sign and exponent, with
 * counts that trigger transfers into the small one), the per-workgroup small
 * superaccumulators are merged with integer additions (Discussion, on
 * splitting a sum across processors and adding small superaccumulators)
 * and the merged value is rounded once.
 *   x   : n binary64 terms, device memory, 8-byte aligned, read only.
 *   n   : number of terms, 0 <= n < 2^40.
 *   out : one binary64 result, device memory.
 * Returns EXSUM_EINVAL for n < 0, n >= 2^40, or a NULL x (n > 0) / out.
 */
int exsum_f64(const double *x, int64_t n, double *out, void *stream);

/*
 * exsum_f64_noalloc -- exsum_f64 without any device allocation, for callers
 * that cannot allocate: code under HIP graph capture before any other call
 * on its stream, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, result bits, kernels and launch configuration as
 * exsum_f64; instead of the per-stream workspace it uses a fixed scratch
 * buffer in the library's static device memory: one 576-byte merge
 * accumulator per device, held until the process ends.  Every n the
 * scratch can serve is accepted (0 <= n < 2^40, as exsum_f64; a larger n,
 * or a NULL x with n > 0 or a NULL out, returns EXSUM_EINVAL).  The first
 * call on a device finds the scratch's address and clears it with a kernel
 * on `stream`; later calls launch only the summing kernel.  The scratch is
 * shared by every call on that device and each call leaves it cleared: calls
 * that overlap on one device (other streams, other threads) race on it and
 * give wrong results, so order them, e.g. on one stream.
 */
int exsum_f64_noalloc(const double *x, int64_t n, double *out, void *stream);

/*
 * exsum_segmented_f64 -- out[i] = exact sum of x[offsets[i] .. offsets[i+1])
 * for 0 <= i < nseg.
 *
 * Many independent exact sums (same definition as exsum_f64) in two
 * launches on `stream` that write disjoint outputs.  Segments longer than
 * seg_small_max terms are summed first, by workgroups with the large
 * superaccumulator, each workgroup taking an equal share of the
 * concatenated terms; a segment cut by workgroup boundaries is merged from
 * its pieces with integer additions.  Segments of at most seg_small_max
 * terms (empty ones included) are then summed whole, each by one wavefront
 * with a small superaccumulator; one workgroup per compute unit takes an
 * equal share of their total length and hands its segments to its
 * wavefronts as they come free (Performance evaluations: the small method
 * wins for short sums, the large one for long sums; Discussion: parts summed
 * separately are added as small superaccumulators).
 *   x       : terms, device memory; may be NULL when every segment is
 *             empty (offsets[0] == offsets[nseg]), and then is never read.
 *   offsets : nseg+1 int64 values, device memory, non-decreasing;
 *             offsets[0] need not be 0.  Not checked here (see
 *             exsum_check_offsets).
 *   nseg    : number of segments, 0 <= nseg < 2^31.  An empty segment sums
 *             to +0.0.
 *   out     : nseg binary64 results, device memory.
 * Nothing is planned on the host and nothing synchronises; after one call on
 * a stream (which allocates that stream's workspace) the call may be
 * captured in a HIP graph.
 */
int exsum_segmented_f64(const double *x, const int64_t *offsets, int64_t nseg,
                        double *out, void *stream);

/*
 * exsum_check_offsets -- validate the offsets of a segmented call (a
 * debugging aid: exsum_segmented_f64 trusts its offsets, and offsets past the
 * end of x make it read outside x).
 *   offsets   : nseg+1 int64 values, device memory.
 *   nseg      : number of segments, 0 <= nseg < 2^31.
 *   n         : the number of terms in x, or -1 to skip that bound.
 *   first_bad : one int64, device memory; receives -1 if offsets[0] >= 0,
 *               the offsets do not decrease and offsets[nseg] <= n (when
 *               n >= 0), else the smallest segment index i whose bounds
 *               break one of these (i = 0 for offsets[0] < 0, i = nseg-1 for
 *               offsets[nseg] > n).
 * Asynchronous on `stream`; allocates nothing, so it may be captured in a
 * HIP graph.  Returns EXSUM_EINVAL for nseg out of range or NULL pointers.
 */
int exsum_check_offsets(const int64_t *offsets, int64_t nseg, int64_t n, int64_t *first_bad, void *stream);

/*
 * exsum_inexact_f64 -- out[0] = an ordinary (rounded at every addition)
 * binary64 sum of x[0..n), reduced as a tree over the same launch geometry.
 * Not exact: it is the comparator of the paper's Performance evaluations
 * (its "simple unordered" summation), here to price exactness on the GPU.
 * Deterministic for a fixed n and device.
 */
int exsum_inexact_f64(const double *x, int64_t n, double *out, void *stream);

/*
 * Launch configuration of the exact sum (tuning and testing).  Every field
 * changes only speed, never a result bit.
 *   large_block : threads per workgroup of the large-accumulator kernel.
 *   large_vec   : 16-byte loads per thread per tile.
 *   large_depth : tiles of loads kept in flight per thread.
 *   large_mode  : when a large-accumulator chunk is transferred to the small
 *                 one.  0 = by count (the paper's rule: raw bit patterns are
 *                 added and a count per chunk triggers the transfer); 1 = by
 *                 carry (mantissas with their implicit bit are added and the
 *                 LDS add that wraps a chunk past 2^64 forwards the carry).
 *                 Built (block, vec, depth, mode): (256,6,3,0) (256,4,3,0)
 *                 (256,2,4,0) (512,3,2,0) (512,2,2,0) (256,4,3,1) (512,4,2,1)
 *                 (512,2,4,1) (1024,2,2,1) (1024,4,2,1).
 *   large_grid  : workgroups of the large kernel; 0 = one per compute unit.
 *   precombine  : pre-combine across a wavefront: a tile whose terms all
 *                 share one (sign, exponent) chunk is summed across the
 *                 wavefront and added with a single LDS update, and on the
 *                 rare slow path (tiles with infinities or NaNs, leftovers)
 *                 this many lanes sharing a chunk are summed first; 0
 *                 disables both.  (The binary32 kernels do not use it: their
 *                 interleaved table copies serve a shared chunk better.)
 *   small_max   : inputs with n <= small_max use the small-only kernel.
 *   small_grid  : workgroups of the small-only kernel; 0 = automatic.
 *   seg_grid    : workgroups of the segmented call's long-segment kernel,
 *                 one term range each, at most 8192.  The batch's terms are
 *                 split into ranges that shrink along the dispatch order,
 *                 from 1.8 to 0.2 times the mean, when the batch has enough
 *                 terms for every range to stay nonempty (N (G - 4) >= 5 G^2);
 *                 otherwise evenly.  0 = eight per compute unit, of which
 *                 three fit at once, so that compute units whose ranges hold
 *                 fewer long segments take more ranges, and the ranges
 *                 started last are short.
 *   seg_small_max : segments of at most this many terms (0 .. 2^20) are
 *                   summed by one wavefront with the small accumulator
 *                   alone; longer ones by workgroups with the large one
 *                   (default 20480).
 *   seg_mode    : 1 = one persistent launch: workgroups sum the long
 *                 segments of their term range, then their wavefronts claim
 *                 short segments from a device-wide cursor, longest length
 *                 class first; 0 = two launches (long segments, then short
 *                 ones on one workgroup per compute unit with an even split
 *                 of their total weight: length plus a fixed cost per
 *                 segment).
 *   seg_block   : threads per workgroup of the persistent launch: 256, 512
 *                 or 1024.
 *   seg_group   : segments per unit of the persistent launch's cursor, 1..64.
 *   seg_pad     : unused, 0.
 *   (seg_grid also sets the persistent launch's workgroups; 0 = as many
 *   per compute unit as fit: three of 256 threads, two of 512, one of 1024.)
 */
typedef struct {
    int32_t large_block;
    int32_t large_vec;
    int32_t large_depth;
    int32_t large_mode;
    int32_t large_grid;
    int32_t precombine;
    int64_t small_max;
    int32_t small_grid;
    int32_t seg_grid;
    int64_t seg_small_max;
    int32_t seg_mode;
    int32_t seg_block;
    int32_t seg_group;
    int32_t seg_pad;
} exsum_config;

/*
 * exsum_autotune -- pick the launch configuration for the current device by
 * timing candidates on synthetic inputs (10^8 terms of three exponent
 * distributions for the large-kernel variant, scored by the worst ratio to
 * the fastest candidate; lengths 512 .. 65536 for the small/large crossover;
 * two batches of 32768 lognormal segments, sigma 2 and 1.63, for the
 * segmented launch: mode, seg_small_max, seg_grid, seg_block and seg_group,
 * again scored by the worst ratio), and make the chosen configuration the
 * process configuration.  Every candidate's result bits are compared with
 * the others'; a difference (a defect: configurations change only speed)
 * returns EXSUM_EDEVICE.  Takes a few seconds and about 2.7 GB of device
 * memory, allocated and freed inside the call; synchronises `stream`.  On
 * any error the previous configuration stays in force.
 *   cache_path : if not NULL, the result is also written there as JSON
 *                (device name, architecture, compute units, configuration,
 *                the measured times), for exsum_load_tuning().
 *   report     : if report_len > 0, the same JSON, truncated to
 *                report_len - 1 bytes and NUL-terminated (host memory).
 * Changes the configuration used by concurrent calls on other threads (the
 * bits they compute are unaffected).
 */
int exsum_autotune(const char *cache_path, char *report, int64_t report_len, void *stream);

/*
 * exsum_load_tuning -- make the configuration stored by exsum_autotune() in
 * cache_path the process configuration.  EXSUM_EINVAL if the file is
 * missing or malformed, holds an out-of-range configuration, or was written
 * on a device with another name, architecture or compute-unit count than
 * the current one.
 */
int exsum_load_tuning(const char *cache_path);

/*
 * exsum_large_variants -- the (block, vec, depth, mode) shapes of the large
 * kernel this library was built with: the values exsum_set_config accepts
 * for large_block, large_vec, large_depth and large_mode.  Writes up to
 * `cap` shapes as 4 int32 each into out (host memory; may be NULL when
 * cap == 0) and the number built to *count.  Host only, no device work.
 */
int exsum_large_variants(int32_t *out, int64_t cap, int64_t *count);

/* Current configuration of the calling process (defaults until set). */
int exsum_get_config(exsum_config *cfg);
/* Replace the configuration; EXSUM_EINVAL if a field is out of range. */
int exsum_set_config(const exsum_config *cfg);

/* exsum_f64 with an explicit configuration for this call only. */
int exsum_f64_cfg(const double *x, int64_t n, double *out, void *stream,
                  const exsum_config *cfg);

/* Free every cached workspace (call with no exsum work in flight). */
int exsum_release(void);

/* ------------------------------------------------------------------------
 * Further exact reductions over the same path (same conventions, argument
 * checks and asynchrony as exsum_f64; `n` counts terms or pairs, and the
 * launch uses the small-only kernel for n <= small_max, else the large
 * kernel in its default variant).
 * ------------------------------------------------------------------------ */

/* out[0] = sum of x[i]*x[i], each product first rounded to binary64 by the
   IEEE multiply, then summed exactly and rounded once (the squared norm of
   the Performance evaluations). */
int exsum_sqnorm_f64(const double *x, int64_t n, double *out, void *stream);

/* out[0] = sum of x[i]*y[i], each product first rounded to binary64, then
   summed exactly and rounded once (the paper's dot product).  x and y need
   not share an alignment.  A NaN product's bits are those the device's IEEE
   multiply gives (the sign is ignored, as for any NaN term). */
int exsum_dot_f64(const double *x, const double *y, int64_t n, double *out, void *stream);

/* out[0] = (exact sum of x[0..n)) / n, rounded once to binary64, ties to
   even (Discussion: a mean that is correctly rounded).  n == 0 gives +0, as
   does a mean that rounds to zero. */
int exsum_mean_f64(const double *x, int64_t n, double *out, void *stream);

/* out[0] = the exact sum of the binary32 terms x[0..n), rounded once to
   binary32 (the single-precision variant of the Introduction).  Terms are
   converted exactly; a NaN result carries the largest binary32 NaN payload
   with the quiet bit set; +Inf with -Inf gives 0x7FC00000; an exact zero
   gives +0.  x and out are float device pointers. */
int exsum_f32(const float *x, int64_t n, float *out, void *stream);

/* out[0] = the exact dot product of two binary32 vectors, rounded once to
   binary32 (Introduction: the single-precision variant; Performance
   evaluations: the dot product).  Each product is formed exactly in
   binary64 (the operands convert exactly, and 24-bit by 24-bit mantissas
   fit in 53 bits), the products are summed exactly, and the sum is rounded
   to nearest, ties to even.  Unlike a binary32 sum, a nonzero result can be
   smaller than half binary32's smallest denormal; it rounds to +0.0, as the
   mean does.  x and y need not share an alignment.  A NaN product's payload
   (from the device's binary64 multiply) maps back to binary32 by dropping
   its 29 low bits. */
int exsum_dot_f32(const float *x, const float *y, int64_t n, float *out, void *stream);

/* ------------------------------------------------------------------------
 * Streaming, mergeable accumulator (Discussion: parts of a sum are summed
 * separately and their small superaccumulators added).  The state is
 * EXSUM_ACC_BYTES of caller-owned device memory, 64-byte aligned: 67
 * signed 64-bit chunks of the small superaccumulator (chunk i weighs
 * 2^(32i-1075), kept below 2^33 in magnitude after every update), a pad
 * word, the +Inf and -Inf flags, the largest NaN pattern, and padding.
 * Updates on one stream are ordered; updates of one state from different
 * streams must be ordered by the caller.  Rounding reads the state and does
 * not change it, so a running sum can be read at any time.
 * ------------------------------------------------------------------------ */
#define EXSUM_ACC_BYTES 576

/* Set the state to the empty sum. */
int exsum_acc_zero(void *acc, void *stream);
/* Add the exact sum of x[0..n) (not rounded). */
int exsum_acc_add_f64(void *acc, const double *x, int64_t n, void *stream);
/* dst += src (two different states). */
int exsum_acc_merge(void *dst, const void *src, void *stream);
/* out[0] = the state's value rounded once to binary64 (as exsum_f64). */
int exsum_acc_round_f64(const void *acc, double *out, void *stream);

/* ------------------------------------------------------------------------
 * Serving loop: many independent exact sums (requests) arriving over time,
 * served by continuous batching on one stream.
 *
 * A request is a range of device memory (x, n) and a device slot for its
 * one binary64 result; its result is the same bits as exsum_f64(x, n) gives
 * (the exact sum, rounded once), whatever else is in flight.  Each step
 * takes a budget of terms from the active requests in arrival order: first
 * one piece (up to piece_terms) for every active request, then more pieces
 * for the oldest requests; a request of at most piece_terms terms is never
 * split.  One kernel launch sums the step's pieces; a request cut into
 * pieces adds them into an integer accumulator slot (Discussion, on adding
 * the small superaccumulators of parts) and the last piece rounds.  A
 * request is complete when the step holding its last piece has completed on
 * the stream (observed with events by exsum_server_poll).
 *
 * The server owns: its accumulator slots (max_slots x 576 bytes of device
 * memory), pinned host and device piece tables (max_inflight x max_pieces x
 * 32 bytes each) and events, all allocated by exsum_server_create.
 * Admission (Discussion, on the small superaccumulators of parts: each part
 * in flight holds one): a request cut into pieces needs a free slot and room
 * in mem_budget; shorter requests are admitted at once and wait only for
 * room in a step.  LDS is not a separate limit: a step's launch holds at
 * most one workgroup per compute unit, each within the unit's LDS.  The
 * caller owns x and out and keeps them alive until the request completes.
 * A server is used from one host thread at a time.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t step_terms;    /* term budget of one step, >= piece_terms (default 2^27) */
    int64_t piece_terms;   /* most terms in one piece, >= 1 (default 2^16) */
    int64_t short_max;     /* pieces of at most this many terms are summed by one
                              wavefront, the others by one workgroup (default 4096) */
    int32_t max_slots;     /* requests cut into pieces that may be active at once,
                              1 .. 2^20 (default 4096); more wait for admission */
    int32_t max_pieces;    /* most pieces in one step, 1 .. 2^20 (default 16384) */
    int32_t max_inflight;  /* steps queued on the stream at once, 1 .. 64 (default 2) */
    int32_t precombine;    /* as in exsum_config (default 16) */
    int64_t mem_budget;    /* bytes of device memory that admitted requests may hold
                              at once: 576 per accumulator slot of a request cut
                              into pieces, plus 32 per piece descriptor of the
                              steps queued on the stream.  A long request is
                              admitted only when its slot and one piece fit beside
                              what is already held, and a step's pieces are capped
                              by what is left.  0 = no limit beyond max_slots and
                              max_pieces (default); else >= 608 */
} exsum_server_config;

typedef struct exsum_server exsum_server;

/* Fill *cfg with the defaults. */
int exsum_server_default_config(exsum_server_config *cfg);

/* Create a server on the current device that launches on `stream`.
   EXSUM_EINVAL for a bad configuration, EXSUM_ENOMEM / EXSUM_EDEVICE if an
   allocation fails (nothing is left allocated then). */
int exsum_server_create(const exsum_server_config *cfg, void *stream, exsum_server **out);

/* Wait for the server's work to finish and free everything it owns. */
int exsum_server_destroy(exsum_server *srv);

/* Queue one request: the exact sum of x[0..n) into *out (device pointers).
   *id receives the request's id (0, 1, 2, ... in submission order).
   EXSUM_EINVAL for n < 0, n >= 2^40, a NULL out, or a NULL x with n > 0. */
int exsum_server_submit(exsum_server *srv, const double *x, int64_t n, double *out, int64_t *id);

/* Plan and launch one step if there is work and fewer than max_inflight
   steps are queued; *launched = number of pieces launched (0 if none).
   Never blocks. */
int exsum_server_step(exsum_server *srv, int64_t *launched);

/* Ids of requests completed since the previous call, in completion order:
   up to `max` into ids[0..*count).  Never blocks. */
int exsum_server_poll(exsum_server *srv, int64_t *ids, int64_t max, int64_t *count);

/* Step and wait until every submitted request is complete (completed ids
   stay available to exsum_server_poll). */
int exsum_server_drain(exsum_server *srv);

/* Requests submitted and not yet reported complete. */
int exsum_server_pending(exsum_server *srv, int64_t *count);

/* Replay a trace in real time through the server.  Request i sums
   pool[starts[i] .. starts[i]+lens[i]) into out[i] and arrives arrival_s[i]
   seconds after the replay starts (non-decreasing).  latency_s[i] receives
   the time from its arrival to the host observing its completion;
   *makespan_s the time from the start to the last completion.  pool and out
   are device memory; starts, lens, arrival_s and latency_s host memory. */
int exsum_server_replay(exsum_server *srv, const double *pool, const int64_t *starts, const int64_t *lens,
                        const double *arrival_s, int64_t nreq, double *out, double *latency_s,
                        double *makespan_s);

/* The same trace served without batching: each request is one exsum_f64
   call, launched on `stream` when it arrives (first in, first out). */
int exsum_serial_replay(const double *pool, const int64_t *starts, const int64_t *lens,
                        const double *arrival_s, int64_t nreq, double *out, void *stream,
                        double *latency_s, double *makespan_s);

/* The server's scheduling plan, on the host only (no device work): requests
   of the given lengths all submitted at once, steps planned until every
   term is scheduled, each step's slots released before the next.  Writes
   up to `cap` pieces (request, offset, length, step, slot, expected count
   or 0xFFFFFFFF for a piece of a step that does not complete its request)
   and the total number of pieces to *count. */
int exsum_server_plan(const exsum_server_config *cfg, const int64_t *lens, int64_t nreq, int64_t cap,
                      int64_t *req, int64_t *off, int64_t *len, int64_t *step, int32_t *slot,
                      uint32_t *expected, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* EXSUM_H */
