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
 * workspace (merge rows, accumulators and tickets, about 10 MiB) that it
 * allocates on the first call
 * on that stream, zero-initialises synchronously, and keeps clean itself
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
 * exsum_segmented_f64 -- out[i] = exact sum of x[offsets[i] .. offsets[i+1])
 * for 0 <= i < nseg, all in one persistent launch.
 *
 * Many independent exact sums (same definition as exsum_f64), one launch.
 * Workgroups take equal shares of the concatenated terms; each piece of a
 * segment takes the small-superaccumulator path (one wavefront) or the
 * large-plus-small path (a workgroup) by its length (Performance
 * evaluations: the small method wins for short sums, the large one for long
 * sums); a segment cut by workgroup boundaries is merged from its pieces.
 *   x       : terms, device memory.
 *   offsets : nseg+1 int64 values, device memory, non-decreasing;
 *             offsets[0] need not be 0.  Not checked on the device.
 *   nseg    : number of segments, >= 0.  An empty segment sums to +0.0.
 *   out     : nseg binary64 results, device memory.
 * Nothing is planned on the host and nothing synchronises; after one call on
 * a stream (which allocates that stream's workspace) the call may be
 * captured in a HIP graph.
 */
int exsum_segmented_f64(const double *x, const int64_t *offsets, int64_t nseg,
                        double *out, void *stream);

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
 *   precombine  : lanes of a wavefront that must share one (sign, exponent)
 *                 chunk before they are first summed across the wavefront and
 *                 added with a single LDS update; 0 disables the pre-combine.
 *   small_max   : inputs with n <= small_max use the small-only kernel.
 *   small_grid  : workgroups of the small-only kernel; 0 = automatic.
 *   seg_grid    : workgroups of the segmented kernel; 0 = one per compute unit.
 *   seg_small_max : segment pieces of at most this many terms are summed by
 *                   one wavefront with the small accumulator alone; longer
 *                   ones by a workgroup with the large accumulator.
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
} exsum_config;

/* Current configuration of the calling process (defaults until set). */
int exsum_get_config(exsum_config *cfg);
/* Replace the configuration; EXSUM_EINVAL if a field is out of range. */
int exsum_set_config(const exsum_config *cfg);

/* exsum_f64 with an explicit configuration for this call only. */
int exsum_f64_cfg(const double *x, int64_t n, double *out, void *stream,
                  const exsum_config *cfg);

/* Free every cached workspace (call with no exsum work in flight). */
int exsum_release(void);

#ifdef __cplusplus
}
#endif

#endif /* EXSUM_H */
