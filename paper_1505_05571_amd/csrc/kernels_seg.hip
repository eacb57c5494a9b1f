// kernels_seg.hip -- many exact sums of uneven length in one launch (gfx950).
//
// The segments x[offsets[i] .. offsets[i+1]) tile the range [offsets[0],
// offsets[nseg]) of x.  Workgroup w of G takes the terms
// [o0 + N*w/G, o0 + N*(w+1)/G)  (N = offsets[nseg] - offsets[0]; G is the
// grid capped at N, so that no range is empty),
// so every workgroup reads the same number of bytes whatever the lengths,
// and no planning pass or work queue is needed.  It finds its first segment
// with a wavefront-wide search of the offsets and walks the segments that
// meet its range in batches of up to 256:
//   * pieces of at most small_max terms are summed by single wavefronts with
//     the small-superaccumulator body, wave v taking pieces v, v + NW, ...
//     of the batch (the Performance evaluations find the small method the
//     faster one for short sums).  The piece index is a plain scalar loop
//     counter: a counter claimed by one lane and broadcast with
//     readfirstlane is not safe here, since the compiler may route the other
//     lanes round the loop without that lane;
//   * longer pieces are summed by the whole workgroup with the large
//     accumulator body (carry-triggered transfers, no tile barriers).
// A segment inside one workgroup's range is rounded by that workgroup.  A
// segment cut by range boundaries (at most one per boundary) is merged
// through the accumulator slot of the first workgroup that meets it, with a
// ticket counting its pieces; the piece that completes it rounds it.  An
// empty segment is written (+0.0) by the workgroup whose range holds its
// position (the last workgroup for position offsets[nseg]).
#include "exsum_blocks.h"
#include "exsum_internal.h"

namespace exsum {
namespace {

constexpr int kSegBatch = 256;

// Workgroup of G whose term range contains relative position p (0 <= p < N):
// the largest w with floor(N*w/G) <= p.
__device__ __forceinline__ long long wg_of(long long p, long long N, long long G) {
  return ((p + 1) * G + N - 1) / N - 1;
}

struct SegShared {
  LargeShared L;
  long long off[kSegBatch + 1];        // a batch of segment offsets
  long long wacc[16][68];              // per-wave small accumulators
  unsigned long long wspec[16][4];     // per-wave side words
  unsigned int wD[16][70];             // per-wave rounding scratch
  unsigned int nb;                     // segments of this batch that meet the range
  long long first;                     // first segment of the range
};

template <int BLOCK, int VEC, int DEPTH>
__global__ __launch_bounds__(BLOCK) void seg_kernel(const double *__restrict__ x,
                                                    const long long *__restrict__ offsets, long long nseg,
                                                    double *__restrict__ out, GlobalAcc *__restrict__ accs,
                                                    long long small_max, int precombine) {
  static_assert(BLOCK / 64 <= 16, "per-wave LDS sized for 16 waves");
  __shared__ SegShared S;
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // all lanes active here
  const long long o0 = offsets[0], oN = offsets[nseg];
  const long long N = oN - o0;
  // at most one workgroup per term, so every range is nonempty and a
  // segment's pieces are exactly the workgroups wg_of(first) .. wg_of(last)
  const long long G = ((long long)gridDim.x < N) ? (long long)gridDim.x : (N > 0 ? N : 1);
  const long long w = blockIdx.x;
  if (w >= G) return;                                   // whole workgroup, before any barrier
  large_init(S.L, tid, BLOCK);
  const long long lo_w = o0 + N * w / G, hi_w = o0 + N * (w + 1) / G;
  const bool last_wg = (w == G - 1);

  // first segment: i = j - 1 for the smallest j in [1, nseg] with
  // offsets[j] >= lo_w (offsets[nseg] qualifies).  Wave 0 cuts the candidate
  // interval [lo, hi] 64 ways per round.
  if (wave == 0) {
    long long lo = 1, hi = nseg;
    while (hi - lo > 63) {
      const long long span = hi - lo;
      const long long p = lo + span * lane / 64;       // < hi
      const unsigned long long m = __ballot(offsets[p] >= lo_w);
      const int f = m ? (__ffsll((long long)m) - 1) : 64;
      const long long nlo = (f == 0) ? lo : lo + span * (f - 1) / 64 + 1;
      const long long nhi = (f == 64) ? hi : lo + span * f / 64;
      lo = nlo;
      hi = nhi;
    }
    const long long p = lo + lane;
    const long long pc = p <= hi ? p : hi;
    const unsigned long long m = __ballot(p <= hi && offsets[pc] >= lo_w);
    const long long j = m ? lo + (__ffsll((long long)m) - 1) : hi;
    if (lane == 0) S.first = j - 1;
  }
  __syncthreads();
  long long i = S.first;
  unsigned int tile = 0;

  while (i < nseg) {
    const int cnt = (int)((nseg - i < kSegBatch) ? (nseg - i) : kSegBatch);
    for (int k = tid; k <= cnt; k += BLOCK) S.off[k] = offsets[i + k];
    if (tid == 0) S.nb = (unsigned int)cnt;
    __syncthreads();
    // the segments of the batch that meet the range form a prefix
    for (int k = tid; k < cnt; k += BLOCK) {
      const long long s0 = S.off[k];
      const bool beyond = last_wg ? (s0 > hi_w) : (s0 >= hi_w);
      if (beyond) atomicMin(&S.nb, (unsigned int)k);
    }
    __syncthreads();
    const int nb = (int)S.nb;

    // wave phase: short pieces
    {
      long long *acc = S.wacc[wave];
      unsigned long long *spec = S.wspec[wave];
      unsigned int *D = S.wD[wave];
      for (int k = wave; k < nb; k += NW) {
        const long long s0 = S.off[k], s1 = S.off[k + 1];
        const long long a = s0 > lo_w ? s0 : lo_w;
        const long long b = s1 < hi_w ? s1 : hi_w;
        if (s0 != s1 && a >= b) continue;              // a nonempty segment this range misses
        if (b - a > small_max) continue;               // a long piece: workgroup phase
        acc[lane] = 0;
        if (lane < 4) acc[64 + lane] = 0;
        if (lane < 3) spec[lane] = 0ull;
        small_wave_accumulate(acc, spec, x, a, b, lane);
        const bool split = (s0 < lo_w) || (s1 > hi_w);
        unsigned int expected = 1;
        GlobalAcc *g = nullptr;
        if (split) {
          const long long w1 = wg_of(s0 - o0, N, G);
          expected = (unsigned int)(wg_of(s1 - 1 - o0, N, G) - w1 + 1);
          g = &accs[w1];
        }
        wave_merge_and_round(acc, spec, D, g, expected, &out[i + k], lane);
      }
    }
    __syncthreads();

    // workgroup phase: long pieces, in order
    for (int k = 0; k < nb; k++) {
      const long long s0 = S.off[k], s1 = S.off[k + 1];
      const long long a = s0 > lo_w ? s0 : lo_w;
      const long long b = s1 < hi_w ? s1 : hi_w;
      if (b - a <= small_max) continue;
      accumulate_range<BLOCK, VEC, DEPTH, kCarryMode>(S.L, x, a, b, precombine, tile);
      final_flush<BLOCK, true, kCarryMode>(S.L);
      const bool split = (s0 < lo_w) || (s1 > hi_w);
      unsigned int expected = 1;
      GlobalAcc *g = nullptr;
      if (split) {
        const long long w1 = wg_of(s0 - o0, N, G);
        expected = (unsigned int)(wg_of(s1 - 1 - o0, N, G) - w1 + 1);
        g = &accs[w1];
      }
      merge_and_round(S.L.small, S.L.spec, &S.L.ticket, S.L.D, g, expected, &out[i + k]);
      if (tid < 68) S.L.small[tid] = 0;
      if (tid < 3) S.L.spec[tid] = 0ull;
      __syncthreads();
    }
    if (nb < cnt) break;                               // the range ended inside this batch
    i += cnt;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_segmented(const double *x, const int64_t *offsets, int64_t nseg, double *out, GlobalAcc *accs,
                            hipStream_t s, int grid, int64_t small_max, int precombine) {
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((seg_kernel<512, 4, 2>), dim3(grid), dim3(512), 0, s, x, (const long long *)offsets,
                     (long long)nseg, out, accs, (long long)small_max, precombine);
  return hipGetLastError();
}

size_t global_acc_bytes() { return sizeof(GlobalAcc); }

}  // namespace exsum
