// kernels_seg.hip -- many exact sums of uneven length (gfx950): two launches
// on the caller's stream that write disjoint outputs.
//
// Short segments (at most small_max terms, empty ones included) are summed
// whole by single wavefronts with the small-superaccumulator body and
// rounded where they are summed (the Performance evaluations find the small
// method the faster one for short sums).  Wave v of W takes segments
// [nseg*v/W, nseg*(v+1)/W) and skips the long ones; every wave's work is
// thus at most ceil(nseg/W) * small_max terms.  The kernel is light (small
// LDS and register footprint), so many wavefronts share a compute unit and
// hide each other's memory latency.
//
// Long segments are summed by workgroups with the large accumulator (carry
// mode).  Workgroup w of G takes the terms [o0 + N*w/G, o0 + N*(w+1)/G)
// (N = offsets[nseg] - offsets[0]; G is the grid capped at N, so that no
// range is empty), so every workgroup reads the same number of bytes of the
// concatenated input whatever the lengths.  It finds the segment holding its
// first term with a wavefront-wide search of the offsets and walks the long
// segments that meet its range in batches of up to 256.  A segment inside
// one range is rounded by that workgroup; a segment cut by range boundaries
// adds its pieces into the accumulator slot of the first workgroup that
// holds one, a ticket counts the pieces (exactly the workgroups
// wg_of(first) .. wg_of(last)), and the piece that completes the count
// rounds.
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
  unsigned int nb;                     // segments of this batch that meet the range
  long long first;                     // first segment of the range
};

template <int BLOCK, int VEC, int DEPTH>
__global__ __launch_bounds__(BLOCK) void seg_long_kernel(const double *__restrict__ x,
                                                         const long long *__restrict__ offsets, long long nseg,
                                                         double *__restrict__ out, GlobalAcc *__restrict__ accs,
                                                         long long small_max, int precombine) {
  __shared__ SegShared S;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // all lanes active here
  const long long o0 = offsets[0], oN = offsets[nseg];
  const long long N = oN - o0;
  if (N <= 0) return;                                   // no terms: only empty (short) segments
  // at most one workgroup per term, so every range is nonempty and a
  // segment's pieces are exactly the workgroups wg_of(first) .. wg_of(last)
  const long long G = ((long long)gridDim.x < N) ? (long long)gridDim.x : N;
  const long long w = blockIdx.x;
  if (w >= G) return;                                   // whole workgroup, before any barrier
  large_init(S.L, tid, BLOCK);
  const long long lo_w = o0 + N * w / G, hi_w = o0 + N * (w + 1) / G;

  // first segment: i = j - 1 for the smallest j in [1, nseg] with
  // offsets[j] > lo_w, the segment that holds term lo_w (offsets[nseg] > lo_w
  // qualifies).  Wave 0 cuts the candidate interval [lo, hi] 64 ways per round.
  if (wave == 0) {
    long long lo = 1, hi = nseg;
    while (hi - lo > 63) {
      const long long span = hi - lo;
      const long long p = lo + span * lane / 64;       // < hi
      const unsigned long long m = __ballot(offsets[p] > lo_w);
      const int f = m ? (__ffsll((long long)m) - 1) : 64;
      const long long nlo = (f == 0) ? lo : lo + span * (f - 1) / 64 + 1;
      const long long nhi = (f == 64) ? hi : lo + span * f / 64;
      lo = nlo;
      hi = nhi;
    }
    const long long p = lo + lane;
    const long long pc = p <= hi ? p : hi;
    const unsigned long long m = __ballot(p <= hi && offsets[pc] > lo_w);
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
    for (int k = tid; k < cnt; k += BLOCK)
      if (S.off[k] >= hi_w) atomicMin(&S.nb, (unsigned int)k);
    __syncthreads();
    const int nb = (int)S.nb;
    for (int k = 0; k < nb; k++) {
      const long long s0 = S.off[k], s1 = S.off[k + 1];
      if (s1 - s0 <= small_max) continue;              // short: the other kernel's
      const long long a = s0 > lo_w ? s0 : lo_w;
      const long long b = s1 < hi_w ? s1 : hi_w;
      accumulate_range<BLOCK, VEC, DEPTH, kCarryMode>(S.L, SrcF64{x}, a, b, precombine, tile);
      final_flush<BLOCK, true, kCarryMode>(S.L);
      const bool split = (s0 < lo_w) || (s1 > hi_w);
      unsigned int expected = 1;
      GlobalAcc *g = nullptr;
      if (split) {
        const long long w1 = wg_of(s0 - o0, N, G);
        expected = (unsigned int)(wg_of(s1 - 1 - o0, N, G) - w1 + 1);
        g = &accs[w1];
      }
      merge_and_round(S.L.small, S.L.spec, &S.L.ticket, g, expected, &out[i + k]);
      if (tid < 68) S.L.small[tid] = 0;
      if (tid < 3) S.L.spec[tid] = 0ull;
      __syncthreads();
    }
    if (nb < cnt) break;                               // the range ended inside this batch
    i += cnt;
    __syncthreads();
  }
}

constexpr int kShortCopies = 8;

template <int NW>
struct ShortShared {
  long long acc[NW][small_acc_words<kShortCopies>()];
  unsigned long long spec[NW][4];
};

// Short segments, one wavefront each.  Offsets are read 64 at a time into
// the lanes and taken one by one with readlane.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void seg_short_kernel(const double *__restrict__ x,
                                                          const long long *__restrict__ offsets, long long nseg,
                                                          double *__restrict__ out, long long small_max) {
  constexpr int NW = BLOCK / 64;
  __shared__ ShortShared<NW> S;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);   // all lanes active here
  long long *acc = S.acc[wave];
  unsigned long long *spec = S.spec[wave];
  const long long W = (long long)gridDim.x * NW;
  const long long v = (long long)blockIdx.x * NW + wave;
  const long long i1 = nseg * (v + 1) / W;
  for (long long i0 = nseg * v / W; i0 < i1; i0 += 63) {
    long long idx = i0 + lane;
    idx = idx < nseg ? idx : nseg;
    const unsigned long long ov = (unsigned long long)offsets[idx];
    const int cnt = (int)((i1 - i0 < 63) ? (i1 - i0) : 63);
    for (int k = 0; k < cnt; k++) {
      const long long s0 = (long long)readlane_u64(ov, k);
      const long long s1 = (long long)readlane_u64(ov, k + 1);
      if (s1 - s0 > small_max) continue;               // long: the other kernel's
      small_wave_zero<kShortCopies>(acc, spec, lane);
      small_wave_accumulate<kShortCopies>(acc, spec, SrcF64{x}, s0, s1, lane);
      wave_merge_and_round(acc, spec, nullptr, 1u, &out[i0 + k], lane);
    }
  }
}

constexpr int kShortBlock = 256;

}  // namespace

hipError_t launch_segmented(const double *x, const int64_t *offsets, int64_t nseg, double *out, GlobalAcc *accs,
                            hipStream_t s, int grid, int short_grid, int64_t small_max, int precombine) {
  if (grid < 1) grid = 1;
  if (short_grid < 1) short_grid = 1;
  hipLaunchKernelGGL((seg_short_kernel<kShortBlock>), dim3(short_grid), dim3(kShortBlock), 0, s, x,
                     (const long long *)offsets, (long long)nseg, out, (long long)small_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((seg_long_kernel<512, 4, 2>), dim3(grid), dim3(512), 0, s, x, (const long long *)offsets,
                     (long long)nseg, out, accs, (long long)small_max, precombine);
  return hipGetLastError();
}

int seg_short_waves_per_block() { return kShortBlock / 64; }

size_t global_acc_bytes() { return sizeof(GlobalAcc); }

}  // namespace exsum
