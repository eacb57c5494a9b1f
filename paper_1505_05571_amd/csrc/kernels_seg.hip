// kernels_seg.hip -- many exact sums of uneven length (gfx950): two launches
// on the caller's stream that write disjoint outputs.
//
// Long segments (more than small_max terms) are summed first, by workgroups
// with the large accumulator (carry mode).  Workgroup w of G takes term range
// w of the concatenated input (N = offsets[nseg] - offsets[0] terms): the
// ranges split the terms whatever the lengths, shrinking along the dispatch
// order when N is large enough (RangeSplit), evenly otherwise.  A workgroup
// finds the segment holding its first term with a wavefront-wide search of
// the offsets and walks the long segments that meet its range in batches of
// up to 256.  A segment inside one range is rounded by that workgroup; a
// segment cut by range boundaries adds its pieces into the accumulator slot
// of the first range that holds one, a ticket counts the pieces (exactly
// the ranges range_of(first) .. range_of(last)), and the piece that
// completes the count rounds.  The same launch also sums the weights of the
// short kernel's chunks of segments, from which that kernel partitions its
// work.
//
// Short segments (at most small_max terms, empty ones included) are then
// summed whole by single wavefronts with the small-superaccumulator body and
// rounded where they are summed (the Performance evaluations find the small
// method the faster one for short sums).  One workgroup per compute unit
// takes an equal share of the total weight (terms plus a fixed cost per
// segment) and hands its segments to its wavefronts one at a time from an
// LDS counter, longest first: wavefronts of one compute unit do not progress
// at the same rate (older ones issue first), so a fixed per-wavefront split
// leaves a long tail.
#include "exsum_blocks.h"
#include "exsum_internal.h"

namespace exsum {
namespace {

constexpr int kSegBatch = 256;
// Cost of one short segment beyond its terms (the finish over its window,
// rounding, the first load's latency), in terms: the weight the short
// kernel's partition gives each segment.
constexpr long long kSegCost = 1024;

// The long-segment kernel's term ranges: range w of G is [o0 + B(w),
// o0 + B(w + 1)) with B(w) = floor(N f(w) / D), f(w) = w (5G + A (G - w)),
// D = 5 G^2, so B(0) = 0 and B(G) = N.  With A = 0 the ranges are equal;
// with A = 4 they shrink along the dispatch order from 1.8 N/G to 0.2 N/G,
// so that the ranges started last, when the chip drains, are short (a
// workgroup streams at a bounded rate, and a long range started late sets
// the end of the launch).  A = 4 is taken when N ((5 - A) G - A) >= D, which
// keeps every range nonempty (f rises by at least (5 - A) G - A per step, so
// B by more than N ((5 - A) G - A) / D - 1 >= 0); otherwise A = 0 and
// G <= N.  B is evaluated as q f + floor(r f / D) with N = q D + r, exact and
// without overflow for N < 2^62 and G <= 8192 (r f < 2^58).
struct RangeSplit {
  long long N, G, D, q, r;
  int A;
  __device__ __forceinline__ long long B(long long w) const {
    const long long f = w * (5 * G + A * (G - w));
    // floor(r f / D) from a binary64 estimate, corrected exactly (no 64-bit
    // division; r f < 2^58, so the estimate is off by a few units at most)
    const long long rf = r * f;
    long long t = (long long)((double)rf / (double)D);
    long long m = rf - t * D;
    while (m < 0) { t--; m += D; }
    while (m >= D) { t++; m -= D; }
    return q * f + t;
  }
  // The range holding relative position p (0 <= p < N): the largest w with
  // B(w) <= p, from the inverse of the quadratic, corrected exactly.
  __device__ __forceinline__ long long range_of(long long p) const {
    const double x = ((double)p + 0.5) / (double)N;
    double t = x;
    if (A) {
      const double a = A / 5.0;
      t = ((1.0 + a) - sqrt((1.0 + a) * (1.0 + a) - 4.0 * a * x)) / (2.0 * a);
    }
    long long w = (long long)(t * (double)G);
    w = w < 0 ? 0 : (w > G - 1 ? G - 1 : w);
    while (w > 0 && B(w) > p) w--;
    while (w + 1 < G && B(w + 1) <= p) w++;
    return w;
  }
};
__device__ __forceinline__ RangeSplit range_split(long long N, long long grid, bool guided) {
  RangeSplit R;
  R.N = N;
  R.A = 0;
  R.G = grid < N ? grid : N;
  // N (G - 4) >= 5 G^2, as N >= ceil(5 G^2 / (G - 4)) (no overflow)
  if (guided && grid > 4 && N >= (5 * grid * grid + grid - 5) / (grid - 4)) {
    R.A = 4;
    R.G = grid;
  }
  R.D = 5 * R.G * R.G;
  R.q = N / R.D;
  R.r = N % R.D;
  return R;
}

struct SegShared {
  LargeShared L;
  long long off[kSegBatch + 1];        // a batch of segment offsets
  unsigned int nb;                     // segments of this batch that meet the range
  long long first;                     // first segment of the range
  long long split[6];                  // the term split (RangeSplit), read back where needed
  long long red[16];                   // wave partial sums
};

// The long segments meeting workgroup w's term range [o0 + N*w/G,
// o0 + N*(w+1)/G) of G = min(grid, N) workgroups, summed with the large
// accumulator; a segment inside the range is rounded here, a segment cut by
// range boundaries adds its piece into the slot of its first workgroup and
// the piece that completes the ticket count rounds.  Called by every thread
// of the workgroup; returns at once (uniformly) when there are no terms or
// w >= G.
template <int BLOCK, int VEC, int DEPTH>
__device__ __forceinline__ void long_phase(SegShared &S, const double *__restrict__ x,
                                           const long long *__restrict__ offsets, long long nseg,
                                           double *__restrict__ out, GlobalAcc *__restrict__ accs,
                                           long long small_max, int precombine, bool guided) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // all lanes active here
  const long long o0 = offsets[0], oN = offsets[nseg];
  const long long N = oN - o0;
  if (N <= 0) return;                                   // no terms: only empty (short) segments
  // every range is nonempty, so a segment's pieces are exactly the ranges
  // range_of(first) .. range_of(last)
  long long lo_w, hi_w;
  {
    const RangeSplit RS = range_split(N, (long long)gridDim.x, guided);
    const long long w = blockIdx.x;
    if (w >= RS.G) return;                              // whole workgroup, before any barrier
    lo_w = o0 + RS.B(w);
    hi_w = o0 + RS.B(w + 1);
    // kept in LDS, not in registers through the streaming loop
    if (tid == 0) {
      S.split[0] = RS.N; S.split[1] = RS.G; S.split[2] = RS.D;
      S.split[3] = RS.q; S.split[4] = RS.r; S.split[5] = RS.A;
    }
  }
  large_init(S.L, tid, BLOCK);

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
  const SrcF64 src{x};
  LargeRange<VEC, DEPTH, SrcF64> R;

  while (i < nseg) {
    const int cnt = (int)((nseg - i < kSegBatch) ? (nseg - i) : kSegBatch);
    for (int k = tid; k <= cnt; k += BLOCK) S.off[k] = offsets[i + k];
    if (tid == 0) S.nb = (unsigned int)cnt;
    __syncthreads();
    // the segments of the batch that meet the range form a prefix
    for (int k = tid; k < cnt; k += BLOCK)
      if (S.off[k] >= hi_w) atomicMin(&S.nb, (unsigned int)k);
    __syncthreads();
    // every value that steers the loop below is read from LDS through
    // readfirstlane, so the compiler sees it wave-uniform (the loop holds
    // workgroup barriers)
    const int nb = __builtin_amdgcn_readfirstlane((int)S.nb);
    // the next long segment of the batch from k on (short ones are summed
    // elsewhere), and its piece in this range
    const auto next_long = [&](int k) {
      while (k < nb && uniform_i64(S.off[k + 1]) - uniform_i64(S.off[k]) <= small_max) k++;
      return k;
    };
    const auto piece_begin = [&](int k) {
      const long long s0 = uniform_i64(S.off[k]), s1 = uniform_i64(S.off[k + 1]);
      large_range_begin<BLOCK>(R, src, s0 > lo_w ? s0 : lo_w, s1 < hi_w ? s1 : hi_w);
    };
    int k = next_long(0);
    if (k < nb) piece_begin(k);
    while (k < nb) {
      const long long s0 = uniform_i64(S.off[k]), s1 = uniform_i64(S.off[k + 1]);
      large_range_add<BLOCK, VEC, DEPTH, kCarryMode>(S.L, R, src, precombine, tile);
      // the next piece's first loads fly while this one is flushed and rounded
      const int kn = next_long(k + 1);
      if (kn < nb) piece_begin(kn);
      final_flush<BLOCK, true, kCarryMode>(S.L);
      const bool split = (s0 < lo_w) || (s1 > hi_w);
      unsigned int expected = 1;
      GlobalAcc *g = nullptr;
      if (split) {
        // the ranges of the segment's first and last terms (this range's own
        // index where the segment starts or ends in it)
        RangeSplit RS;
        RS.N = uniform_i64(S.split[0]); RS.G = uniform_i64(S.split[1]); RS.D = uniform_i64(S.split[2]);
        RS.q = uniform_i64(S.split[3]); RS.r = uniform_i64(S.split[4]); RS.A = (int)uniform_i64(S.split[5]);
        const long long w = blockIdx.x;
        const long long w1 = s0 >= lo_w ? w : RS.range_of(s0 - o0);
        const long long wl = s1 <= hi_w ? w : RS.range_of(s1 - 1 - o0);
        expected = (unsigned int)(wl - w1 + 1);
        g = &accs[w1];
      }
      merge_and_round(S.L.small, S.L.spec, &S.L.ticket, g, expected, &out[i + k]);
      if (tid < 68) S.L.small[tid] = 0;
      if (tid < 3) S.L.spec[tid] = 0ull;
      __syncthreads();
      k = kn;
    }
    if (nb < cnt) break;                               // the range ended inside this batch
    i += cnt;
    __syncthreads();
  }
}

template <int BLOCK, int VEC, int DEPTH>
__global__ __launch_bounds__(BLOCK) void seg_long_kernel(const double *__restrict__ x,
                                                         const long long *__restrict__ offsets, long long nseg,
                                                         double *__restrict__ out, GlobalAcc *__restrict__ accs,
                                                         long long small_max, int precombine,
                                                         long long *__restrict__ chunks, int nchunks) {
  __shared__ SegShared S;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // all lanes active here
  if (chunks) {
    // weights of the short kernel's chunks (segments [k*nseg/C, (k+1)*nseg/C))
    for (long long k = blockIdx.x; k < nchunks; k += gridDim.x) {
      const long long c0 = k * nseg / nchunks, c1 = (k + 1) * nseg / nchunks;
      long long t = 0;
      for (long long i = c0 + tid; i < c1; i += BLOCK) {
        const long long len = offsets[i + 1] - offsets[i];
        if (len <= small_max) t += len + kSegCost;
      }
      t = wave_sum_i64(t);
      if (lane == 0) S.red[wave] = t;
      __syncthreads();
      if (tid == 0) {
        long long u = 0;
        for (int w = 0; w < BLOCK / 64; w++) u += S.red[w];
        chunks[k] = u;
      }
      __syncthreads();
    }
  }
  long_phase<BLOCK, VEC, DEPTH>(S, x, offsets, nseg, out, accs, small_max, precombine, true);
}

constexpr int kShortCopies = 16;
constexpr int kShortBlock = 1024;      // one workgroup per compute unit
// Long segments: workgroups of 256 threads, several per compute unit, so
// that one streams while another flushes and rounds a segment (measured on
// the 65,536-segment batch: 436 us with two against 480-530 us for one
// 512-thread workgroup per compute unit).
constexpr int kLongBlock = 256;
// Length classes: a round's segments are handed out longest class first.
constexpr long long kClassA = 4096, kClassB = 512;

// Inclusive sum over a workgroup (BLOCK threads, every thread calls it).
// red: BLOCK/64 words of LDS.
template <int BLOCK>
__device__ __forceinline__ long long block_incl_scan(long long v, long long *red, long long &total) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const long long u = (long long)__shfl_up((unsigned long long)v, d, 64);
    if (lane >= d) v += u;
  }
  __syncthreads();
  if (lane == 63) red[wave] = v;
  __syncthreads();
  long long before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; w++) {
    const long long r = red[w];
    if (w < wave) before += r;
    all += r;
  }
  total = uniform_i64(all);
  return v + before;
}

template <int BLOCK>
struct ShortShared {
  long long acc[BLOCK / 64][small_acc_words<kShortCopies>()];
  unsigned long long spec[BLOCK / 64][4];
  long long lo[BLOCK + 1];             // a round's segment starts and its end (also scan scratch)
  int ord[BLOCK];                      // the round's short segments, longest class first
  int ccount[3][BLOCK / 64];
  int cnt;                             // 64 x the next entry of ord to hand out
  long long red[BLOCK / 64];
  int kk[2];                           // the chunks holding the range's two ends
  unsigned long long f[2];             // the range's two ends
};

// Weight of segment i in the partition of the short kernel's work.
__device__ __forceinline__ long long seg_weight(const long long *__restrict__ offsets, long long i,
                                                long long small_max) {
  const long long len = offsets[i + 1] - offsets[i];
  return len <= small_max ? len + kSegCost : 0;
}

// Both ends of workgroup g's range of G in the weight partition, in one pass
// (every chunk of segments holds at most BLOCK of them): range g starts at
// the first segment whose exclusive weight prefix reaches ceil(g T / G) (T
// the total weight) and ends where range g + 1 starts (the last one at
// nseg).  Chunk k holds segments [k*nseg/C, (k+1)*nseg/C) and chunks[k]
// their total weight.  The chunk weights are scanned once, the chunks that
// hold the two targets are found together, both chunks' segment weights are
// loaded at once, and two block scans give, in each chunk, the first
// segment whose prefix reaches its target (the chunk's end if none).  Each
// end is computed the same way by both workgroups it separates, so every
// segment belongs to exactly one range.  Returns T (0: no short segments,
// and g0, g1 unset).  Called by every thread.
template <int BLOCK>
__device__ __forceinline__ long long short_range_pair(const long long *__restrict__ offsets, long long nseg,
                                                      long long small_max, const long long *__restrict__ chunks,
                                                      int C, long long g, long long G, ShortShared<BLOCK> &S,
                                                      long long &g0, long long &g1) {
  const int tid = threadIdx.x;
  long long T = 0;
  const long long wk = tid < C ? chunks[tid] : 0;
  const long long inc = block_incl_scan<BLOCK>(wk, S.red, T);
  if (T == 0) return 0;
  S.lo[tid] = inc - wk;                               // weight before chunk tid
  if (tid < 2) S.kk[tid] = 0;
  __syncthreads();
  const bool has1 = g + 1 < G;
  const long long t0 = (g * T + G - 1) / G;
  const long long t1 = has1 ? ((g + 1) * T + G - 1) / G : T;
  // the last chunk whose prefix is at most each target (chunk 0's is 0)
  const unsigned long long m0 = __ballot(tid < C && S.lo[tid] <= t0);
  const unsigned long long m1 = __ballot(tid < C && S.lo[tid] <= t1);
  if ((tid & 63) == 0) {
    if (m0) atomicMax(&S.kk[0], tid + 63 - __clzll(m0));
    if (m1) atomicMax(&S.kk[1], tid + 63 - __clzll(m1));
  }
  __syncthreads();
  const long long k0 = __builtin_amdgcn_readfirstlane(S.kk[0]), k1 = __builtin_amdgcn_readfirstlane(S.kk[1]);
  const long long base0 = uniform_i64(S.lo[k0]), base1 = uniform_i64(S.lo[k1]);
  const long long a0 = k0 * nseg / C, b0 = (k0 + 1) * nseg / C;
  const long long a1 = k1 * nseg / C, b1 = (k1 + 1) * nseg / C;
  const long long i0 = a0 + tid, i1 = a1 + tid;
  const long long w0 = i0 < b0 ? seg_weight(offsets, i0, small_max) : 0;
  const long long w1 = (has1 && i1 < b1) ? seg_weight(offsets, i1, small_max) : 0;
  if (tid == 0) {
    S.f[0] = (unsigned long long)b0;
    S.f[1] = (unsigned long long)b1;
  }
  long long step = 0;
  const long long e0 = base0 + block_incl_scan<BLOCK>(w0, S.red, step) - w0;
  if (i0 < b0 && e0 >= t0) atomicMin(&S.f[0], (unsigned long long)i0);
  const long long e1 = base1 + block_incl_scan<BLOCK>(w1, S.red, step) - w1;
  if (has1 && i1 < b1 && e1 >= t1) atomicMin(&S.f[1], (unsigned long long)i1);
  __syncthreads();
  g0 = uniform_i64((long long)S.f[0]);
  g1 = has1 ? uniform_i64((long long)S.f[1]) : nseg;
  __syncthreads();
  return T;
}

// Short segments (at most small_max terms, empty ones included).  Workgroup
// g of G takes the segments [start(g), start(g+1)): with `plan`, the ranges
// split the total weight (length + kSegCost over short segments) evenly,
// found from the chunk weights the long-segment kernel wrote; otherwise they
// split the segment count.  Within its range a workgroup stages up to BLOCK
// segments at a time in LDS and its wavefronts take them one by one from an
// LDS counter, longest class first, each summing a whole segment into its
// own small accumulator and rounding it.  Handing segments out inside the
// workgroup keeps every wavefront busy whatever its issue priority.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void seg_short_kernel(const double *__restrict__ x,
                                                          const long long *__restrict__ offsets, long long nseg,
                                                          double *__restrict__ out, long long small_max,
                                                          const long long *__restrict__ chunks, int plan) {
  constexpr int NW = BLOCK / 64;
  __shared__ ShortShared<BLOCK> S;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // all lanes active here
  const long long G = gridDim.x, g = blockIdx.x;
  long long g0, g1;
  if (plan) {
    if (short_range_pair<BLOCK>(offsets, nseg, small_max, chunks, (int)G, g, G, S, g0, g1) == 0)
      return;                                           // no short segments
  } else {
    g0 = nseg * g / G;
    g1 = nseg * (g + 1) / G;
  }
  long long *acc = S.acc[wave];
  unsigned long long *spec = S.spec[wave];
  for (long long r0 = g0; r0 < g1; r0 += BLOCK) {
    const long long i = r0 + tid;
    long long s0 = 0, s1 = 0;
    int cls = 3;
    if (i < g1) {
      s0 = offsets[i];
      s1 = offsets[i + 1];
      const long long len = s1 - s0;
      if (len <= small_max) cls = len >= kClassA ? 0 : (len >= kClassB ? 1 : 2);
    } else if (i == g1) {
      s0 = offsets[i];
    }
    // segment r0 + j of the round is [lo[j], lo[j + 1])
    S.lo[tid] = s0;
    if (tid == BLOCK - 1) S.lo[BLOCK] = s1;
    const unsigned long long m0 = __ballot(cls == 0), m1 = __ballot(cls == 1), m2 = __ballot(cls == 2);
    if (lane == 0) {
      S.ccount[0][wave] = __popcll(m0);
      S.ccount[1][wave] = __popcll(m1);
      S.ccount[2][wave] = __popcll(m2);
    }
    if (tid == 0) S.cnt = 0;
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      int before = 0, all = 0;
      for (int w = 0; w < NW; w++) {
        const int n = S.ccount[c][w];
        if (w < wave) before += n;
        all += n;
      }
      if (cls == c) {
        const unsigned long long m = c == 0 ? m0 : (c == 1 ? m1 : m2);
        S.ord[total + before + __popcll(m & ((1ull << lane) - 1ull))] = tid;
      }
      total += all;
    }
    total = __builtin_amdgcn_readfirstlane(total);
    __syncthreads();
    // Every lane adds 1, so one claim advances the counter by 64 and the
    // first lane's old value (wave-uniform) names the claimed entry; no
    // value of one lane is broadcast, and every loop and branch stays scalar.
    const auto claim = [&](int &j, long long &a, long long &b) -> bool {
      const int k = __builtin_amdgcn_readfirstlane(atomicAdd(&S.cnt, 1)) >> 6;
      if (k >= total) return false;
      j = __builtin_amdgcn_readfirstlane(S.ord[k]);
      a = uniform_i64(S.lo[j]);
      b = uniform_i64(S.lo[j + 1]);
      return true;
    };
    // A segment's first loads are issued as soon as the previous segment's
    // last batch has been added, so they are in flight while that segment
    // is finished and rounded; the accumulator is cleared under them.
    const SrcF64 src{x};
    int j = 0;
    long long a = 0, b = 0;
    PairRange<SrcF64> R;
    bool have = claim(j, a, b);
    if (have && b > a) pair_range_begin(R, src, a, b, lane);
    small_wave_zero<kShortCopies>(acc, spec, lane);
    while (have) {
      SmallWin w;
      if (b > a) pair_range_add<kShortCopies>(acc, spec, src, R, lane, w);
      int j1 = 0;
      long long a1 = 0, b1 = 0;
      const bool next = claim(j1, a1, b1);
      if (next && b1 > a1) pair_range_begin(R, src, a1, b1, lane);
      int hb, W;
      const bool win = small_window<kShortCopies>(w, b - a, hb, W);
      if (win) small_wave_finish_window<kShortCopies>(acc, lane, b - a < 1024, hb, W);
      else small_wave_finish<kShortCopies>(acc, lane, b - a < 1024);
      wave_merge_and_round(acc, spec, nullptr, 1u, &out[r0 + j], lane);
      if (!next) break;
      if (win) small_window_clear(acc, lane, hb, W);
      else small_wave_zero<kShortCopies>(acc, spec, lane);
      j = j1;
      a = a1;
      b = b1;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One persistent launch for the whole batch.  Every workgroup first sums the
// long segments of its term range (long_phase, as above); then every wave,
// on its own, claims units of short segments until none are left.  A unit is
// (class c, group g): the segments [g*group, (g+1)*group) whose length falls
// in class c (at least 4096 terms, at least 512, the rest; at most
// small_max).  The groups are dealt to kCursors cursors, group g to cursor
// g mod kCursors, and each cursor hands out all its class-A units, then its
// class-B ones, then class C: the longest short segments start first and
// the last units handed out are the shortest, so no compute unit waits long
// for another at the end, and a workgroup whose term range held few
// long-segment terms goes on to short ones at once.  A wave claims from the
// cursor of its own XCD (workgroups are dealt to the eight XCDs in turn)
// and, once that is exhausted, from the others, so the claims spread over
// kCursors separate addresses.  Each claimed segment is summed whole by the
// wave with the small superaccumulator and rounded there (Performance
// evaluations: the small method for short sums, the large one for long
// sums).  A wave claims its next unit and issues that unit's offset loads
// before it sums the current one, so neither latency stands between units.
//
// The cursors and a count of finished waves live in the workspace, zeroed.
// A wave counts itself finished after the claims that found every cursor
// exhausted, so the last one to finish knows every claim has been made and
// resets them all: the next launch on the stream starts clean (and a
// captured graph can be replayed).  Claims are made by lane 0 and read back
// with readfirstlane, so every loop below is wave-uniform; nothing waits on
// another wave or workgroup.
// ---------------------------------------------------------------------------
constexpr int kCursors = 8;
// Length classes of the cursors' order: at least kClassA terms, at least
// kClassB, the rest (two classes, the shorter ones together, measured slower).
constexpr int kUnitClasses = 3;
struct SegCtl {
  unsigned int cursor[kCursors][32];    // one 128-byte line each
  unsigned int done;                    // waves that have made their last claim
};

template <int NW>
struct PersistShort {
  long long acc[NW][small_acc_words<kShortCopies>()];
  unsigned long long spec[NW][4];
};
template <int NW>
union PersistShared {
  SegShared L;                          // the long phase
  PersistShort<NW> S;                   // the short phase
};

// A claimed unit: its first segment and class (wave-uniform; cls < 0 means
// every cursor was exhausted), and this lane's segment (have: it exists).
struct SegUnit {
  long long g0;
  long long cls;
  long long s0, s1;
  bool have;
};

struct UnitClaimer {
  SegCtl *ctl;
  long long ngroups, group;
  int home;                             // this workgroup's XCD's cursor
  int t;                                // cursors home .. home+t-1 (mod kCursors) are exhausted
  // Claim a unit (blocking on the atomic); cls < 0 when none is left.
  __device__ void claim(SegUnit &u, int lane) {
    u.cls = -1;
    u.g0 = 0;
    while (t < kCursors) {
      const int k = (home + t) % kCursors;
      unsigned int v = 0;
      if (lane == 0) v = atomicAdd(&ctl->cursor[k][0], 1u);
      const long long vv = (long long)(unsigned int)__builtin_amdgcn_readfirstlane((int)v);
      // cursor k holds the groups k, k + kCursors, ... below ngroups
      const long long ngk = (ngroups - k + kCursors - 1) / kCursors;
      if (vv < kUnitClasses * ngk) {
        u.cls = vv / ngk;
        u.g0 = ((vv - u.cls * ngk) * kCursors + k) * group;
        return;
      }
      t++;
    }
  }
};

// Issue the unit's offset loads (lanes below `group`); their values are
// first used by unit_run.
__device__ __forceinline__ void unit_load(SegUnit &u, const long long *__restrict__ offsets, long long nseg,
                                          long long group, int lane) {
  const long long i = u.g0 + lane;
  u.have = u.cls >= 0 && lane < group && i < nseg;
  u.s0 = 0;
  u.s1 = 0;
  if (u.have) {
    u.s0 = offsets[i];
    u.s1 = offsets[i + 1];
  }
}

// Sum and round the unit's segments of its class, one after another;
// `before_last` runs once, just before the last of them (at once if there
// are none), so the next unit is claimed late enough that a wave never sits
// on a unit another wave could have taken, yet its latency still hides
// behind one segment.
template <class Hook>
__device__ __forceinline__ void unit_run(const SegUnit &u, const SrcF64 &src, double *__restrict__ out,
                                         long long small_max, long long *acc, unsigned long long *spec, int lane,
                                         const Hook &before_last) {
  const long long len = u.s1 - u.s0;
  const long long c = len >= kClassA ? 0 : (len >= kClassB ? 1 : 2);
  unsigned long long m = __ballot(u.have && len <= small_max && c == u.cls);
  if (m == 0ull) before_last();
  for (; m; m &= m - 1) {
    if ((m & (m - 1)) == 0ull) before_last();
    const int k = __ffsll((long long)m) - 1;
    const long long a = (long long)readlane_u64((unsigned long long)u.s0, k);
    const long long b = (long long)readlane_u64((unsigned long long)u.s1, k);
    small_wave_zero<kShortCopies>(acc, spec, lane);
    small_wave_accumulate<kShortCopies>(acc, spec, src, a, b, lane, true);
    wave_merge_and_round(acc, spec, nullptr, 1u, &out[u.g0 + k], lane);
  }
}

template <int BLOCK, int VEC, int DEPTH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK <= 256 ? 2 : 4)))
void seg_persistent_kernel(const double *__restrict__ x, const long long *__restrict__ offsets, long long nseg,
                           double *__restrict__ out, GlobalAcc *__restrict__ accs, long long small_max,
                           int precombine, SegCtl *__restrict__ ctl, int group) {
  constexpr int NW = BLOCK / 64;
  __shared__ PersistShared<NW> U;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // all lanes active here
  long_phase<BLOCK, VEC, DEPTH>(U.L, x, offsets, nseg, out, accs, small_max, precombine, false);
  __syncthreads();                                    // the long phase's LDS is reused below

  long long *acc = U.S.acc[wave];
  unsigned long long *spec = U.S.spec[wave];
  const SrcF64 src{x};
  // a wave starts at the cursor of its workgroup's XCD
  UnitClaimer cl{ctl, (nseg + group - 1) / group, group, (int)(blockIdx.x % kCursors), 0};
  SegUnit A, B;
  cl.claim(A, lane);
  unit_load(A, offsets, nseg, group, lane);
  auto next_b = [&]() {
    cl.claim(B, lane);
    unit_load(B, offsets, nseg, group, lane);
  };
  auto next_a = [&]() {
    cl.claim(A, lane);
    unit_load(A, offsets, nseg, group, lane);
  };
  while (A.cls >= 0) {
    unit_run(A, src, out, small_max, acc, spec, lane, next_b);
    if (B.cls < 0) break;
    unit_run(B, src, out, small_max, acc, spec, lane, next_a);
  }
  if (lane == 0) {
    const unsigned int total = gridDim.x * (unsigned int)NW;
    if (atomicAdd(&ctl->done, 1u) == total - 1u) {
      for (int k = 0; k < kCursors; k++) atomicExch(&ctl->cursor[k][0], 0u);
      atomicExch(&ctl->done, 0u);
    }
  }
}

}  // namespace

hipError_t launch_segmented(const double *x, const int64_t *offsets, int64_t nseg, double *out, GlobalAcc *accs,
                            long long *chunks, hipStream_t s, int grid, int short_grid, int64_t small_max,
                            int precombine) {
  if (grid < 1) grid = 1;
  if (short_grid < 1) short_grid = 1;
  if (short_grid > kShortBlock) short_grid = kShortBlock;
  // the weight partition needs at most BLOCK segments per chunk
  const int plan = nseg <= (int64_t)short_grid * kShortBlock ? 1 : 0;
  hipLaunchKernelGGL((seg_long_kernel<kLongBlock, 4, 2>), dim3(grid), dim3(kLongBlock), 0, s, x, (const long long *)offsets,
                     (long long)nseg, out, accs, (long long)small_max, precombine, plan ? chunks : nullptr,
                     short_grid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((seg_short_kernel<kShortBlock>), dim3(short_grid), dim3(kShortBlock), 0, s, x,
                     (const long long *)offsets, (long long)nseg, out, (long long)small_max,
                     (const long long *)chunks, plan);
  return hipGetLastError();
}

namespace {
// Offset validation (a debugging aid; the summing kernels trust the offsets).
__global__ __launch_bounds__(64) void check_init_kernel(unsigned long long *first_bad) {
  if (threadIdx.x == 0) first_bad[0] = ~0ull;
}
// Segment i is invalid when offsets[i] > offsets[i+1], when i = 0 and
// offsets[0] < 0, or when i = nseg-1 and offsets[nseg] > n (n >= 0).  The
// smallest such i is kept with an unsigned minimum, so "none" stays all ones
// (-1 as int64).
__global__ __launch_bounds__(256) void check_offsets_kernel(const long long *__restrict__ offsets, long long nseg,
                                                            long long n, unsigned long long *first_bad) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += stride) {
    const long long a = offsets[i], b = offsets[i + 1];
    bool bad = a > b;
    if (i == 0 && a < 0) bad = true;
    if (i == nseg - 1 && n >= 0 && b > n) bad = true;
    if (bad) atomicMin(first_bad, (unsigned long long)i);
  }
}
}  // namespace

hipError_t launch_check_offsets(const int64_t *offsets, int64_t nseg, int64_t n, int64_t *first_bad, hipStream_t s) {
  unsigned long long *fb = reinterpret_cast<unsigned long long *>(first_bad);
  hipLaunchKernelGGL(check_init_kernel, dim3(1), dim3(64), 0, s, fb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nseg == 0) return e;
  long long blocks = (nseg + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(check_offsets_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const long long *)offsets,
                     (long long)nseg, (long long)n, fb);
  return hipGetLastError();
}

hipError_t launch_segmented_persistent(const double *x, const int64_t *offsets, int64_t nseg, double *out,
                                       GlobalAcc *accs, void *ctl, hipStream_t s, int grid, int block,
                                       int64_t small_max, int precombine, int group) {
  if (grid < 1) grid = 1;
  if (group < 1) group = 1;
  if (group > 64) group = 64;
#define EXSUM_SEG_LAUNCH(B, V, D)                                                                              \
  if (block == B) {                                                                                            \
    hipLaunchKernelGGL((seg_persistent_kernel<B, V, D>), dim3(grid), dim3(B), 0, s, x, (const long long *)offsets, \
                       (long long)nseg, out, accs, (long long)small_max, precombine, static_cast<SegCtl *>(ctl),   \
                       group);                                                                                 \
    return hipGetLastError();                                                                                  \
  }
  EXSUM_SEG_LAUNCH(256, 4, 2)
  EXSUM_SEG_LAUNCH(512, 2, 2)
  EXSUM_SEG_LAUNCH(1024, 2, 2)
#undef EXSUM_SEG_LAUNCH
  return hipErrorInvalidValue;
}

size_t seg_ctl_bytes() { return (sizeof(SegCtl) + 255) / 256 * 256; }

int seg_short_block() { return kShortBlock; }

size_t global_acc_bytes() { return sizeof(GlobalAcc); }

}  // namespace exsum
