// kernels_seg.hip -- many exact sums of uneven length in one persistent
// launch (plus a small planning launch), gfx950.
//
// Planning (one thread per segment, no host round trip): a segment of length
// L <= small_max goes on the short list; a longer one becomes a long entry
// with ceil(L / tile) tiles.  The small/large choice follows the Performance
// evaluations section (the small superaccumulator alone is faster for short
// sums, the large one for long sums); the threshold is a tuning knob.
//
// Persistent kernel, two phases per workgroup:
//   A. long tiles: thread 0 takes (entry, tile) from a two-level cursor; the
//      whole workgroup adds the tile into its large accumulator in LDS,
//      transfers it into the small accumulator (cleaning the LDS for the next
//      tile), and merges into the segment's global accumulator; the tile that
//      completes the segment rounds it.  A one-tile segment is rounded in
//      place.
//   B. short segments: each wavefront takes a batch of short segments and
//      sums each with the small-only wave body, rounding in the wavefront.
// The last workgroup to finish resets the cursors, so the workspace is clean
// for the next call.
#include "exsum_blocks.h"
#include "exsum_internal.h"

namespace exsum {
namespace {

struct SegHeader {
  unsigned int nlong;       // long entries planned
  unsigned int nshort;      // short segments planned
  unsigned int long_cur;    // entry currently handed out
  unsigned int short_cur;   // next short slot
  unsigned int done;        // workgroups finished
  unsigned int pad[59];
};
static_assert(sizeof(SegHeader) == 256, "SegHeader layout");

struct LongEntry {
  int seg;
  unsigned int ntiles;
  unsigned int next_tile;
  unsigned int pad;
};

struct SegLayout {
  SegHeader *hdr;
  LongEntry *entries;
  int *short_ids;
  GlobalAcc *accs;
};

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

__host__ __device__ inline SegLayout seg_layout(void *ws, long long nseg) {
  SegLayout L;
  char *p = static_cast<char *>(ws);
  size_t off = 0;
  L.hdr = reinterpret_cast<SegHeader *>(p + off);
  off += sizeof(SegHeader);
  L.entries = reinterpret_cast<LongEntry *>(p + off);
  off = align_up(off + sizeof(LongEntry) * (size_t)nseg, 256);
  L.short_ids = reinterpret_cast<int *>(p + off);
  off = align_up(off + sizeof(int) * (size_t)nseg, 256);
  L.accs = reinterpret_cast<GlobalAcc *>(p + off);
  return L;
}

constexpr int kShortBatch = 8;

__global__ __launch_bounds__(256) void seg_plan_kernel(const long long *__restrict__ offsets, long long nseg,
                                                       void *ws, long long cap, long long small_max,
                                                       long long tile) {
  SegLayout Lw = seg_layout(ws, cap);
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  long long L = 0;
  if (i < nseg) L = offsets[i + 1] - offsets[i];
  const bool is_short = (i < nseg) && (L <= small_max);
  const bool is_long = (i < nseg) && (L > small_max);
  // wave-aggregated slot allocation: one atomic per wave per list
  const unsigned long long ms = __ballot(is_short);
  const unsigned long long ml = __ballot(is_long);
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned int bs = 0, bl = 0;
  if (lane == 0) {
    if (ms) bs = atomicAdd(&Lw.hdr->nshort, (unsigned int)__popcll(ms));
    if (ml) bl = atomicAdd(&Lw.hdr->nlong, (unsigned int)__popcll(ml));
  }
  bs = __shfl(bs, 0, 64);
  bl = __shfl(bl, 0, 64);
  if (is_short) Lw.short_ids[bs + __popcll(ms & below)] = (int)i;
  if (is_long) {
    LongEntry e;
    e.seg = (int)i;
    e.ntiles = (unsigned int)((L + tile - 1) / tile);
    e.next_tile = 0u;
    e.pad = 0u;
    Lw.entries[bl + __popcll(ml & below)] = e;
  }
}

template <int BLOCK, int VEC>
__global__ __launch_bounds__(BLOCK) void seg_kernel(const double *__restrict__ x,
                                                    const long long *__restrict__ offsets, long long nseg,
                                                    double *__restrict__ out, void *ws, long long cap,
                                                    long long tile_terms, int precombine) {
  __shared__ LargeShared S;
  SegLayout Lw = seg_layout(ws, cap);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  large_init(S, tid, BLOCK);
  __syncthreads();
  const unsigned int nlong = Lw.hdr->nlong;
  const unsigned int nshort = Lw.hdr->nshort;
  unsigned int tile = 0;

  // phase A: tiles of long segments
  while (nlong) {
    if (tid == 0) {
      unsigned int eidx = 0xFFFFFFFFu, t = 0;
      while (true) {
        const unsigned int cur = __hip_atomic_load(&Lw.hdr->long_cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur >= nlong) break;
        t = atomicAdd(&Lw.entries[cur].next_tile, 1u);
        if (t < Lw.entries[cur].ntiles) { eidx = cur; break; }
        atomicCAS(&Lw.hdr->long_cur, cur, cur + 1u);
      }
      S.bcast[0] = eidx;
      S.bcast[1] = t;
    }
    __syncthreads();
    const unsigned int eidx = S.bcast[0], t = S.bcast[1];
    __syncthreads();
    if (eidx == 0xFFFFFFFFu) break;
    const LongEntry e = Lw.entries[eidx];
    const long long start = offsets[e.seg], end = offsets[e.seg + 1];
    const long long r0 = start + (long long)t * tile_terms;
    const long long r1 = (r0 + tile_terms < end) ? r0 + tile_terms : end;
    accumulate_range<BLOCK, VEC, 2, kCountMode>(S, x, r0, r1, precombine, tile);
    final_flush<BLOCK, true, kCountMode>(S);
    merge_and_round(S.small, S.spec, &S.ticket, S.D, &Lw.accs[eidx], e.ntiles, &out[e.seg]);
    if (tid < 68) S.small[tid] = 0;
    if (tid < 3) S.spec[tid] = 0ull;
    __syncthreads();
  }

  // phase B: short segments, one wavefront per segment, in batches
  {
    char *base = reinterpret_cast<char *>(&S.chunk[0]) + wave * 1024;
    long long *acc = reinterpret_cast<long long *>(base);
    unsigned long long *spec = reinterpret_cast<unsigned long long *>(base + 576);
    unsigned int *D = reinterpret_cast<unsigned int *>(base + 640);
    while (true) {
      unsigned int j0 = 0;
      if (lane == 0) j0 = atomicAdd(&Lw.hdr->short_cur, (unsigned int)kShortBatch);
      j0 = __shfl(j0, 0, 64);
      if (j0 >= nshort) break;
      const unsigned int j1 = (j0 + kShortBatch < nshort) ? j0 + kShortBatch : nshort;
      for (unsigned int j = j0; j < j1; j++) {
        const int seg = Lw.short_ids[j];
        acc[lane] = 0;
        if (lane < 4) acc[64 + lane] = 0;
        if (lane < 3) spec[lane] = 0ull;
        __builtin_amdgcn_wave_barrier();
        small_wave_accumulate(acc, spec, x, offsets[seg], offsets[seg + 1], lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane == 0) out[seg] = __longlong_as_double((long long)round_chunks(acc, spec[0], spec[1], spec[2], D));
        __builtin_amdgcn_wave_barrier();
      }
    }
  }

  // completion: the last workgroup resets the cursors for the next call
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const unsigned int d = atomicAdd(&Lw.hdr->done, 1u);
    if (d == gridDim.x - 1) {
      atomicExch(&Lw.hdr->nlong, 0u);
      atomicExch(&Lw.hdr->nshort, 0u);
      atomicExch(&Lw.hdr->long_cur, 0u);
      atomicExch(&Lw.hdr->short_cur, 0u);
      atomicExch(&Lw.hdr->done, 0u);
    }
  }
}

}  // namespace

// The layout depends only on the capacity (segments the workspace was sized
// for), never on a call's nseg, so regions that must stay zero between calls
// (the per-segment accumulators) never move.
size_t seg_workspace_bytes(int64_t nseg) {
  size_t off = sizeof(SegHeader);
  off = align_up(off + sizeof(LongEntry) * (size_t)nseg, 256);
  off = align_up(off + sizeof(int) * (size_t)nseg, 256);
  off += sizeof(GlobalAcc) * (size_t)nseg;
  return off;
}

hipError_t launch_segmented(const double *x, const int64_t *offsets, int64_t nseg, double *out, void *ws,
                            int64_t cap, hipStream_t s, int grid, int64_t small_max, int64_t tile,
                            int precombine) {
  const int plan_blocks = (int)((nseg + 255) / 256);
  hipLaunchKernelGGL(seg_plan_kernel, dim3(plan_blocks), dim3(256), 0, s, (const long long *)offsets,
                     (long long)nseg, ws, (long long)cap, (long long)small_max, (long long)tile);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((seg_kernel<256, 4>), dim3(grid), dim3(256), 0, s, x, (const long long *)offsets,
                     (long long)nseg, out, ws, (long long)cap, (long long)tile, precombine);
  return hipGetLastError();
}

}  // namespace exsum
