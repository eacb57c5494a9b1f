// exsum_blocks.h -- workgroup- and wave-level building blocks shared by the
// single-sum and segmented kernels (gfx950, wave64).
//
// Large-accumulator body (section "Faster exact summation of many terms with a
// large superaccumulator"), re-planned for a GPU workgroup:
//   * the workgroup owns one large superaccumulator in LDS: 4096 raw-pattern
//     chunks (32 KiB) and 4096 32-bit counts (16 KiB);
//   * terms arrive by coalesced 16-byte loads, the next tile's loads issued
//     before the current tile is added;
//   * a term is one 64-bit LDS add of its whole bit pattern to the chunk its
//     top 12 bits (sign and exponent) select, and one count add -- no mask,
//     no sign test, no mantissa split;
//   * lanes of a wavefront that share a chunk are summed across the wave
//     first, so one lane updates a hot chunk once instead of 64 times;
//   * the paper's per-add count check becomes a threshold: the add that lifts
//     a count to THR = 4096 - (terms per tile) marks the chunk, and marked
//     chunks are transferred to the small superaccumulator at the next tile
//     barrier.  Between barriers a chunk gains at most one tile of adds, so no
//     chunk ever holds more than 4095 adds and its mantissa sum stays exact;
//   * at the end every used chunk is transferred, grouped by the top six
//     exponent bits so one wavefront reduction serves 64 chunks.
#pragma once

#include "exsum_device.h"

namespace exsum {

__device__ __forceinline__ unsigned long long as_bits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

// ---------------------------------------------------------------------------
// LDS state of the large-accumulator body
// ---------------------------------------------------------------------------
struct LargeShared {
  unsigned long long chunk[kLChunks];   // raw-pattern sums
  unsigned int cnt[kLChunks];           // adds since the last transfer
  long long small[68];                  // the workgroup's small accumulator
  unsigned int flushbits[kLChunks / 32];
  unsigned long long spec[3];           // +Inf seen, -Inf seen, max NaN bits
  unsigned int flag[4];                 // "some chunk marked", by tile mod 3
  unsigned int ticket;
  unsigned int bcast[4];                // broadcast slots
  unsigned int D[70];                   // rounding scratch
};

__device__ __forceinline__ void large_init(LargeShared &S, int tid, int block) {
  uint4 *p = reinterpret_cast<uint4 *>(&S.chunk[0]);
  const int nz = (int)((sizeof(S.chunk) + sizeof(S.cnt)) / 16);
  for (int i = tid; i < nz; i += block) p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (tid < 68) S.small[tid] = 0;
  if (tid < kLChunks / 32) S.flushbits[tid] = 0u;
  if (tid < 3) S.spec[tid] = 0ull;
  if (tid < 4) S.flag[tid] = 0u;
}

__device__ __forceinline__ void mark_chunk(LargeShared &S, unsigned int ix, unsigned int tile) {
  atomicOr(&S.flushbits[ix >> 5], 1u << (ix & 31));
  S.flag[tile % 3] = 1u;
}

// Transfer chunk ix into the small accumulator and reset it.
__device__ __forceinline__ void flush_chunk(LargeShared &S, unsigned int ix) {
  const unsigned long long C = S.chunk[ix];
  const unsigned int k = S.cnt[ix];
  long long p0, p1, p2;
  int h;
  chunk_pieces(ix, C, k, p0, p1, p2, h);
  atomicAdd((unsigned long long *)&S.small[h], (unsigned long long)p0);
  atomicAdd((unsigned long long *)&S.small[h + 1], (unsigned long long)p1);
  atomicAdd((unsigned long long *)&S.small[h + 2], (unsigned long long)p2);
  S.chunk[ix] = 0ull;
  S.cnt[ix] = 0u;
}

// Add the NT terms a lane holds for this tile.  Every lane of the wave calls
// this together; valid[j] masks lanes without a term j.  The LDS updates of
// all NT terms are issued before any count is examined, so one wait covers
// the tile; crossings of the threshold are rare and handled after a ballot.
template <int NT>
__device__ __forceinline__ void add_terms(LargeShared &S, const unsigned long long (&b)[NT], const bool (&valid)[NT],
                                          int precombine, unsigned int tile, int lane, unsigned int thr) {
  constexpr unsigned int kNone = 0xFFFFFFFFu;
  unsigned int key[NT];
  bool any_special = false;
#pragma unroll
  for (int j = 0; j < NT; j++) {
    const bool sp = is_special(b[j]);
    any_special |= valid[j] && sp;
    key[j] = (valid[j] && !sp) ? (unsigned int)(b[j] >> 52) : kNone;
  }
  if (__builtin_expect(__ballot(any_special) != 0ull, 0)) {
#pragma unroll
    for (int j = 0; j < NT; j++)
      if (valid[j] && is_special(b[j])) note_special(b[j], &S.spec[0], &S.spec[1], &S.spec[2]);
  }
  if (precombine > 0) {
#pragma unroll
    for (int j = 0; j < NT; j++) {
      const unsigned int leader = __builtin_amdgcn_readfirstlane(key[j]);
      const unsigned long long m = __ballot(key[j] == leader);
      const int k = __popcll(m);
      if (leader != kNone && k >= precombine) {
        const unsigned long long s = wave_sum_u64(key[j] == leader ? b[j] : 0ull);
        if (lane == __ffsll((long long)m) - 1) {
          atomicAdd(&S.chunk[leader], s);
          const unsigned int old = atomicAdd(&S.cnt[leader], (unsigned int)k);
          if (old < thr && old + (unsigned int)k >= thr) mark_chunk(S, leader, tile);
        }
        if (key[j] == leader) key[j] = kNone;
      }
    }
  }
  unsigned int old[NT];
#pragma unroll
  for (int j = 0; j < NT; j++) {
    old[j] = 0u;
    if (key[j] != kNone) {
      atomicAdd(&S.chunk[key[j]], b[j]);
      old[j] = atomicAdd(&S.cnt[key[j]], 1u);
    }
  }
  bool cross = false;
#pragma unroll
  for (int j = 0; j < NT; j++) cross |= (key[j] != kNone) && (old[j] == thr - 1u);
  if (__builtin_expect(__ballot(cross) != 0ull, 0)) {
#pragma unroll
    for (int j = 0; j < NT; j++)
      if (key[j] != kNone && old[j] == thr - 1u) mark_chunk(S, key[j], tile);
  }
}

// End of a tile: barrier, then transfer the chunks marked during the tile.
// The "marked" flag is kept per tile mod 3 so one barrier per tile suffices:
// flag[t%3] is set during tile t, read after tile t's barrier, and cleared
// during tile t+2.
__device__ __forceinline__ void tile_end(LargeShared &S, unsigned int tile, int tid) {
  lds_barrier();
  const unsigned int f = S.flag[tile % 3];
  if (tid == 0) S.flag[(tile + 2) % 3] = 0u;
  if (f) {
    if (tid < kLChunks / 32) {
      unsigned int bits = S.flushbits[tid];
      if (bits) {
        S.flushbits[tid] = 0u;
        while (bits) {
          const int bp = __ffs(bits) - 1;
          bits &= bits - 1u;
          flush_chunk(S, (unsigned int)(tid * 32 + bp));
        }
      }
    }
    lds_barrier();
  }
}

// Add x[r0 .. r1) into the workgroup's large accumulator.  A misaligned first
// term and an odd last term are added as scalars; the rest by 16-byte loads,
// BLOCK*VEC per tile, with the next two tiles' loads in flight.
template <int BLOCK, int VEC>
__device__ __forceinline__ void accumulate_range(LargeShared &S, const double *__restrict__ x, long long r0,
                                                 long long r1, int precombine, unsigned int &tile) {
  constexpr int TILE_V = BLOCK * VEC;
  constexpr unsigned int THR = kCap - 2 * TILE_V;
  static_assert(2 * TILE_V < kCap, "tile too large for the count bound");
  const int tid = threadIdx.x, lane = tid & 63;
  if (r1 <= r0) return;
  const long long head = (reinterpret_cast<uintptr_t>(x + r0) & 15) ? 1 : 0;
  const long long a = r0 + head;
  const long long nv = (r1 - a) >> 1;
  const bool has_tail = ((r1 - a) & 1) != 0;
  if (head || has_tail) {
    unsigned long long b[1] = {0ull};
    bool valid[1] = {false};
    if (tid == 0 && head) { b[0] = as_bits(x[r0]); valid[0] = true; }
    if (tid == 1 && has_tail) { b[0] = as_bits(x[r1 - 1]); valid[0] = true; }
    add_terms<1>(S, b, valid, precombine, tile, lane, THR);
    tile_end(S, tile++, tid);
  }
  const ulonglong2 *__restrict__ xv = reinterpret_cast<const ulonglong2 *>(x + a);
  const long long ntiles = nv / TILE_V;
  // Two tiles in flight: buffer A holds even tiles, B odd ones.  Loads are
  // unconditional (an index past the last tile re-reads the last tile) so the
  // compiler's wait counts stay exact and a prefetch is never waited early.
  ulonglong2 bufA[VEC], bufB[VEC];
  auto load = [&](ulonglong2(&buf)[VEC], long long t) {
    const long long tb = (t < ntiles ? t : ntiles - 1) * TILE_V + tid;
#pragma unroll
    for (int j = 0; j < VEC; j++) buf[j] = xv[tb + j * BLOCK];
    // keep the scheduler from hoisting work on the other buffer above these
    // loads (which would force an early wait on them)
    __builtin_amdgcn_sched_barrier(0);
  };
  auto process = [&](const ulonglong2(&buf)[VEC]) {
    unsigned long long b[2 * VEC];
    bool valid[2 * VEC];
#pragma unroll
    for (int j = 0; j < VEC; j++) {
      b[2 * j] = buf[j].x;
      b[2 * j + 1] = buf[j].y;
      valid[2 * j] = valid[2 * j + 1] = true;
    }
    add_terms<2 * VEC>(S, b, valid, precombine, tile, lane, THR);
    tile_end(S, tile++, tid);
  };
  if (ntiles > 0) {
    load(bufA, 0);
    load(bufB, 1);
    for (long long t = 0; t < ntiles; t += 2) {
      process(bufA);
      load(bufA, t + 2);
      if (t + 1 < ntiles) process(bufB);
      load(bufB, t + 3);
    }
  }
  const long long base = ntiles * TILE_V;
  if (base < nv) {
    unsigned long long b[2 * VEC];
    bool valid[2 * VEC];
#pragma unroll
    for (int j = 0; j < VEC; j++) {
      const long long idx = base + j * BLOCK + tid;
      const bool ok = idx < nv;
      ulonglong2 v = make_ulonglong2(0ull, 0ull);
      if (ok) v = xv[idx];
      b[2 * j] = v.x;
      b[2 * j + 1] = v.y;
      valid[2 * j] = valid[2 * j + 1] = ok;
    }
    add_terms<2 * VEC>(S, b, valid, precombine, tile, lane, THR);
    tile_end(S, tile++, tid);
  }
}

// Transfer every used chunk into S.small.  Group gi holds the 64 chunks whose
// exponent field has top six bits gi (both signs, 32 low-exponent values);
// all of them land on small chunks gi .. gi+2, so three wavefront sums and
// three LDS adds serve the group.  With `clean`, the chunks and counts read
// are reset to zero (so the next unit of work needs no initialisation).
template <int BLOCK, bool clean>
__device__ __forceinline__ void final_flush(LargeShared &S) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __syncthreads();
  for (int gi = wave; gi < 64; gi += NW) {
    const unsigned int ix = ((unsigned int)(lane >> 5) << 11) | (unsigned int)(gi * 32 + (lane & 31));
    const unsigned int k = S.cnt[ix];
    if (__ballot(k != 0u) == 0ull) continue;
    long long p0 = 0, p1 = 0, p2 = 0;
    int h = gi;
    if (k) {
      chunk_pieces(ix, S.chunk[ix], k, p0, p1, p2, h);
      if (clean) { S.chunk[ix] = 0ull; S.cnt[ix] = 0u; }
    }
    p0 = wave_sum_i64(p0);
    p1 = wave_sum_i64(p1);
    p2 = wave_sum_i64(p2);
    if (lane == 0) {
      atomicAdd((unsigned long long *)&S.small[gi], (unsigned long long)p0);
      atomicAdd((unsigned long long *)&S.small[gi + 1], (unsigned long long)p1);
      atomicAdd((unsigned long long *)&S.small[gi + 2], (unsigned long long)p2);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Merge (Discussion: add the parts' small superaccumulators, round once).
// A workgroup adds its 67 chunks into `g` with 64-bit integer atomics (exact
// and order independent), takes a ticket, and the one that completes the
// expected count reads and clears `g`, rounds, and writes *out.  Called by
// every thread; returns true in the workgroup that wrote the result.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool merge_and_round(long long *s_small, unsigned long long *spec,
                                                unsigned int *s_ticket, unsigned int *s_D,
                                                GlobalAcc *__restrict__ g, unsigned int expected,
                                                double *__restrict__ out) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (expected <= 1) {
    if (tid == 0) out[0] = __longlong_as_double((long long)round_chunks(s_small, spec[0], spec[1], spec[2], s_D));
    __syncthreads();
    return true;
  }
  if (tid < kSChunks) {
    const long long v = s_small[tid];
    if (v) atomicAdd(&g->chunk[tid], (unsigned long long)v);
  }
  if (tid == 0) {
    if (spec[0]) atomicOr(&g->pos_inf, 1ull);
    if (spec[1]) atomicOr(&g->neg_inf, 1ull);
    if (spec[2]) atomicMax(&g->nan_bits, spec[2]);
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) *s_ticket = atomicAdd(&g->ticket, 1u);
  __syncthreads();
  const bool last = (*s_ticket == expected - 1);
  __syncthreads();
  if (!last) return false;
  __threadfence();
  if (tid < kSChunks) s_small[tid] = (long long)atomicExch(&g->chunk[tid], 0ull);
  if (tid == 96) spec[0] = atomicExch(&g->pos_inf, 0ull);
  if (tid == 97) spec[1] = atomicExch(&g->neg_inf, 0ull);
  if (tid == 98) spec[2] = atomicExch(&g->nan_bits, 0ull);
  if (tid == 99) atomicExch(&g->ticket, 0u);
  __syncthreads();
  if (tid == 0) out[0] = __longlong_as_double((long long)round_chunks(s_small, spec[0], spec[1], spec[2], s_D));
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// Small-only wave body (section "Exact summation using a small
// superaccumulator"): the wave adds its terms into one 67-chunk accumulator
// in LDS, two 64-bit LDS adds per term (a 32-bit low piece to chunk
// e_eff>>5, the rest to the next).  The sign is applied without a branch
// (Discussion).  A chunk receives at most 64 pieces below 2^52 per wave step,
// so a parallel carry step every 31 steps keeps every chunk below 2^63.
// ---------------------------------------------------------------------------

// One parallel carry step over 67 chunks: c_i <- low32(c_i) + (c_{i-1} >> 32)
// (chunk 66 keeps its high part).  Leaves |c_i| < 2^33, value unchanged.
__device__ __forceinline__ void carry_step(long long *c, int lane) {
  const long long a0 = c[lane];
  const long long b0 = lane > 0 ? c[lane - 1] : 0;
  long long a1 = 0, b1 = 0;
  if (lane < 3) { a1 = c[64 + lane]; b1 = c[63 + lane]; }
  const long long n0 = (lane == 0) ? (a0 & 0xFFFFFFFFll) : ((a0 & 0xFFFFFFFFll) + (b0 >> 32));
  long long n1 = 0;
  if (lane < 2) n1 = (a1 & 0xFFFFFFFFll) + (b1 >> 32);
  else if (lane == 2) n1 = a1 + (b1 >> 32);
  __builtin_amdgcn_wave_barrier();
  c[lane] = n0;
  if (lane < 3) c[64 + lane] = n1;
  __builtin_amdgcn_wave_barrier();
}

// Wave adds x[lo .. hi) into acc (68 chunks, zeroed by the caller); specials
// into spec[3].  Ends with a carry step, so |acc[i]| < 2^33 on return.
__device__ __forceinline__ void small_wave_accumulate(long long *acc, unsigned long long *spec,
                                                      const double *__restrict__ x, long long lo, long long hi,
                                                      int lane) {
  int steps = 0;
  for (long long base = lo; base < hi; base += 64) {
    const long long i = base + lane;
    if (i < hi) {
      const unsigned long long b = as_bits(x[i]);
      if (is_special(b)) {
        note_special(b, &spec[0], &spec[1], &spec[2]);
      } else {
        int h;
        long long plo, phi;
        term_pieces(b, h, plo, phi);
        atomicAdd((unsigned long long *)&acc[h], (unsigned long long)plo);
        atomicAdd((unsigned long long *)&acc[h + 1], (unsigned long long)phi);
      }
    }
    if (++steps == 31) {
      steps = 0;
      carry_step(acc, lane);
    }
  }
  carry_step(acc, lane);
}

}  // namespace exsum
