// exsum_blocks.h -- workgroup- and wave-level building blocks shared by the
// single-sum and segmented kernels (gfx950, wave64).
//
// Large-accumulator body (section "Faster exact summation of many terms with a
// large superaccumulator"), re-planned for a GPU workgroup:
//   * the workgroup owns one large superaccumulator in LDS: 4096 chunks, one
//     per (sign, exponent) combination, indexed by the top 12 bits of a term;
//   * terms arrive by coalesced 16-byte loads with the next DEPTH tiles in
//     flight; a term costs one 64-bit LDS add to the chunk it selects;
//   * lanes of a wavefront whose whole tile lands in one chunk are summed
//     across the wave first, so a hot chunk takes one update per tile;
//   * chunks reach the workgroup's small superaccumulator (67 chunks, LDS)
//     before a 64-bit chunk could lose information, and at the end every used
//     chunk is transferred, grouped by the top six exponent bits so one
//     wavefront reduction serves 64 chunks.
//
// Two ways of deciding when a chunk must be transferred (template MODE):
//   kCountMode -- the paper's: a chunk holds the plain sum of raw bit
//     patterns and a count of its adds; after k <= 4096 adds the mantissa sum
//     is chunk - k*(index<<52).  On the GPU the per-add count check becomes a
//     threshold: the add that lifts a count to THR = 4096 - (terms per tile)
//     marks the chunk, and marked chunks are transferred at the next tile
//     barrier.  Between barriers a chunk gains at most one tile of adds, so no
//     chunk ever holds more than 4095 adds.
//   kCarryMode -- GPU-native: a chunk holds the sum of the 53-bit mantissas
//     (implicit bit included, so no correction is ever needed) modulo 2^64.
//     The LDS add returns the chunk's previous value, so the lane whose add
//     wraps past 2^64 sees it and adds the lost 2^64 units directly to the
//     small superaccumulator (+-2^(e_eff&31) at small chunk (e_eff>>5)+2).
//     No counts, no thresholds and no tile barriers: waves run independently
//     and a tile may hold any number of terms.
#pragma once

#include "exsum_device.h"

namespace exsum {

constexpr int kCountMode = 0;
constexpr int kCarryMode = 1;

__device__ __forceinline__ unsigned long long as_bits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

// 53-bit mantissa of a finite term with its implicit bit (none for e == 0).
__device__ __forceinline__ unsigned long long mantissa53(unsigned long long b) {
  const unsigned int e = (unsigned int)(b >> 52) & 2047u;
  return (b & ((1ull << 52) - 1)) | ((unsigned long long)(e != 0u) << 52);
}

// ---------------------------------------------------------------------------
// LDS state of the large-accumulator body
// ---------------------------------------------------------------------------
struct LargeShared {
  unsigned long long chunk[kLChunks];   // raw-pattern sums (count mode) or mantissa sums (carry mode)
  unsigned int cnt[kLChunks];           // adds since the last transfer (count mode)
  long long small[68];                  // the workgroup's small accumulator
  unsigned int flushbits[kLChunks / 32];
  unsigned long long spec[3];           // +Inf seen, -Inf seen, max NaN bits
  unsigned int flag[4];                 // "some chunk marked", by tile mod 3
  unsigned int ticket;
  unsigned int bcast[4];                // broadcast slots
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

// Count mode: transfer chunk ix into the small accumulator and reset it.
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

// Carry mode: one wrap of chunk ix past 2^64 = 2^64 * 2^(e_eff-1075), which is
// 2^(e_eff & 31) units of small chunk (e_eff >> 5) + 2, signed by the index.
__device__ __forceinline__ void carry_out(LargeShared &S, unsigned int ix) {
  const unsigned int e = ix & 2047u;
  const unsigned int e_eff = e ? e : 1u;
  const long long v = (long long)(1ull << (e_eff & 31u));
  atomicAdd((unsigned long long *)&S.small[(e_eff >> 5) + 2], (unsigned long long)((ix >> 11) ? -v : v));
}

// Add `val` (k terms' worth) to chunk ix, with the mode's overflow rule.
template <int MODE>
__device__ __forceinline__ void chunk_add(LargeShared &S, unsigned int ix, unsigned long long val, unsigned int k,
                                          unsigned int tile, unsigned int thr) {
  if (MODE == kCountMode) {
    atomicAdd(&S.chunk[ix], val);
    const unsigned int old = atomicAdd(&S.cnt[ix], k);
    if (old < thr && old + k >= thr) mark_chunk(S, ix, tile);
  } else {
    const unsigned long long old = atomicAdd(&S.chunk[ix], val);
    if (old + val < old) carry_out(S, ix);
  }
}

// The value a term contributes to its chunk in each mode.
template <int MODE>
__device__ __forceinline__ unsigned long long chunk_value(unsigned long long b) {
  return MODE == kCountMode ? b : mantissa53(b);
}

// Add one term per lane (the general, rarely used path).  Every lane of the
// wave calls this together; `valid` masks lanes without a term.  Handles
// infinities and NaNs (side words), the cross-wave pre-combine of a widely
// shared chunk, and the mode's overflow rule.
template <int MODE>
__device__ __forceinline__ void add_slot(LargeShared &S, unsigned long long b, bool valid, int precombine,
                                         unsigned int tile, int lane, unsigned int thr) {
  constexpr unsigned int kNone = 0xFFFFFFFFu;
  const bool sp = valid && is_special(b);
  if (sp) note_special(b, &S.spec[0], &S.spec[1], &S.spec[2]);
  unsigned int key = (valid && !sp) ? (unsigned int)(b >> 52) : kNone;
  const unsigned long long val = chunk_value<MODE>(b);
  if (precombine > 0) {
    const unsigned int ld = __builtin_amdgcn_readfirstlane(key);
    const unsigned long long m = __ballot(key == ld);
    const int k = __popcll(m);
    if (ld != kNone && k >= precombine) {
      // count mode: k raw patterns sum exactly mod 2^64 (the count corrects);
      // carry mode: k < 2^11 mantissas below 2^53 sum below 2^64
      const unsigned long long s = wave_sum_u64(key == ld ? val : 0ull);
      if (lane == __ffsll((long long)m) - 1) chunk_add<MODE>(S, ld, s, (unsigned int)k, tile, thr);
      if (key == ld) key = kNone;
    }
  }
  if (key != kNone) chunk_add<MODE>(S, key, val, 1u, tile, thr);
}

// Slow tile: re-read this lane's vector positions (tb + j*stride for
// j < nslots <= kMaxSlots, present below `limit`, counted from the aligned
// term a) and add their terms one slot at a time.  All loads are issued
// before the first add, so a tile costs one memory latency.  Kept out of line
// so the hot loop stays small.
constexpr int kMaxSlots = 9;
template <int MODE, class Src>
__device__ __noinline__ void slow_tile(LargeShared *S, Src src, long long a, long long tb, long long limit,
                                       int stride, int nslots, int precombine, unsigned int tile, unsigned int thr) {
  constexpr int T = Src::kTPV;
  const int lane = threadIdx.x & 63;
  const typename Src::Ptr base = src.at(a, 0);
  typename Src::Vec v[kMaxSlots];
#pragma unroll
  for (int j = 0; j < kMaxSlots; j++) {
    const long long idx = tb + (long long)j * stride;
    v[j] = Src::zero();
    if (j < nslots && idx < limit) v[j] = Src::load_plain(base, idx);
  }
#pragma unroll
  for (int j = 0; j < kMaxSlots; j++) {
    if (j < nslots) {
      const bool ok = tb + (long long)j * stride < limit;
      unsigned long long t[T];
      src.terms(v[j], t);
#pragma unroll
      for (int k = 0; k < T; k++) add_slot<MODE>(*S, t[k], ok, precombine, tile, lane, thr);
    }
  }
}

// Fast tile: the NT terms every lane holds are all present.  Returns false,
// having changed nothing, when the tile needs the slow path (an infinity or
// NaN somewhere).
//   * whole wave, whole tile in one chunk: each lane sums its NT values, the
//     wave sums those, one lane adds the total (64*NT terms) to the chunk
//     (64 same-address adds per instruction would bind the LDS);
//   * otherwise one 64-bit LDS add per term (plus a count add in count
//     mode), all issued before any returned value is examined; the rare
//     threshold crossings or carries are found with one ballot per term.
//     Lanes that share a chunk partly serialise their adds, which costs far
//     less than taking the tile through the slow path.
template <int NT, int MODE>
__device__ __forceinline__ bool fast_tile(LargeShared &S, const unsigned long long (&b)[NT], int precombine,
                                          unsigned int tile, int lane, unsigned int thr) {
  static_assert(MODE == kCountMode || 64 * NT < 2048, "carry mode: a wave's tile sum must stay below 2^64");
  unsigned long long odd = 0;
  unsigned int key[NT];
#pragma unroll
  for (int j = 0; j < NT; j++) {
    odd |= __ballot(!__builtin_isfinite(__longlong_as_double((long long)b[j])));
    key[j] = (unsigned int)(b[j] >> 52);
  }
  if (odd) return false;
  if (precombine > 0) {
    const unsigned int leader = __builtin_amdgcn_readfirstlane(key[0]);
    unsigned long long all = ~0ull;
#pragma unroll
    for (int j = 0; j < NT; j++) all &= __ballot(key[j] == leader);
    if (all == ~0ull) {
      unsigned long long s = 0;
#pragma unroll
      for (int j = 0; j < NT; j++) s += chunk_value<MODE>(b[j]);
      s = wave_sum_u64(s);
      if (lane == 0) chunk_add<MODE>(S, leader, s, 64u * NT, tile, thr);
      return true;
    }
  }
  if (MODE == kCountMode) {
    unsigned int old[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) {
      atomicAdd(&S.chunk[key[j]], b[j]);
      old[j] = atomicAdd(&S.cnt[key[j]], 1u);
    }
    unsigned long long cross = 0;
#pragma unroll
    for (int j = 0; j < NT; j++) cross |= __ballot(old[j] == thr - 1u);
    if (cross) {
#pragma unroll
      for (int j = 0; j < NT; j++)
        if (old[j] == thr - 1u) mark_chunk(S, key[j], tile);
    }
  } else {
    unsigned long long m[NT], old[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) {
      m[j] = mantissa53(b[j]);
      old[j] = atomicAdd(&S.chunk[key[j]], m[j]);
    }
    unsigned long long wrap = 0;
#pragma unroll
    for (int j = 0; j < NT; j++) wrap |= __ballot(old[j] + m[j] < old[j]);
    if (wrap) {
#pragma unroll
      for (int j = 0; j < NT; j++)
        if (old[j] + m[j] < old[j]) carry_out(S, key[j]);
    }
  }
  return true;
}

// Count mode: transfer the chunks marked during a tile (out of line: rare).
__device__ __noinline__ void flush_marked(LargeShared *S) {
  const int tid = threadIdx.x;
  if (tid < kLChunks / 32) {
    unsigned int bits = S->flushbits[tid];
    if (bits) {
      S->flushbits[tid] = 0u;
      while (bits) {
        const int bp = __ffs(bits) - 1;
        bits &= bits - 1u;
        flush_chunk(*S, (unsigned int)(tid * 32 + bp));
      }
    }
  }
}

// Count mode, end of a tile: barrier, then transfer the chunks marked during
// the tile.  The "marked" flag is kept per tile mod 3 so one barrier per tile
// suffices: flag[t%3] is set during tile t, read after tile t's barrier, and
// cleared during tile t+2.  Carry mode needs nothing here.
template <int MODE>
__device__ __forceinline__ void tile_end(LargeShared &S, unsigned int tile, int tid) {
  if (MODE != kCountMode) return;
  lds_barrier();
  const unsigned int f = S.flag[tile % 3];
  if (tid == 0) S.flag[(tile + 2) % 3] = 0u;
  if (f) {
    flush_marked(&S);
    lds_barrier();
  }
}

// 16-byte streaming loads that do not displace cached data (the input is
// read exactly once).
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ ulonglong2 stream_load(const ulonglong2 *p) {
  const u64x2 v = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(p));
  return make_ulonglong2(v.x, v.y);
}

// Target of the prefetches issued past a stream's last tile (their values are
// never used).  Small and read by every wave, so it stays in L2: pointing
// them here instead of at input already read keeps the kernel's HBM traffic
// at one read of the input.
constexpr int kMaxVec = 8;
static __device__ ulonglong2 g_pad_tile[64 * kMaxVec];

// ---------------------------------------------------------------------------
// Term sources.  A source yields the terms to sum as binary64 bit patterns:
//   kTPV               terms per vector position (one 16-byte load of the
//                      primary input);
//   head_terms(r0)     terms before the first 16-byte-aligned position;
//   at(a, v), pad()    where vector position v (counted from the aligned
//                      term a) and the pad tile are; load(p, k) a
//                      non-temporal load of position k from there,
//                      load_plain(p, k) an ordinary one, zero() empty
//                      registers;
//   terms(V, t)        the kTPV patterns of loaded registers;
//   sload(i), sterm(R) the raw load of scalar term i and its pattern;
//                      sload_nt(i) the same load, non-temporal (the small
//                      body reads every term once).
// Loads and transforms are separate, so a transform (a product, a format
// conversion) never forces an early wait on a prefetch.
// ---------------------------------------------------------------------------

// binary64 terms.
struct SrcF64 {
  const double *x;
  static constexpr int kTPV = 2;
  static constexpr bool kPairs = true;        // the small body reads it in 16-byte pairs
  typedef const ulonglong2 *Ptr;
  typedef ulonglong2 Vec;
  typedef unsigned long long Raw;
  __device__ long long head_terms(long long r0) const {
    return (reinterpret_cast<uintptr_t>(x + r0) & 15) ? 1 : 0;
  }
  __device__ Ptr at(long long a, long long v) const { return reinterpret_cast<Ptr>(x + a) + v; }
  __device__ static Ptr pad() { return g_pad_tile; }
  __device__ static Vec load(Ptr p, long long k) { return stream_load(p + k); }
  __device__ static Vec load_plain(Ptr p, long long k) { return p[k]; }
  __device__ static Vec zero() { return make_ulonglong2(0ull, 0ull); }
  __device__ void terms(const Vec &v, unsigned long long (&t)[2]) const {
    t[0] = v.x;
    t[1] = v.y;
  }
  __device__ Raw sload(long long i) const { return as_bits(x[i]); }
  __device__ Raw sload_nt(long long i) const {
    return (unsigned long long)__builtin_nontemporal_load(reinterpret_cast<const long long *>(x) + i);
  }
  __device__ unsigned long long sterm(Raw r) const { return r; }
};

// Products x[i]*x[i], each rounded to binary64 by the IEEE multiply (the
// paper's squared norm, Performance evaluations).
struct SrcSq : SrcF64 {
  __device__ static unsigned long long sq(unsigned long long b) {
    const double v = __longlong_as_double((long long)b);
    return as_bits(v * v);
  }
  __device__ void terms(const Vec &v, unsigned long long (&t)[2]) const {
    t[0] = sq(v.x);
    t[1] = sq(v.y);
  }
  __device__ unsigned long long sterm(Raw r) const { return sq(r); }
};

// Products x[i]*y[i], each rounded to binary64 (the paper's dot product).
// YA: y + a is 16-byte aligned whenever x + a is; otherwise y is read with
// two 8-byte loads per position.
template <bool YA>
struct SrcDot {
  const double *x;
  const double *y;
  static constexpr int kTPV = 2;
  static constexpr bool kPairs = false;
  struct Ptr {
    const ulonglong2 *p;
    const double *q;
  };
  struct Vec {
    ulonglong2 a, b;
  };
  struct Raw {
    unsigned long long a, b;
  };
  __device__ static unsigned long long mul(unsigned long long u, unsigned long long v) {
    return as_bits(__longlong_as_double((long long)u) * __longlong_as_double((long long)v));
  }
  __device__ long long head_terms(long long r0) const {
    return (reinterpret_cast<uintptr_t>(x + r0) & 15) ? 1 : 0;
  }
  __device__ Ptr at(long long a, long long v) const {
    return Ptr{reinterpret_cast<const ulonglong2 *>(x + a) + v, y + a + 2 * v};
  }
  __device__ static Ptr pad() { return Ptr{g_pad_tile, reinterpret_cast<const double *>(g_pad_tile)}; }
  __device__ static Vec load(Ptr p, long long k) {
    Vec r;
    r.a = stream_load(p.p + k);
    if (YA) {
      r.b = stream_load(reinterpret_cast<const ulonglong2 *>(p.q) + k);
    } else {
      r.b.x = (unsigned long long)__builtin_nontemporal_load(reinterpret_cast<const long long *>(p.q) + 2 * k);
      r.b.y = (unsigned long long)__builtin_nontemporal_load(reinterpret_cast<const long long *>(p.q) + 2 * k + 1);
    }
    return r;
  }
  __device__ static Vec load_plain(Ptr p, long long k) {
    Vec r;
    r.a = p.p[k];
    r.b.x = as_bits(p.q[2 * k]);
    r.b.y = as_bits(p.q[2 * k + 1]);
    return r;
  }
  __device__ static Vec zero() { return Vec{make_ulonglong2(0ull, 0ull), make_ulonglong2(0ull, 0ull)}; }
  __device__ void terms(const Vec &v, unsigned long long (&t)[2]) const {
    t[0] = mul(v.a.x, v.b.x);
    t[1] = mul(v.a.y, v.b.y);
  }
  __device__ Raw sload(long long i) const { return Raw{as_bits(x[i]), as_bits(y[i])}; }
  __device__ Raw sload_nt(long long i) const {
    return Raw{(unsigned long long)__builtin_nontemporal_load(reinterpret_cast<const long long *>(x) + i),
               (unsigned long long)__builtin_nontemporal_load(reinterpret_cast<const long long *>(y) + i)};
  }
  __device__ unsigned long long sterm(Raw r) const { return mul(r.a, r.b); }
};

// binary32 terms, converted exactly to binary64 patterns with integer
// operations (every binary32 value is a binary64 value; Formats).  NaN
// payloads move up by 29 bits, so the largest binary64 NaN pattern maps back
// to the largest binary32 one.
__device__ __forceinline__ unsigned long long f32_to_f64_bits(unsigned int b) {
  const unsigned long long s = (unsigned long long)(b >> 31) << 63;
  const unsigned int e = (b >> 23) & 255u, m = b & 0x7FFFFFu;
  if (e == 255u) return s | (0x7FFull << 52) | ((unsigned long long)m << 29);
  if (e != 0u) return s | ((unsigned long long)(e + 896u) << 52) | ((unsigned long long)m << 29);
  if (m == 0u) return s;
  const int p = 31 - __clz(m);                       // leading bit of a denormal, 0..22
  return s | ((unsigned long long)(p + 874) << 52) | (((unsigned long long)m << (52 - p)) & ((1ull << 52) - 1));
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// binary32 terms for the small-only kernel (scalar loads; the large path of
// binary32 sums is the narrow accumulator below).
struct SrcF32 {
  const float *x;
  static constexpr bool kPairs = false;
  typedef unsigned int Raw;
  __device__ Raw sload(long long i) const { return __float_as_uint(x[i]); }
  __device__ Raw sload_nt(long long i) const {
    return __builtin_nontemporal_load(reinterpret_cast<const unsigned int *>(x) + i);
  }
  __device__ unsigned long long sterm(Raw r) const { return f32_to_f64_bits(r); }
};

// Products x[i]*y[i] of binary32 values, formed exactly in binary64 (the
// operands are converted exactly, and 24-bit by 24-bit significands fit in
// 53 bits with the exponents in range), for the small-only kernel (scalar
// loads; the large path of binary32 dot products is the narrow accumulator
// below).
struct SrcDotF32 {
  const float *x;
  const float *y;
  static constexpr bool kPairs = false;
  struct Raw {
    unsigned int a, b;
  };
  __device__ static unsigned long long mul(unsigned long long u, unsigned long long v) {
    return as_bits(__longlong_as_double((long long)u) * __longlong_as_double((long long)v));
  }
  __device__ Raw sload(long long i) const { return Raw{__float_as_uint(x[i]), __float_as_uint(y[i])}; }
  __device__ Raw sload_nt(long long i) const {
    return Raw{__builtin_nontemporal_load(reinterpret_cast<const unsigned int *>(x) + i),
               __builtin_nontemporal_load(reinterpret_cast<const unsigned int *>(y) + i)};
  }
  __device__ unsigned long long sterm(Raw r) const { return mul(f32_to_f64_bits(r.a), f32_to_f64_bits(r.b)); }
};

// Add the source's terms r0 .. r1 into the workgroup's large accumulator.
// Terms before the first 16-byte-aligned position and after the last whole
// one are added as scalars.  The vector positions are split into one
// contiguous stream per wavefront; a wave's tile is 64*VEC positions (each
// load instruction covers 1 KiB per input), with the next DEPTH tiles'
// loads in flight in a ring of register buffers.  Every wave runs the same
// number of full tiles (count mode puts a workgroup barrier after each); the
// leftover positions of each stream form one last, partial tile.
// One tile's loads for a wave's stream (an index past the last full tile
// reads the pad tile, so loads are unconditional: the compiler's wait
// counts stay exact and a prefetch is never waited for early).
template <int VEC, class Src>
__device__ __forceinline__ void large_tile_load(typename Src::Vec (&bf)[VEC], const Src &src, long long a,
                                                long long ws, long long ntiles, long long t, int lane) {
  constexpr int TILE_W = 64 * VEC;
  const typename Src::Ptr tp = (t < ntiles) ? src.at(a, ws + t * TILE_W) : Src::pad();
#pragma unroll
  for (int j = 0; j < VEC; j++) bf[j] = Src::load(tp, lane + j * 64);
  // keep the scheduler from hoisting work on other buffers above these
  // loads (which would force an early wait on them)
  __builtin_amdgcn_sched_barrier(0);
}

// A range split into begin and add, so that a caller can issue a range's
// first loads (its scalar edge terms and first DEPTH tiles) while it still
// finishes another range, and add the range later.
template <int VEC, int DEPTH, class Src>
struct LargeRange {
  long long a;                  // first vector position's term
  long long nv;                 // vector positions
  long long ws, we;             // this wave's stream of positions
  long long ntiles;             // full tiles per stream
  long long head, tail;         // scalar edge terms
  typename Src::Raw hr;         // this lane's edge term, as loaded
  bool hvalid;
  typename Src::Vec buf[DEPTH][VEC];
};

template <int BLOCK, int VEC, int DEPTH, class Src>
__device__ __forceinline__ void large_range_begin(LargeRange<VEC, DEPTH, Src> &R, const Src &src, long long r0,
                                                  long long r1) {
  constexpr int T = Src::kTPV;
  constexpr int NW = BLOCK / 64;
  constexpr int TILE_W = 64 * VEC;            // positions per wave per tile
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (r1 <= r0) {
    R.a = r0;
    R.nv = R.ws = R.we = R.ntiles = R.head = R.tail = 0;
    R.hvalid = false;
    return;
  }
  long long head = src.head_terms(r0);
  if (head > r1 - r0) head = r1 - r0;
  R.head = head;
  R.a = r0 + head;
  R.nv = (r1 - R.a) / T;
  R.tail = (r1 - R.a) - R.nv * T;
  // scalar terms (at most 2(T-1), on the first lanes of wave 0): loaded now,
  // added last
  R.hr = typename Src::Raw{};
  R.hvalid = false;
  if (tid < head) {
    R.hr = src.sload(r0 + tid);
    R.hvalid = true;
  } else if (tid < head + R.tail) {
    R.hr = src.sload(r1 - R.tail + (tid - head));
    R.hvalid = true;
  }
  const long long q = R.nv / NW;                     // positions per stream (the last takes the rest)
  R.ws = (long long)wave * q;
  R.we = (wave == NW - 1) ? R.nv : R.ws + q;
  R.ntiles = q / TILE_W;                             // full tiles, the same for every wave
  static_assert(VEC <= kMaxVec && VEC + 1 <= kMaxSlots, "pad tile or slow tile too small");
  if (R.ntiles > 0) {
#pragma unroll
    for (int d = 0; d < DEPTH; d++) large_tile_load<VEC>(R.buf[d], src, R.a, R.ws, R.ntiles, d, lane);
  }
}

// Add the source's terms r0 .. r1 into the workgroup's large accumulator.
// Terms before the first 16-byte-aligned position and after the last whole
// one are added as scalars.  The vector positions are split into one
// contiguous stream per wavefront; a wave's tile is 64*VEC positions (each
// load instruction covers 1 KiB per input), with the next DEPTH tiles'
// loads in flight in a ring of register buffers.  Every wave runs the same
// number of full tiles (count mode puts a workgroup barrier after each); the
// leftover positions of each stream form one last, partial tile.
template <int BLOCK, int VEC, int DEPTH, int MODE, class Src>
__device__ __forceinline__ void large_range_add(LargeShared &S, LargeRange<VEC, DEPTH, Src> &R, const Src &src,
                                                int precombine, unsigned int &tile) {
  constexpr int T = Src::kTPV;
  constexpr int NW = BLOCK / 64;
  constexpr int TILE_W = 64 * VEC;            // positions per wave per tile
  constexpr int TILE_V = BLOCK * VEC;         // positions per workgroup per tile
  static_assert(MODE != kCountMode || T * TILE_V < kCap, "tile too large for the count bound");
  constexpr unsigned int THR = (MODE == kCountMode) ? (unsigned int)(kCap - T * TILE_V) : 0u;
  const int tid = threadIdx.x, lane = tid & 63;
  const long long a = R.a, ws = R.ws, we = R.we, ntiles = R.ntiles;
  auto process = [&](const typename Src::Vec(&bf)[VEC], long long t) {
    unsigned long long b[T * VEC];
#pragma unroll
    for (int j = 0; j < VEC; j++) {
      unsigned long long u[T];
      src.terms(bf[j], u);
#pragma unroll
      for (int k = 0; k < T; k++) b[T * j + k] = u[k];
    }
    if (!fast_tile<T * VEC, MODE>(S, b, precombine, tile, lane, THR))
      slow_tile<MODE, Src>(&S, src, a, ws + t * TILE_W + lane, we, 64, VEC, precombine, tile, THR);
    tile_end<MODE>(S, tile++, tid);
  };
  if (ntiles > 0) {
    for (long long t = 0; t < ntiles; t += DEPTH) {
#pragma unroll
      for (int d = 0; d < DEPTH; d++) {
        if (d == 0 || t + d < ntiles) process(R.buf[d], t + d);
        large_tile_load<VEC>(R.buf[d], src, a, ws, ntiles, t + d + DEPTH, lane);
      }
    }
  }
  // leftover: fewer than TILE_W positions per stream (plus up to NW-1 more
  // in the last), so at most VEC+1 slots and fewer terms than one full tile
  if (R.nv > (long long)NW * ntiles * TILE_W) {
    slow_tile<MODE, Src>(&S, src, a, ws + ntiles * TILE_W + lane, we, 64, VEC + 1, precombine, tile, THR);
    tile_end<MODE>(S, tile++, tid);
  }
  if (R.head || R.tail) {
    add_slot<MODE>(S, R.hvalid ? src.sterm(R.hr) : 0ull, R.hvalid, precombine, tile, lane, THR);
    tile_end<MODE>(S, tile++, tid);
  }
}

template <int BLOCK, int VEC, int DEPTH, int MODE, class Src>
__device__ __forceinline__ void accumulate_range(LargeShared &S, const Src &src, long long r0, long long r1,
                                                 int precombine, unsigned int &tile) {
  if (r1 <= r0) return;
  LargeRange<VEC, DEPTH, Src> R;
  large_range_begin<BLOCK>(R, src, r0, r1);
  large_range_add<BLOCK, VEC, DEPTH, MODE>(S, R, src, precombine, tile);
}

// Transfer every used chunk into S.small.  Group gi holds the 64 chunks whose
// exponent field has top six bits gi (both signs, 32 low-exponent values);
// all of them land on small chunks gi .. gi+2, so three wavefront sums and
// three LDS adds serve the group.  With `clean`, the chunks (and counts) read
// are reset to zero, so the next unit of work needs no initialisation.
template <int BLOCK, bool clean, int MODE>
__device__ __forceinline__ void final_flush(LargeShared &S) {
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __syncthreads();
  for (int gi = wave; gi < 64; gi += NW) {
    const unsigned int ix = ((unsigned int)(lane >> 5) << 11) | (unsigned int)(gi * 32 + (lane & 31));
    const unsigned long long C = S.chunk[ix];
    const unsigned int k = (MODE == kCountMode) ? S.cnt[ix] : (C != 0ull ? 1u : 0u);
    if (__ballot(k != 0u) == 0ull) continue;
    long long p0 = 0, p1 = 0, p2 = 0;
    int h = gi;
    if (k) {
      if (MODE == kCountMode) chunk_pieces(ix, C, k, p0, p1, p2, h);
      else mantissa_sum_pieces(ix, C, p0, p1, p2, h);
      if (clean) {
        S.chunk[ix] = 0ull;
        if (MODE == kCountMode) S.cnt[ix] = 0u;
      }
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
// Narrow large superaccumulators for binary32 inputs.  A binary32 term has
// an 8-bit exponent field and a 24-bit significand (Formats), so one chunk
// per (sign, exponent field) makes 512 chunks, and a 64-bit chunk takes 2^40
// significands before it can wrap.  An exact product of two binary32 values
// has a 48-bit significand; split into two 24-bit halves, added to the
// chunks of its exponent and of its exponent + 24, it fits the same scheme
// with 2 x 536 chunks.  A workgroup's range never holds 2^40 terms (the host
// keeps n below 2^40), so the count bound of the large method
// (Large superaccumulator) is never reached: the chunks need no counts and
// no carry checks, every add is a 64-bit LDS add whose old value is not read,
// and the one transfer into the small accumulator is the final one.
//
// KC copies of the table, interleaved per chunk (chunk[key * KC + copy], copy
// = lane mod KC), spread the lanes of one wave that hit the same chunk in the
// same instruction over KC addresses in different banks; with 8 copies this
// beats a wave-wide pre-combine even when every term shares one chunk.
//
// A term kind T gives: the chunks per sign (kKeysPerSign, key = sign *
// kKeysPerSign + k), the k that the transfer reads (kKeyLo .. kKeyHi), the
// binary64 exponent field of the same weight as k (k + kExpOffset), the
// vector interface of the term sources above (head_terms, at, pad, load,
// load_plain), tile() for a tile of present terms, add_vec() for one
// position of any class and add_scalar() for one scalar term.
// ---------------------------------------------------------------------------
// Terms below which no chunk can wrap (checked by the host).
constexpr long long kNarrowMaxTerms = 1ll << 40;

template <int KEYS, int KC>
struct NarrowShared {
  unsigned long long chunk[KEYS * KC];       // sums of 24-bit pieces, chunk[key * KC + copy]
  long long small[68];                       // the workgroup's small accumulator
  unsigned long long spec[3];                // +Inf seen, -Inf seen, max NaN bits (binary64 form)
  unsigned int ticket;
};

template <int KEYS, int KC>
__device__ __forceinline__ void narrow_init(NarrowShared<KEYS, KC> &S, int tid, int block) {
  uint4 *p = reinterpret_cast<uint4 *>(&S.chunk[0]);
  for (int i = tid; i < (int)(sizeof(S.chunk) / 16); i += block) p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (tid < 68) S.small[tid] = 0;
  if (tid < 3) S.spec[tid] = 0ull;
}

// Which of the classes -normal, -0, +0, +normal (v_cmp_class) a value is in.
__device__ __forceinline__ bool f32_normal_or_zero(unsigned int w) {
  return __builtin_amdgcn_classf(__uint_as_float(w), 0x168);
}
__device__ __forceinline__ bool f32_normal(unsigned int w) {
  return __builtin_amdgcn_classf(__uint_as_float(w), 0x108);
}

// binary32 sum terms.  Key k is the exponent field.  A subnormal term has
// the weight of exponent field 1 and goes to that chunk, so the chunks of
// exponent field 0 are never read: the fast path adds zeros there (with the
// implicit bit, like a normal term) instead of branching on them.
struct NarrowSumF32 {
  static constexpr int kKeysPerSign = 256, kKeyLo = 1, kKeyHi = 254, kExpOffset = 925;
  static constexpr int kKeys = 2 * kKeysPerSign;
  const float *x;
  typedef const uint4 *Ptr;
  typedef uint4 Vec;
  __device__ long long head_terms(long long r0) const {
    return (long long)(((16u - (unsigned int)(reinterpret_cast<uintptr_t>(x + r0) & 15)) & 15u) >> 2);
  }
  __device__ Ptr at(long long a, long long v) const { return reinterpret_cast<Ptr>(x + a) + v; }
  __device__ static Ptr pad() { return reinterpret_cast<Ptr>(g_pad_tile); }
  __device__ static Vec load(Ptr p, long long k) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p + k));
    return make_uint4(v.x, v.y, v.z, v.w);
  }
  __device__ static Vec load_plain(Ptr p, long long k) { return p[k]; }
  // one term of any class: infinities and NaNs go to the side words in
  // their binary64 form; zeros add nothing
  template <int KC>
  __device__ static void add_any(NarrowShared<kKeys, KC> &S, unsigned int w, unsigned int copy) {
    const unsigned int e = (w >> 23) & 255u, m = w & 0x7FFFFFu;
    if (e == 255u) {
      note_special(f32_to_f64_bits(w), &S.spec[0], &S.spec[1], &S.spec[2]);
    } else if (e != 0u) {
      atomicAdd(&S.chunk[(w >> 23) * KC + copy], (unsigned long long)(m | 0x800000u));
    } else if (m != 0u) {
      atomicAdd(&S.chunk[((w >> 23) | 1u) * KC + copy], (unsigned long long)m);
    }
  }
  template <int KC>
  __device__ static void add_vec(NarrowShared<kKeys, KC> &S, const Vec &v, unsigned int copy) {
    add_any(S, v.x, copy);
    add_any(S, v.y, copy);
    add_any(S, v.z, copy);
    add_any(S, v.w, copy);
  }
  template <int KC>
  __device__ void add_scalar(NarrowShared<kKeys, KC> &S, long long i, unsigned int copy) const {
    add_any(S, __float_as_uint(x[i]), copy);
  }
  // Common case: every term of the wave is normal or zero (one class test
  // per term); each adds its fraction with the implicit bit set to the
  // chunk of its sign and exponent field.
  template <int VEC, int KC>
  __device__ static void tile(NarrowShared<kKeys, KC> &S, const Vec (&v)[VEC], int lane) {
    const unsigned int copy = (unsigned int)lane & (KC - 1);
    unsigned int w[4 * VEC];
#pragma unroll
    for (int j = 0; j < VEC; j++) {
      w[4 * j] = v[j].x;
      w[4 * j + 1] = v[j].y;
      w[4 * j + 2] = v[j].z;
      w[4 * j + 3] = v[j].w;
    }
    bool plain = true;
#pragma unroll
    for (int j = 0; j < 4 * VEC; j++) plain &= f32_normal_or_zero(w[j]);
    if (__all(plain)) {
#pragma unroll
      for (int j = 0; j < 4 * VEC; j++)
        atomicAdd(&S.chunk[(w[j] >> 23) * KC + copy], (unsigned long long)((w[j] & 0x7FFFFFu) | 0x800000u));
    } else {
#pragma unroll
      for (int j = 0; j < VEC; j++) add_vec(S, v[j], copy);
    }
  }
};

// binary32 dot-product terms.  The product of x = (-1)^sx Mx 2^(ex-150) and
// y = (-1)^sy My 2^(ey-150) (M with the implicit bit, e the exponent field,
// raised to 1 for subnormals) is (-1)^(sx^sy) P 2^(k-300), P = Mx My < 2^48,
// k = ex + ey in 2 .. 508: the low 24 bits of P go to key (sx^sy, k) and the
// high 24 bits to key (sx^sy, k + 24), which has weight 2^24 more.  The
// product is exact (Formats), so any infinity or NaN among the operands
// makes it an infinity or NaN, recorded in its binary64 form (the operands'
// binary64 product).  YA: y + a is 16-byte aligned whenever x + a is;
// otherwise y is read with four 4-byte loads per position.
template <bool YA>
struct NarrowDotF32 {
  static constexpr int kKeysPerSign = 536, kKeyLo = 2, kKeyHi = 532, kExpOffset = 775;
  static constexpr int kKeys = 2 * kKeysPerSign;
  const float *x;
  const float *y;
  struct Ptr {
    const uint4 *p;
    const float *q;
  };
  struct Vec {
    uint4 a, b;
  };
  __device__ long long head_terms(long long r0) const {
    return (long long)(((16u - (unsigned int)(reinterpret_cast<uintptr_t>(x + r0) & 15)) & 15u) >> 2);
  }
  __device__ Ptr at(long long a, long long v) const {
    return Ptr{reinterpret_cast<const uint4 *>(x + a) + v, y + a + 4 * v};
  }
  __device__ static Ptr pad() {
    return Ptr{reinterpret_cast<const uint4 *>(g_pad_tile), reinterpret_cast<const float *>(g_pad_tile)};
  }
  __device__ static Vec load(Ptr p, long long k) {
    Vec r;
    const u32x4 va = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p.p + k));
    r.a = make_uint4(va.x, va.y, va.z, va.w);
    if (YA) {
      const u32x4 vb = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p.q) + k);
      r.b = make_uint4(vb.x, vb.y, vb.z, vb.w);
    } else {
      const unsigned int *q = reinterpret_cast<const unsigned int *>(p.q) + 4 * k;
      r.b = make_uint4(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1),
                       __builtin_nontemporal_load(q + 2), __builtin_nontemporal_load(q + 3));
    }
    return r;
  }
  __device__ static Vec load_plain(Ptr p, long long k) {
    Vec r;
    r.a = p.p[k];
    const unsigned int *q = reinterpret_cast<const unsigned int *>(p.q) + 4 * k;
    r.b = make_uint4(q[0], q[1], q[2], q[3]);
    return r;
  }
  // add P's two halves for key base kb (sign * kKeysPerSign + k)
  template <int KC>
  __device__ static void add_product(NarrowShared<kKeys, KC> &S, unsigned int kb, unsigned int mx, unsigned int my,
                                     unsigned int copy) {
    const unsigned long long P = (unsigned long long)mx * my;          // below 2^48
    unsigned long long *c = &S.chunk[kb * KC + copy];
    atomicAdd(c, P & 0xFFFFFFull);
    atomicAdd(c + 24 * KC, P >> 24);
  }
  // one pair of any class
  template <int KC>
  __device__ static void add_pair(NarrowShared<kKeys, KC> &S, unsigned int wx, unsigned int wy, unsigned int copy) {
    const unsigned int ex = (wx >> 23) & 255u, ey = (wy >> 23) & 255u;
    if (ex == 255u || ey == 255u) {
      note_special(as_bits(__longlong_as_double((long long)f32_to_f64_bits(wx)) *
                           __longlong_as_double((long long)f32_to_f64_bits(wy))),
                   &S.spec[0], &S.spec[1], &S.spec[2]);
      return;
    }
    const unsigned int mx = (wx & 0x7FFFFFu) | (ex ? 0x800000u : 0u);
    const unsigned int my = (wy & 0x7FFFFFu) | (ey ? 0x800000u : 0u);
    if (mx == 0u || my == 0u) return;                                  // a zero product
    const unsigned int k = (ex ? ex : 1u) + (ey ? ey : 1u);
    add_product(S, ((wx ^ wy) >> 31) * kKeysPerSign + k, mx, my, copy);
  }
  template <int KC>
  __device__ static void add_vec(NarrowShared<kKeys, KC> &S, const Vec &v, unsigned int copy) {
    add_pair(S, v.a.x, v.b.x, copy);
    add_pair(S, v.a.y, v.b.y, copy);
    add_pair(S, v.a.z, v.b.z, copy);
    add_pair(S, v.a.w, v.b.w, copy);
  }
  template <int KC>
  __device__ void add_scalar(NarrowShared<kKeys, KC> &S, long long i, unsigned int copy) const {
    add_pair(S, __float_as_uint(x[i]), __float_as_uint(y[i]), copy);
  }
  // Common case: every operand in the wave is a normal number (one class
  // test each).
  template <int VEC, int KC>
  __device__ static void tile(NarrowShared<kKeys, KC> &S, const Vec (&v)[VEC], int lane) {
    const unsigned int copy = (unsigned int)lane & (KC - 1);
    unsigned int wx[4 * VEC], wy[4 * VEC];
#pragma unroll
    for (int j = 0; j < VEC; j++) {
      wx[4 * j] = v[j].a.x;
      wx[4 * j + 1] = v[j].a.y;
      wx[4 * j + 2] = v[j].a.z;
      wx[4 * j + 3] = v[j].a.w;
      wy[4 * j] = v[j].b.x;
      wy[4 * j + 1] = v[j].b.y;
      wy[4 * j + 2] = v[j].b.z;
      wy[4 * j + 3] = v[j].b.w;
    }
    bool normal = true;
#pragma unroll
    for (int j = 0; j < 4 * VEC; j++) normal &= f32_normal(wx[j]) && f32_normal(wy[j]);
    if (__all(normal)) {
#pragma unroll
      for (int j = 0; j < 4 * VEC; j++) {
        const unsigned int k = ((wx[j] >> 23) & 255u) + ((wy[j] >> 23) & 255u);
        add_product(S, ((wx[j] ^ wy[j]) >> 31) * kKeysPerSign + k, (wx[j] & 0x7FFFFFu) | 0x800000u,
                    (wy[j] & 0x7FFFFFu) | 0x800000u, copy);
      }
    } else {
#pragma unroll
      for (int j = 0; j < VEC; j++) add_vec(S, v[j], copy);
    }
  }
};

// Terms [r0, r1) of the source into S.  Same geometry as accumulate_range:
// up to three scalar terms before the first 16-byte boundary and after the
// last, per-wave contiguous streams of 16-byte positions in tiles of 64*VEC,
// DEPTH tiles of loads in flight (past-the-end prefetches read the pad
// tile), and each stream's leftover positions one per lane.
template <int BLOCK, int VEC, int DEPTH, int KC, class T>
__device__ __forceinline__ void narrow_accumulate_range(NarrowShared<T::kKeys, KC> &S, const T &src, long long r0,
                                                        long long r1) {
  constexpr int NW = BLOCK / 64;
  constexpr int TILE_W = 64 * VEC;
  static_assert(VEC <= kMaxVec, "pad tile too small");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned int copy = (unsigned int)lane & (KC - 1);
  if (r1 <= r0) return;
  long long head = src.head_terms(r0);
  if (head > r1 - r0) head = r1 - r0;
  const long long a = r0 + head;
  const long long nv = (r1 - a) / 4;
  const long long tail = (r1 - a) - nv * 4;
  const long long q = nv / NW;
  const long long ws = (long long)wave * q;
  const long long we = (wave == NW - 1) ? nv : ws + q;
  const long long ntiles = q / TILE_W;
  typename T::Vec buf[DEPTH][VEC];
  auto load = [&](typename T::Vec(&bf)[VEC], long long t) {
    const typename T::Ptr tp = (t < ntiles) ? src.at(a, ws + t * TILE_W) : T::pad();
#pragma unroll
    for (int j = 0; j < VEC; j++) bf[j] = T::load(tp, lane + j * 64);
    __builtin_amdgcn_sched_barrier(0);
  };
  if (ntiles > 0) {
#pragma unroll
    for (int d = 0; d < DEPTH; d++) load(buf[d], d);
    for (long long t = 0; t < ntiles; t += DEPTH) {
#pragma unroll
      for (int d = 0; d < DEPTH; d++) {
        if (d == 0 || t + d < ntiles) T::template tile<VEC, KC>(S, buf[d], lane);
        load(buf[d], t + d + DEPTH);
      }
    }
  }
  const typename T::Ptr base = src.at(a, 0);
  for (long long p = ws + ntiles * TILE_W + lane; p < we; p += 64) T::add_vec(S, T::load_plain(base, p), copy);
  if (tid < head) src.add_scalar(S, r0 + tid, copy);
  else if (tid < head + tail) src.add_scalar(S, r1 - tail + (tid - head), copy);
}

// Transfer the chunks with k in kKeyLo .. kKeyHi into S.small.  Chunk k has
// the weight of the binary64 chunk with exponent field k + kExpOffset, so the
// binary64 transfer applies.  Group h (one wave's iteration) holds the 32
// such binary64 exponents with top bits h, of both signs, which land on
// small chunks h .. h+2.
template <int BLOCK, int KC, class T>
__device__ __forceinline__ void narrow_final_flush(NarrowShared<T::kKeys, KC> &S) {
  constexpr int NW = BLOCK / 64;
  constexpr int kH0 = (T::kKeyLo + T::kExpOffset) >> 5, kH1 = (T::kKeyHi + T::kExpOffset) >> 5;
  static_assert(kH1 + 2 < 68 && T::kKeyHi + T::kExpOffset < 2047, "transfer range");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __syncthreads();
  for (int h = kH0 + wave; h <= kH1; h += NW) {
    const unsigned int sign = (unsigned int)lane >> 5;
    const int e64 = 32 * h + (lane & 31);
    const int k = e64 - T::kExpOffset;
    unsigned long long C = 0;
    if (k >= T::kKeyLo && k <= T::kKeyHi) {
#pragma unroll
      for (int c = 0; c < KC; c++) C += S.chunk[(sign * T::kKeysPerSign + (unsigned int)k) * KC + c];
    }
    long long p0 = 0, p1 = 0, p2 = 0;
    int hh = h;
    if (C) mantissa_sum_pieces((sign << 11) | (unsigned int)e64, C, p0, p1, p2, hh);
    p0 = wave_sum_i64(p0);
    p1 = wave_sum_i64(p1);
    p2 = wave_sum_i64(p2);
    if (lane == 0) {
      atomicAdd((unsigned long long *)&S.small[h], (unsigned long long)p0);
      atomicAdd((unsigned long long *)&S.small[h + 1], (unsigned long long)p1);
      atomicAdd((unsigned long long *)&S.small[h + 2], (unsigned long long)p2);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Cross-workgroup hand-over.  Everything one workgroup hands to another goes
// through device-scope atomics (performed at the device's coherence point
// rather than in a per-die cache), and each producer waits for its
// accesses to complete before it takes a ticket.  That orders the hand-over
// without device-wide cache write-back or invalidation (several microseconds
// each here).
// ---------------------------------------------------------------------------
// Wait until this thread's memory operations have completed.
__device__ __forceinline__ void wait_memory() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ unsigned int ticket_add(unsigned int *p, unsigned int k = 1u) {
  return __hip_atomic_fetch_add(p, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Merge into one accumulator (Discussion: add the parts' small
// superaccumulators, round once).  A workgroup adds its 67 chunks into `g`
// with 64-bit integer atomics (exact and order independent), advances the
// ticket by the number of parts its accumulator holds (`parts`), and the one
// that completes the expected count reads and clears `g`, rounds, and writes
// *out.  Called by every thread; returns true in the workgroup that wrote the
// result.  Used where few parts meet (a segment cut by workgroup boundaries,
// a served request's runs of pieces), so the atomics see little contention.
__device__ __forceinline__ bool merge_and_round(long long *s_small, unsigned long long *spec,
                                                unsigned int *s_ticket, GlobalAcc *__restrict__ g,
                                                unsigned int expected, double *__restrict__ out,
                                                unsigned int parts = 1u) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (expected <= 1) {
    if (tid < 64) {
      const unsigned long long r = round_chunks_wave<FmtF64>(s_small, spec[0], spec[1], spec[2], tid);
      if (tid == 0) out[0] = __longlong_as_double((long long)r);
    }
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
  wait_memory();
  __syncthreads();
  if (tid == 0) *s_ticket = ticket_add(&g->ticket, parts);
  __syncthreads();
  const bool last = (*s_ticket + parts == expected);
  __syncthreads();
  if (!last) return false;
  if (tid < kSChunks) s_small[tid] = (long long)atomicExch(&g->chunk[tid], 0ull);
  if (tid == 96) spec[0] = atomicExch(&g->pos_inf, 0ull);
  if (tid == 97) spec[1] = atomicExch(&g->neg_inf, 0ull);
  if (tid == 98) spec[2] = atomicExch(&g->nan_bits, 0ull);
  if (tid == 99) atomicExch(&g->ticket, 0u);
  __syncthreads();
  if (tid < 64) {
    const unsigned long long r = round_chunks_wave<FmtF64>(s_small, spec[0], spec[1], spec[2], tid);
    if (tid == 0) out[0] = __longlong_as_double((long long)r);
  }
  __syncthreads();
  return true;
}

// The same for a single wavefront's small accumulator (acc: 68 chunks in
// LDS, spec: 3 words).  All 64 lanes call it.
__device__ __forceinline__ void wave_merge_and_round(long long *acc, unsigned long long *spec,
                                                     GlobalAcc *__restrict__ g, unsigned int expected,
                                                     double *__restrict__ out, int lane) {
  if (expected > 1) {
    const long long v0 = acc[lane];
    if (v0) atomicAdd(&g->chunk[lane], (unsigned long long)v0);
    if (lane < 3) {
      const long long v1 = acc[64 + lane];
      if (v1) atomicAdd(&g->chunk[64 + lane], (unsigned long long)v1);
    }
    if (lane == 0) {
      if (spec[0]) atomicOr(&g->pos_inf, 1ull);
      if (spec[1]) atomicOr(&g->neg_inf, 1ull);
      if (spec[2]) atomicMax(&g->nan_bits, spec[2]);
    }
    wait_memory();
    unsigned int tk = 0;
    if (lane == 0) tk = ticket_add(&g->ticket);
    tk = (unsigned int)__builtin_amdgcn_readfirstlane((int)tk);
    if (tk != expected - 1) return;
    acc[lane] = (long long)atomicExch(&g->chunk[lane], 0ull);
    if (lane < 3) acc[64 + lane] = (long long)atomicExch(&g->chunk[64 + lane], 0ull);
    if (lane == 0) {
      spec[0] = atomicExch(&g->pos_inf, 0ull);
      spec[1] = atomicExch(&g->neg_inf, 0ull);
      spec[2] = atomicExch(&g->nan_bits, 0ull);
      atomicExch(&g->ticket, 0u);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  }
  const unsigned long long r = round_chunks_wave<FmtF64>(acc, spec[0], spec[1], spec[2], lane);
  if (lane == 0) out[0] = __longlong_as_double((long long)r);
}

// Merge of a whole grid into one accumulator (the one-sum kernels): every
// workgroup adds its small accumulator into `g` with 64-bit device atomics
// (exact and order independent), waits for them to complete and takes a
// ticket; the last one reads and clears `g` with atomic exchanges and
// applies the finisher (Discussion: add the small superaccumulators of the
// parts, finish once).  The adds need no fence: the device-scope atomics
// and the wait for this thread's memory operations order them before the
// ticket.  Returns true in the finishing workgroup.  Called by every thread
// (at least 128).
template <class Fin>
__device__ __forceinline__ bool merge_grid_and_finish(long long *s_small, unsigned long long *spec,
                                                      unsigned int *s_ticket, GlobalAcc *__restrict__ g,
                                                      const Fin &fin) {
  const int tid = threadIdx.x;
  const unsigned int G = gridDim.x;
  __syncthreads();
  if (G == 1) {
    fin(s_small, spec);
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
  wait_memory();
  __syncthreads();
  if (tid == 0) *s_ticket = ticket_add(&g->ticket);
  __syncthreads();
  if (*s_ticket != G - 1u) return false;
  if (tid < kSChunks) s_small[tid] = (long long)atomicExch(&g->chunk[tid], 0ull);
  if (tid == 96) spec[0] = atomicExch(&g->pos_inf, 0ull);
  if (tid == 97) spec[1] = atomicExch(&g->neg_inf, 0ull);
  if (tid == 98) spec[2] = atomicExch(&g->nan_bits, 0ull);
  if (tid == 99) atomicExch(&g->ticket, 0u);
  __syncthreads();
  fin(s_small, spec);
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

// The small-accumulator body of one wavefront.  The wave's accumulator is
// COPIES copies of 68 chunks (small_acc_words<COPIES>() words in LDS); lane l
// adds into copy l % COPIES, so the 64 lanes' adds to one chunk land on
// several addresses instead of one (same-address LDS atomics serialise).
// The copies are copy-major (they measured fewer LDS bank conflicts than
// copies interleaved per chunk), copy_words<COPIES>() 64-bit words apart.
// A 64-bit word w sits on the bank pair w mod 32 of the 64 banks, so copy c
// puts chunk h on pair (stride c + h) mod 32.  With 8 copies the stride is
// 68 (4c: distinct for c < 8); with 16 it is 70 (6c: 16 distinct even
// pairs, where 68 would give copies c and c + 8 the same pairs), so for
// terms on two neighbouring chunks (h of either parity) no two copies
// share a bank pair and only lanes of one copy on one chunk meet.  After
// small_wave_accumulate the first 68 words hold the plain 68 chunks.
template <int COPIES>
constexpr int copy_words() { return COPIES > 8 ? 70 : 68; }
template <int COPIES>
constexpr int small_acc_words() { return copy_words<COPIES>() * COPIES; }

// Zero a wave's accumulator copies and side words.
template <int COPIES>
__device__ __forceinline__ void small_wave_zero(long long *acc, unsigned long long *spec, int lane) {
  constexpr int kWords = small_acc_words<COPIES>();
#pragma unroll
  for (int k = 0; k < (kWords + 63) / 64; k++) {
    const int i = lane + 64 * k;
    if (i < kWords) acc[i] = 0;
  }
  if (lane < 3) spec[lane] = 0ull;
}

// Each lane takes kSmallU terms per batch (term base + 64 j + lane); two
// batches of registers alternate, so the next batch's loads are in flight
// while the current one is added.  A whole batch (base + 64 kSmallU <= hi)
// is loaded from one address per lane with constant offsets.  In the last,
// partial batch the load indices are clamped to the last term, so every
// load is still issued unconditionally and the compiler's wait counts stay
// exact; clamped lanes add nothing.
constexpr int kSmallU = 8;
template <class Src>
__device__ __forceinline__ void small_batch_load(typename Src::Raw (&b)[kSmallU], const Src &src, long long base,
                                                 long long hi, int lane) {
  if (base + 64 * kSmallU <= hi) {
#pragma unroll
    for (int j = 0; j < kSmallU; j++) b[j] = src.sload_nt(base + lane + (long long)j * 64);
  } else {
    const long long last = hi - 1;
#pragma unroll
    for (int j = 0; j < kSmallU; j++) {
      long long i = base + (long long)j * 64 + lane;
      i = i < last ? i : last;
      b[j] = src.sload_nt(i);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}
// Add one lane's K terms (bit patterns; a 0 adds nothing).  A batch of
// finite terms takes one branch-free path; only a batch holding an infinity
// or NaN (exponent field 2047) goes term by term.
template <int K>
__device__ __forceinline__ unsigned int umax_of(const unsigned int (&e)[K]) {
  unsigned int m = e[0];
#pragma unroll
  for (int j = 1; j < K; j++) m = m > e[j] ? m : e[j];
  return m;
}
template <int K>
__device__ __forceinline__ unsigned int umin_of(const unsigned int (&e)[K]) {
  unsigned int m = e[0];
#pragma unroll
  for (int j = 1; j < K; j++) m = m < e[j] ? m : e[j];
  return m;
}
template <int K>
__device__ __forceinline__ void small_terms_add(long long *mine, unsigned long long *spec,
                                                const unsigned long long (&t)[K]) {
  unsigned int e[K];
#pragma unroll
  for (int j = 0; j < K; j++) e[j] = term_exp(t[j]);
  if (!__any(umax_of(e) == 2047u)) {
#pragma unroll
    for (int j = 0; j < K; j++) {
      int h;
      long long plo, phi;
      term_pieces_e(t[j], e[j], h, plo, phi);
      atomicAdd((unsigned long long *)&mine[h], (unsigned long long)plo);
      atomicAdd((unsigned long long *)&mine[h + 1], (unsigned long long)phi);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < K; j++) {
    if (is_special(t[j])) {
      note_special(t[j], &spec[0], &spec[1], &spec[2]);
    } else {
      int h;
      long long plo, phi;
      term_pieces_e(t[j], e[j], h, plo, phi);
      atomicAdd((unsigned long long *)&mine[h], (unsigned long long)plo);
      atomicAdd((unsigned long long *)&mine[h + 1], (unsigned long long)phi);
    }
  }
}

// The range of exponent fields of the terms a lane has loaded, from which
// the wave's window of touched small chunks follows (small_window).
// Lanes past the end of a ragged batch load terms of the range too (their
// indices are clamped), so every term noted belongs to the sum.  NoWin
// notes nothing.
struct NoWin {
  template <int K>
  __device__ __forceinline__ void note(const unsigned long long (&)[K]) {}
};
struct SmallWin {
  unsigned int mn = 0xFFFFu, mx = 0u;
  template <int K>
  __device__ __forceinline__ void note(const unsigned long long (&t)[K]) {
    unsigned int e[K];
#pragma unroll
    for (int j = 0; j < K; j++) e[j] = term_exp(t[j]);
    const unsigned int a = umin_of(e), b = umax_of(e);
    mn = mn < a ? mn : a;
    mx = mx > b ? mx : b;
  }
};

// Add one batch.  Lanes past hi in the last batch carry the term 0.
template <class Src, class Win>
__device__ __forceinline__ void small_batch_add(long long *mine, unsigned long long *spec, const Src &src,
                                                const typename Src::Raw (&b)[kSmallU], long long base, long long hi,
                                                int lane, Win &w) {
  unsigned long long t[kSmallU], u[kSmallU];
  const bool whole = base + 64 * kSmallU <= hi;
#pragma unroll
  for (int j = 0; j < kSmallU; j++) {
    u[j] = src.sterm(b[j]);
    t[j] = (!whole && base + (long long)j * 64 + lane >= hi) ? 0ull : u[j];
  }
  w.note(u);
  small_terms_add(mine, spec, t);
}

// Sources with kPairs (a single binary64 array) are read two terms per
// 16-byte non-temporal load, as the large kernel reads them: a batch is
// kSmallU / 2 vectors per lane (vector v = vb + 64 j + lane of the aligned
// part, terms 2v and 2v + 1), so a batch still holds kSmallU terms per lane.
constexpr int kPairV = kSmallU / 2;
template <class Src>
__device__ __forceinline__ void pair_batch_load_whole(ulonglong2 (&v)[kPairV], const Src &src, long long a,
                                                      long long vb, int lane) {
  const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(src.x + a);
#pragma unroll
  for (int j = 0; j < kPairV; j++) v[j] = stream_load(p + vb + lane + (long long)j * 64);
  __builtin_amdgcn_sched_barrier(0);
}
// Any batch, whole or not: indices clamped to the last vector, so the loads
// are issued unconditionally and there is no branch (whose join would make
// the compiler's wait counts cover these loads before the batch in hand).
template <class Src>
__device__ __forceinline__ void pair_batch_load_clamped(ulonglong2 (&v)[kPairV], const Src &src, long long a,
                                                        long long vb, long long nv, int lane) {
  const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(src.x + a);
  const long long last = nv - 1;
#pragma unroll
  for (int j = 0; j < kPairV; j++) {
    long long i = vb + (long long)j * 64 + lane;
    i = i < last ? i : last;
    v[j] = stream_load(p + i);
  }
  __builtin_amdgcn_sched_barrier(0);
}
template <class Src, class Win>
__device__ __forceinline__ void pair_batch_add_whole(long long *mine, unsigned long long *spec, const Src &src,
                                                     const ulonglong2 (&v)[kPairV], Win &w) {
  unsigned long long t[kSmallU];
#pragma unroll
  for (int j = 0; j < kPairV; j++) {
    t[2 * j] = src.sterm(v[j].x);
    t[2 * j + 1] = src.sterm(v[j].y);
  }
  w.note(t);
  small_terms_add(mine, spec, t);
}
template <class Src, class Win>
__device__ __forceinline__ void pair_batch_add(long long *mine, unsigned long long *spec, const Src &src,
                                               const ulonglong2 (&v)[kPairV], long long vb, long long nv, int lane,
                                               Win &w) {
  unsigned long long t[kSmallU], u[kSmallU];
  const bool whole = vb + 64 * kPairV <= nv;
#pragma unroll
  for (int j = 0; j < kPairV; j++) {
    const bool off = !whole && vb + (long long)j * 64 + lane >= nv;
    u[2 * j] = src.sterm(v[j].x);
    u[2 * j + 1] = src.sterm(v[j].y);
    t[2 * j] = off ? 0ull : u[2 * j];
    t[2 * j + 1] = off ? 0ull : u[2 * j + 1];
  }
  w.note(u);
  small_terms_add(mine, spec, t);
}
template <int COPIES>
__device__ __forceinline__ void small_carry_all(long long *acc, int lane) {
#pragma unroll
  for (int c = 0; c < COPIES; c++) carry_step(acc + copy_words<COPIES>() * c, lane);
}

// One wave's pass over a range [lo, hi) (hi > lo) of a kPairs source, split
// in two so that a wave can issue a range's first loads early (while it still
// finishes another range): pair_range_begin issues the loads of the first
// batch and of the two edge terms (one before the first 16-byte boundary,
// one after the last whole vector, added by lanes 0 and 1), and
// pair_range_add adds every term of the range into the accumulator copies.
template <class Src>
struct PairRange {
  long long a;                  // first term of the aligned part
  long long nv;                 // whole 16-byte vectors from a
  bool fix;                     // this lane adds an edge term
  typename Src::Raw fr;         // that term, as loaded
  ulonglong2 A[kPairV];         // the first batch
};
template <class Src>
__device__ __forceinline__ void pair_range_begin(PairRange<Src> &r, const Src &src, long long lo, long long hi,
                                                 int lane) {
  const long long head = (reinterpret_cast<uintptr_t>(src.x + lo) & 15) ? 1 : 0;
  r.a = lo + head < hi ? lo + head : hi;
  r.nv = (hi - r.a) / 2;
  const long long tail = (hi - r.a) - 2 * r.nv;
  r.fix = (lane == 0 && head) || (lane == 1 && tail);
  // the edge loads are clamped into the range, so issued unconditionally
  r.fr = src.sload_nt(lane == 1 ? hi - 1 : lo);
  if (r.nv > 0) pair_batch_load_clamped(r.A, src, r.a, 0, r.nv, lane);
}
template <int COPIES, class Src, class Win = NoWin>
__device__ __forceinline__ void pair_range_add(long long *acc, unsigned long long *spec, const Src &src,
                                               PairRange<Src> &r, int lane, Win &&w = Win{}) {
  constexpr int kEvery = 3 * COPIES;             // as in small_wave_accumulate
  constexpr long long kVB = 64 * kPairV;
  long long *mine = acc + copy_words<COPIES>() * (lane % COPIES);
  int batches = 0;
  const auto tick = [&]() {
    if (++batches == kEvery) {
      batches = 0;
      small_carry_all<COPIES>(acc, lane);
    }
  };
  if (r.nv > 0) {
    ulonglong2 B[kPairV];
    long long vb = 0;
    // Steady state: each pass loads and adds two whole batches, the next
    // batch's loads in flight during each add, with no clamps or masks.
    // It always leaves the batch in hand in r.A.
    while (vb + 3 * kVB <= r.nv) {
      pair_batch_load_whole(B, src, r.a, vb + kVB, lane);
      pair_batch_add_whole(mine, spec, src, r.A, w);
      tick();
      pair_batch_load_whole(r.A, src, r.a, vb + 2 * kVB, lane);
      pair_batch_add_whole(mine, spec, src, B, w);
      tick();
      vb += 2 * kVB;
    }
    // r.A holds the batch at vb; at most two follow, the last maybe ragged.
    if (vb + kVB < r.nv) {
      pair_batch_load_clamped(B, src, r.a, vb + kVB, r.nv, lane);
      pair_batch_add_whole(mine, spec, src, r.A, w);
      tick();
      vb += kVB;
      if (vb + kVB < r.nv) {
        pair_batch_load_clamped(r.A, src, r.a, vb + kVB, r.nv, lane);
        pair_batch_add_whole(mine, spec, src, B, w);
        tick();
        pair_batch_add(mine, spec, src, r.A, vb + kVB, r.nv, lane, w);
      } else {
        pair_batch_add(mine, spec, src, B, vb, r.nv, lane, w);
      }
    } else {
      pair_batch_add(mine, spec, src, r.A, vb, r.nv, lane, w);
    }
  }
  // the edge terms: lanes 0 and 1 only (the others would add zeros); every
  // lane's edge load is a term of the range
  const unsigned long long ft[1] = {src.sterm(r.fr)};
  w.note(ft);
  if (r.fix) small_terms_add(mine, spec, ft);
}

// The end of a wave's sum: carry steps of the copies (skipped when the range
// had fewer than 1024 terms and `direct`; see small_wave_accumulate), then
// the copies added into the first 68 words.
template <int COPIES>
__device__ __forceinline__ void small_wave_finish(long long *acc, int lane, bool skip_carry) {
  if (COPIES == 1) {
    if (!skip_carry) carry_step(acc, lane);
    return;
  }
  __builtin_amdgcn_wave_barrier();
  long long A, B = 0;
  if (skip_carry) {
    // the copies' total stays below 1023 * 2^52 (see small_wave_accumulate)
    long long t0 = 0, t1 = 0;
#pragma unroll
    for (int c = 0; c < COPIES; c++) {
      t0 += acc[copy_words<COPIES>() * c + lane];
      if (lane < 4) t1 += acc[copy_words<COPIES>() * c + 64 + lane];
    }
    A = t0;
    B = t1;
  } else {
    // The copies are added with one parallel carry step folded in, in one
    // pass: every word (below 2^63) splits into its low 32 bits, which stay
    // in its chunk, and its high part, which moves one chunk up (chunk 66
    // keeps its high part).  Over the copies the low sums stay below
    // COPIES * 2^32 and the high sums below COPIES * 2^31 in magnitude, so
    // nothing wraps; the value is the copies' total, with every chunk below
    // 2^38.
    long long lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
#pragma unroll
    for (int c = 0; c < COPIES; c++) {
      const long long v0 = acc[copy_words<COPIES>() * c + lane];
      lo0 += v0 & 0xFFFFFFFFll;
      hi0 += v0 >> 32;
      if (lane < 4) {
        const long long v1 = acc[copy_words<COPIES>() * c + 64 + lane];
        lo1 += v1 & 0xFFFFFFFFll;
        hi1 += v1 >> 32;
      }
    }
    // chunk i receives the high sum of chunk i - 1 (lane i - 1 of the
    // 64-chunk row; chunk 64 from lane 63)
    const long long cA = (long long)shr1_u64((unsigned long long)hi0, 0ull);
    const long long hiA63 = (long long)readlane_u64((unsigned long long)hi0, 63);
    const long long cB = (long long)shr1_u64((unsigned long long)hi1, (unsigned long long)hiA63);
    A = lo0 + cA;
    if (lane < 2) B = lo1 + cB;
    else if (lane == 2) B = lo1 + hi1 * 4294967296ll + cB;
  }
  __builtin_amdgcn_wave_barrier();
  acc[lane] = A;
  if (lane < 4) acc[64 + lane] = B;
  __builtin_amdgcn_wave_barrier();
}

// The window of a wave's sum: small chunks [hb, hb + W) hold everything the
// sum can occupy once the copies are added with the final carry folded in.
// A term of exponent field e adds pieces to chunks e_eff >> 5 and the next,
// and the fold moves high parts one chunk further, so the exponent range of
// the terms bounds the window, provided no carry step ran on the way (each
// moves high parts one chunk up): the range has at most win_max_terms
// terms.  Returns false when the finish must cover every chunk: an infinity
// or NaN among the terms (their side words are set), a window wider than
// kWinRounds * 64 / COPIES chunks, or a longer range.  W = 0: no term.
constexpr int kWinRounds = 2;
template <int COPIES>
constexpr long long win_max_terms() { return (3LL * COPIES - 1) * 64 * kSmallU; }

template <int COPIES>
__device__ __forceinline__ bool small_window(const SmallWin &w, long long n, int &hb, int &W) {
  const unsigned int mn = wave_min_u32(w.mn), mx = wave_max_u32(w.mx);
  hb = 0;
  W = 0;
  if (mn > mx) return true;                                  // no term
  if (mx >= 2047u || n > win_max_terms<COPIES>()) return false;
  hb = (int)((mn > 1u ? mn : 1u) >> 5);
  W = (int)((mx > 1u ? mx : 1u) >> 5) + 3 - hb;
  return W * COPIES <= 64 * kWinRounds;
}

// Sum over each group of COPIES consecutive lanes (8 or 16, within a row of
// 16), left in every lane of the group: swap neighbours, swap pairs, mirror
// the half-rows (and, for 16, the rows).
template <int COPIES>
__device__ __forceinline__ long long group_sum_i64(long long v) {
  static_assert(COPIES == 8 || COPIES == 16, "group of 8 or 16 lanes");
  unsigned long long u = (unsigned long long)v;
  u += dpp_mov_u64<0xB1>(u);
  u += dpp_mov_u64<0x4E>(u);
  u += dpp_mov_u64<0x141>(u);
  if (COPIES == 16) u += dpp_mov_u64<0x140>(u);
  return (long long)u;
}

// small_wave_finish for a sum inside its window (small_window true; every
// copy zero outside it): lane l reads copy l % COPIES of chunk hb + k G +
// l / COPIES (G = 64 / COPIES chunks per round), the copies are added across
// each lane group, and the first lane of the group writes the chunk's total
// into the first copy while the others clear their words.  With the carry
// folded in (skip_carry false), each word splits into its low 32 bits and
// its high part as in small_wave_finish, and a chunk's total takes the high
// sum of the chunk below (from the last lane of the group below: every lane
// of a group holds its sums).  The top chunk of the window received no piece,
// so no high part leaves it.  After it the first copy holds the sum (the
// other copies are zero), each chunk below 2^37 in magnitude.
template <int COPIES>
__device__ __forceinline__ void small_wave_finish_window(long long *acc, int lane, bool skip_carry, int hb, int W) {
  constexpr int G = 64 / COPIES;
  const int c = lane % COPIES;
  long long *mine = acc + copy_words<COPIES>() * c + hb;
  unsigned long long below = 0ull;          // high sum of the chunk below the round's first
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int k = 0; k < kWinRounds; k++) {
    if (k * G >= W) break;
    const int r = k * G + lane / COPIES;
    const bool valid = r < W;
    long long v = 0;
    if (valid) v = mine[r];
    long long t;
    if (skip_carry) {
      t = group_sum_i64<COPIES>(v);
    } else {
      const long long lo = group_sum_i64<COPIES>(v & 0xFFFFFFFFll);
      const long long hi = group_sum_i64<COPIES>(v >> 32);
      t = lo + (long long)shr1_u64((unsigned long long)hi, below);
      below = readlane_u64((unsigned long long)hi, 63);
    }
    if (valid) mine[r] = c == 0 ? t : 0ll;
  }
  __builtin_amdgcn_wave_barrier();
}

// Clear the first copy's window after the sum was rounded (the rest of the
// accumulator is zero already).
__device__ __forceinline__ void small_window_clear(long long *acc, int lane, int hb, int W) {
  __builtin_amdgcn_wave_barrier();
  if (lane < W) acc[hb + lane] = 0;
  __builtin_amdgcn_wave_barrier();
}

// Wave adds the source's terms lo .. hi into acc (small_acc_words<COPIES>()
// words, zeroed by the caller); specials into spec[3].  On return the sum is
// in the first 68 words, each below COPIES * 2^33 in magnitude.  With
// `direct` (the caller rounds the result and merges it nowhere), a range of
// fewer than 1024 terms skips the carry steps of the copies: every term adds
// at most one piece below 2^52 to a given chunk, so each chunk's total over
// all copies stays below 1023 * 2^52 < 2^62, which the rounding accepts.
// With ZERO the accumulator is cleared here, after the first batch's loads
// are issued, so that the clearing overlaps their latency (the caller then
// need not zero it).
template <bool ON>
struct WinOf {
  using T = NoWin;
};
template <>
struct WinOf<true> {
  using T = SmallWin;
};

template <int COPIES, class Src, bool ZERO = false>
__device__ __forceinline__ void small_wave_accumulate(long long *acc, unsigned long long *spec, const Src &src,
                                                      long long lo, long long hi, int lane, bool direct = false) {
  // a copy's chunk receives at most 64 / COPIES pieces below 2^52 per
  // 64-term step; a carry step after every kEvery batches keeps it below
  // 1536 * 2^52 < 2^63
  constexpr int kEvery = 3 * COPIES;
  static_assert(64 % COPIES == 0 && kEvery * kSmallU * (64 / COPIES) <= 1536, "carry interval");
  constexpr bool kWin = COPIES == 8 || COPIES == 16;     // windowed finish (group sums of 8 or 16 lanes)
  typename WinOf<kWin>::T w;
  long long *mine = acc + copy_words<COPIES>() * (lane % COPIES);
  if (ZERO && !(hi > lo)) small_wave_zero<COPIES>(acc, spec, lane);
  if constexpr (Src::kPairs) {
    if (hi > lo) {
      PairRange<Src> r;
      pair_range_begin(r, src, lo, hi, lane);
      if (ZERO) small_wave_zero<COPIES>(acc, spec, lane);
      pair_range_add<COPIES>(acc, spec, src, r, lane, w);
    }
  } else if (hi > lo) {
    constexpr long long kB = 64 * kSmallU;
    typename Src::Raw A[kSmallU], B[kSmallU];
    small_batch_load(A, src, lo, hi, lane);
    if (ZERO) small_wave_zero<COPIES>(acc, spec, lane);
    int batches = 0;
    for (long long base = lo;;) {
      small_batch_load(B, src, base + kB, hi, lane);
      small_batch_add(mine, spec, src, A, base, hi, lane, w);
      base += kB;
      if (++batches == kEvery) {
        batches = 0;
        small_carry_all<COPIES>(acc, lane);
      }
      if (base >= hi) break;
      small_batch_load(A, src, base + kB, hi, lane);
      small_batch_add(mine, spec, src, B, base, hi, lane, w);
      base += kB;
      if (++batches == kEvery) {
        batches = 0;
        small_carry_all<COPIES>(acc, lane);
      }
      if (base >= hi) break;
    }
  }
  if constexpr (kWin) {
    int hb, W;
    if (small_window<COPIES>(w, hi - lo, hb, W)) {
      small_wave_finish_window<COPIES>(acc, lane, direct && hi - lo < 1024, hb, W);
      return;
    }
  }
  small_wave_finish<COPIES>(acc, lane, direct && hi - lo < 1024);
}

// ---------------------------------------------------------------------------
// Finishers: what the workgroup holding the merged small accumulator does
// with it.  Called by every thread of that workgroup; c is 68 chunks in LDS
// (|c[i]| < 2^62) and spec the 3 side words.
// ---------------------------------------------------------------------------

// Round to binary64 (Small: obtaining the correctly rounded result).
struct FinF64 {
  double *out;
  __device__ void operator()(long long *c, unsigned long long *spec) const {
    const int tid = threadIdx.x;
    if (tid < 64) {
      const unsigned long long r = round_chunks_wave<FmtF64>(c, spec[0], spec[1], spec[2], tid);
      if (tid == 0) out[0] = __longlong_as_double((long long)r);
    }
  }
};

// Round to binary32 (the single-precision variant named in the
// Introduction).
struct FinF32 {
  float *out;
  __device__ void operator()(long long *c, unsigned long long *spec) const {
    const int tid = threadIdx.x;
    if (tid < 64) {
      const unsigned long long r = round_chunks_wave<FmtF32>(c, spec[0], spec[1], spec[2], tid);
      if (tid == 0) out[0] = __uint_as_float((unsigned int)r);
    }
  }
};

// The exact sum divided by n, rounded once (Discussion); n = 0 gives +0.
struct FinMean {
  double *out;
  unsigned long long n;
  __device__ void operator()(long long *c, unsigned long long *spec) const {
    const int tid = threadIdx.x;
    if (tid < 64) {
      const unsigned long long r = n ? round_mean_wave(c, spec[0], spec[1], spec[2], n, tid) : 0ull;
      if (tid == 0) out[0] = __longlong_as_double((long long)r);
    }
  }
};

// Add into a caller-owned accumulator (the mergeable state of the streaming
// interface): acc += c with integer additions, one parallel carry step to
// keep every chunk below 2^33, infinity flags ORed, the NaN word maximised
// (Discussion: small superaccumulators of parts are added).  The stream
// orders the calls that touch one accumulator, so plain accesses suffice.
struct FinAcc {
  GlobalAcc *acc;
  __device__ void operator()(long long *c, unsigned long long *spec) const {
    const int tid = threadIdx.x;
    for (int i = tid; i < 68; i += blockDim.x) c[i] += (long long)acc->chunk[i];
    __syncthreads();
    if (tid < 64) carry_step(c, tid);
    __syncthreads();
    for (int i = tid; i < 68; i += blockDim.x) acc->chunk[i] = (unsigned long long)c[i];
    if (tid == 0) {
      acc->pos_inf |= spec[0];
      acc->neg_inf |= spec[1];
      if (spec[2] > acc->nan_bits) acc->nan_bits = spec[2];
    }
  }
};

}  // namespace exsum
