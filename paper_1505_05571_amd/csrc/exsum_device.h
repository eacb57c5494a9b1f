// exsum_device.h -- device-side building blocks of the exact sum (gfx950).
//
// Value model (section "Floating-point and integer formats"): a finite
// binary64 term with bit pattern b has sign s = b>>63, exponent field
// e = (b>>52)&2047 and mantissa field m = b & (2^52-1).  With e_eff = max(e,1)
// and M = m + [e != 0] 2^52 its value is (-1)^s M 2^(e_eff-1075).
//
// Small superaccumulator (section "Exact summation using a small
// superaccumulator"): 67 signed 64-bit chunks c_i, value sum c_i 2^(32i-1075).
// A mantissa placed at exponent e_eff lands at chunk e_eff>>5, shifted left by
// e_eff&31 bits, and spills into the next one or two chunks.
//
// Large superaccumulator (section "Faster exact summation of many terms with a
// large superaccumulator"): 4096 chunks indexed by the top 12 bits (sign and
// exponent) of the pattern, each holding the plain 64-bit sum of the raw bit
// patterns added to it, plus a count of those adds.  After k <= 4096 adds the
// sum of the mantissa fields is chunk - k*(index<<52) (mod 2^64), which is
// below 2^64; the implicit bits add k*2^52 for normal exponents.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exsum_internal.h"

namespace exsum {

constexpr int kSChunks = 67;          // small accumulator chunks
constexpr int kLChunks = 4096;        // large accumulator chunks
constexpr int kCap = 4096;            // raw-pattern adds one large chunk holds exactly

// Merge target shared by the workgroups of one sum (or of one segment's
// tiles).  Every field is updated with device-scope atomics and left zeroed
// by the workgroup that finishes last, so the next call starts clean.
struct alignas(64) GlobalAcc {
  unsigned long long chunk[68];        // int64 two's complement sums (67 used)
  unsigned long long pos_inf;          // nonzero if any +Inf term
  unsigned long long neg_inf;          // nonzero if any -Inf term
  unsigned long long nan_bits;         // max over NaN terms of (bits & ~sign)
  unsigned int ticket;                 // workgroups finished so far
  unsigned int pad0;
};
static_assert(sizeof(GlobalAcc) == 576, "GlobalAcc layout");

// ---- synchronisation -------------------------------------------------------

// Workgroup barrier that waits only for this wave's LDS traffic.  Global loads
// issued ahead of the barrier (the next tile) stay in flight.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---- wavefront reductions (all 64 lanes active) ----------------------------

// Move a 64-bit value across lanes with a DPP pattern (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_mov_u64(unsigned long long v) {
  const unsigned int lo = (unsigned int)__builtin_amdgcn_mov_dpp((int)(unsigned int)v, CTRL, 0xF, 0xF, false);
  const unsigned int hi = (unsigned int)__builtin_amdgcn_mov_dpp((int)(unsigned int)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int lane) {
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)v, lane);
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

// A value that every active lane holds (read from LDS, say), made
// wave-uniform for the compiler, so that loops and branches on it are scalar.
__device__ __forceinline__ long long uniform_i64(long long v) {
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)(unsigned long long)v);
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readfirstlane((int)(unsigned int)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes (mod 2^64), returned as a wave-uniform value.
// Within each row of 16 lanes: swap neighbours, swap pairs, mirror the
// half-rows, mirror the row (every lane then holds its row sum); the four
// row sums are then read out and added.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  v += dpp_mov_u64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov_u64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov_u64<0x141>(v);   // row_half_mirror
  v += dpp_mov_u64<0x140>(v);   // row_mirror
  return readlane_u64(v, 0) + readlane_u64(v, 16) + readlane_u64(v, 32) + readlane_u64(v, 48);
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
  return (long long)wave_sum_u64((unsigned long long)v);
}

// Minimum and maximum over the 64 lanes, the same way (wave-uniform).
__device__ __forceinline__ unsigned int wave_min_u32(unsigned int v) {
  unsigned int u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false); v = v < u ? v : u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false); v = v < u ? v : u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false); v = v < u ? v : u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false); v = v < u ? v : u;
  unsigned int m = (unsigned int)__builtin_amdgcn_readlane((int)v, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    const unsigned int x = (unsigned int)__builtin_amdgcn_readlane((int)v, r);
    m = m < x ? m : x;
  }
  return m;
}
__device__ __forceinline__ unsigned int wave_max_u32(unsigned int v) {
  unsigned int u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false); v = v > u ? v : u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false); v = v > u ? v : u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false); v = v > u ? v : u;
  u = (unsigned int)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false); v = v > u ? v : u;
  unsigned int m = (unsigned int)__builtin_amdgcn_readlane((int)v, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    const unsigned int x = (unsigned int)__builtin_amdgcn_readlane((int)v, r);
    m = m > x ? m : x;
  }
  return m;
}

// ---- large chunk -> three small-chunk pieces -------------------------------

// Chunk index ix (sign<<11 | exponent field), raw-pattern sum C of k adds.
// Produces signed pieces for small chunks hi, hi+1, hi+2 (each |piece| < 2^32).
__device__ __forceinline__ void chunk_pieces(unsigned int ix, unsigned long long C, unsigned int k,
                                             long long &p0, long long &p1, long long &p2, int &hi) {
  const unsigned int e = ix & 2047u;
  const unsigned int e_eff = e ? e : 1u;
  // sum of the 52-bit mantissa fields (exact: k <= 4096 keeps it below 2^64)
  const unsigned long long T = C - (unsigned long long)k * ((unsigned long long)ix << 52);
  const unsigned long long imp = e ? ((unsigned long long)k << 52) : 0ull;
  const unsigned long long qlo = T + imp;           // 65-bit total mantissa sum
  const unsigned long long qhi = qlo < T ? 1ull : 0ull;
  const unsigned int lo = e_eff & 31u;
  hi = (int)(e_eff >> 5);
  const unsigned long long low64 = qlo << lo;
  const unsigned long long top = (qhi << lo) | (lo ? (qlo >> (64 - lo)) : 0ull);
  long long a = (long long)(low64 & 0xFFFFFFFFull);
  long long b = (long long)(low64 >> 32);
  long long c = (long long)top;
  const long long neg = -(long long)(ix >> 11);      // 0 or -1
  p0 = (a ^ neg) - neg;
  p1 = (b ^ neg) - neg;
  p2 = (c ^ neg) - neg;
}

// A chunk holding the plain sum T (< 2^64) of the 53-bit mantissas of terms
// with index ix: three signed pieces for small chunks hi .. hi+2.
__device__ __forceinline__ void mantissa_sum_pieces(unsigned int ix, unsigned long long T, long long &p0,
                                                    long long &p1, long long &p2, int &hi) {
  const unsigned int e = ix & 2047u;
  const unsigned int e_eff = e ? e : 1u;
  const unsigned int lo = e_eff & 31u;
  hi = (int)(e_eff >> 5);
  const unsigned long long low64 = T << lo;
  const unsigned long long top = lo ? (T >> (64 - lo)) : 0ull;
  const long long a = (long long)(low64 & 0xFFFFFFFFull);
  const long long b = (long long)(low64 >> 32);
  const long long c = (long long)top;
  const long long neg = -(long long)(ix >> 11);
  p0 = (a ^ neg) - neg;
  p1 = (b ^ neg) - neg;
  p2 = (c ^ neg) - neg;
}

// ---- one term -> two small-chunk pieces (the small-superaccumulator add) ---

// For a finite term: chunk index h = e_eff>>5 and two pieces with
// plo + phi 2^32 = (-1)^s M 2^(e_eff & 31): the signed significand M' =
// (-1)^s M is shifted left by e_eff & 31, plo is the low 32 bits of that
// (0 <= plo < 2^32, for chunk h) and phi the rest, an arithmetic shift
// (|phi| < 2^52, for chunk h+1).  The sign is applied once, without a branch
// (Discussion), before the split.  The exponent field e is taken apart from
// the rest so that a caller can test it for the special value 2047 first
// and reuse it here.
__device__ __forceinline__ unsigned int term_exp(unsigned long long b) {
  return __builtin_amdgcn_ubfe((unsigned int)(b >> 32), 20u, 11u);
}
__device__ __forceinline__ void term_pieces_e(unsigned long long b, unsigned int e, int &h, long long &plo,
                                              long long &phi) {
  const unsigned int e_eff = e > 1u ? e : 1u;
  // min(e, 1) (0 for a denormal) and e_eff >> 5 as single instructions: the
  // compiler would turn the first into a compare and select and fold the
  // second into the LDS address as a shift and mask; this way the hidden bit
  // joins the significand with one shift-or and the address is one
  // shift-add
  unsigned int hidden, hh;
  asm("v_min_u32 %0, 1, %1" : "=v"(hidden) : "v"(e));
  asm("v_bfe_u32 %0, %1, 5, 6" : "=v"(hh) : "v"(e_eff));
  const unsigned int mhi = (hidden << 20) | ((unsigned int)(b >> 32) & 0xFFFFFu);
  const unsigned long long M = ((unsigned long long)mhi << 32) | (unsigned int)b;
  const unsigned int lo = e_eff & 31u;
  h = (int)hh;
  const long long neg = (long long)b >> 63;          // 0 or -1
  const long long Ms = (long long)((M ^ (unsigned long long)neg) - (unsigned long long)neg);
  plo = (long long)(unsigned int)((unsigned int)(unsigned long long)Ms << lo);
  phi = Ms >> (32 - lo);
}

__device__ __forceinline__ bool is_special(unsigned long long b) {
  return ((unsigned int)(b >> 32) & 0x7FF00000u) == 0x7FF00000u;
}

// Record an infinity or NaN into three 64-bit side words (LDS or global).
__device__ __forceinline__ void note_special(unsigned long long b, unsigned long long *pos_inf,
                                             unsigned long long *neg_inf, unsigned long long *nan_bits) {
  if ((b & ((1ull << 52) - 1)) == 0) {
    if (b >> 63) atomicOr(neg_inf, 1ull); else atomicOr(pos_inf, 1ull);
  } else {
    atomicMax(nan_bits, b & 0x7FFFFFFFFFFFFFFFull);
  }
}

// ---- target formats of the final rounding --------------------------------
//
// A sum is held as X = sum c[i] 2^(32i) in units of 2^-1075 (half the
// smallest binary64 denormal).  A format with P significand bits (hidden bit
// included) whose smallest denormal is 2^U units rounds X at shift
// sh = max(bitlen(X) - P, U): q = the P bits from sh up, then round to
// nearest, ties to even, on the bits below.  The result's magnitude bits are
// ((sh - U) << (P - 1)) + q: a normal q carries its hidden bit into the
// exponent field, a denormal q (sh == U) has exponent field 0, and a rounding
// overflow (q == 2^P) moves into the exponent field by itself.  Exponent
// field EMAX means overflow to infinity (Small: rounding; Formats).
struct FmtF64 {
  static constexpr int P = 53;
  static constexpr int U = 1;
  static constexpr unsigned long long EMAX = 2047;
  static constexpr int SIGN = 63;
};
struct FmtF32 {
  static constexpr int P = 24;
  static constexpr int U = 926;      // 2^-149 = 2^926 * 2^-1075
  static constexpr unsigned long long EMAX = 255;
  static constexpr int SIGN = 31;
};

// Result bits when an infinity or NaN was seen (*has = true), else 0.  Terms
// are binary64 bit patterns (binary32 inputs are converted exactly), so
// nan_bits is the largest binary64 (bits & ~sign) over the NaN terms; for a
// binary32 result it maps back to the largest binary32 payload.
template <class F>
__device__ __forceinline__ unsigned long long special_result(unsigned long long pos_inf, unsigned long long neg_inf,
                                                             unsigned long long nan_bits, bool *has) {
  constexpr unsigned long long kInf = F::EMAX << (F::P - 1);
  constexpr unsigned long long kQuiet = 1ull << (F::P - 2);
  *has = true;
  if (nan_bits) {
    if (F::P == 53) return nan_bits | kQuiet;
    return kInf | ((nan_bits >> 29) & ((1ull << 23) - 1)) | kQuiet;
  }
  if (pos_inf && neg_inf) return kInf | kQuiet;
  if (pos_inf) return kInf;
  if (neg_inf) return (1ull << F::SIGN) | kInf;
  *has = false;
  return 0;
}

// ---- wave-parallel carry propagation and rounding -------------------------

__device__ __forceinline__ unsigned int readlane_u32(unsigned int v, int lane) {
  return (unsigned int)__builtin_amdgcn_readlane((int)v, lane);
}

// Cross-lane moves on the DPP path of the vector unit (a few cycles, where a
// general shuffle goes through the LDS crossbar).  DPP controls (GFX9):
// row_shr:k = 0x110 + k, wave_shr:1 = 0x138, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.  Lanes without a source keep `old`.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ unsigned int dpp_u32(unsigned int old, unsigned int v) {
  return (unsigned int)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}
// Lane i receives v from lane i - 1; lane 0 receives `first`.
__device__ __forceinline__ unsigned long long shr1_u64(unsigned long long v, unsigned long long first) {
  const unsigned int lo = dpp_u32<0x138>((unsigned int)first, (unsigned int)v);
  const unsigned int hi = dpp_u32<0x138>((unsigned int)(first >> 32), (unsigned int)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// One parallel carry step on the 67 chunks held as digit i = A (lane i) for
// i < 64 and digit 64 + j = B (lane j) for j < 3:  c_i <- low32(c_i) +
// (c_{i-1} >> 32); the top digit (66) keeps its high part.  Value unchanged.
__device__ __forceinline__ void carry_step_regs(long long &A, long long &B, int lane) {
  const long long hiA = A >> 32, hiB = B >> 32;
  const long long loA = A & 0xFFFFFFFFll, loB = B & 0xFFFFFFFFll;
  const long long cA = (long long)shr1_u64((unsigned long long)hiA, 0ull);
  const long long hiA63 = (long long)readlane_u64((unsigned long long)hiA, 63);
  const long long cB = (long long)shr1_u64((unsigned long long)hiB, (unsigned long long)hiA63);
  A = loA + cA;
  if (lane < 2) B = loB + cB;
  else if (lane == 2) B = B + cB;
  else B = 0;
}

// Exact carry resolution on a wavefront.  After two parallel carry steps
// every digit below the top is in [-1, 2^32], so the carry out of a digit
// is -1, 0 or +1 and depends only on the digit and its carry in: a map from
// {-1, 0, 1} to itself, packed as f(c) + 1 in bits 2(c+1) .. 2(c+1)+1.
// A digit in [1, 2^32 - 2] absorbs any carry; 0 passes a -1 on; 2^32 - 1
// passes a +1 on; -1 sends -1 unless it receives +1; 2^32 sends +1 unless
// it receives -1.  An inclusive scan of map compositions across the lanes
// (six DPP steps) gives every digit its carry in.
__device__ __forceinline__ unsigned int carry_map(long long d) {
  if (d == -1) return 0u | (0u << 2) | (1u << 4);
  if (d == 0) return 0u | (1u << 2) | (1u << 4);
  if (d == 0xFFFFFFFFll) return 1u | (1u << 2) | (2u << 4);
  if (d == 0x100000000ll) return 1u | (2u << 2) | (2u << 4);
  return 1u | (1u << 2) | (1u << 4);
}
__device__ __forceinline__ int carry_apply(unsigned int f, int c) { return (int)((f >> (2 * (c + 1))) & 3u) - 1; }
// g after f
__device__ __forceinline__ unsigned int carry_compose(unsigned int g, unsigned int f) {
  unsigned int h = 0;
#pragma unroll
  for (int k = 0; k < 3; k++) h |= ((g >> (2 * ((f >> (2 * k)) & 3u))) & 3u) << (2 * k);
  return h;
}

// The magnitude of X = sum c[i] 2^(32i) (67 int64 chunks in LDS,
// |c[i]| < 2^62) held across one wavefront: digit i in lane i (dA, i < 64),
// digit 64 + j in lane j (dB, j < 2), digit 66 in every lane (mtop, >= 0),
// every digit below the top in [0, 2^32).  Called by the whole wavefront.
struct WaveMag {
  unsigned int dA;
  unsigned int dB;
  long long mtop;
  unsigned long long mA, mB;        // ballots of the nonzero dA / dB
  unsigned long long neg;           // 1 if X < 0
  int t;                            // index of the top nonzero digit, -1 if X == 0
};

__device__ inline WaveMag wave_magnitude(const long long *c, int lane) {
  WaveMag m;
  long long A = c[lane];
  long long B = (lane < 3) ? c[64 + lane] : 0;
  carry_step_regs(A, B, lane);
  carry_step_regs(A, B, lane);
  // carries in of digits 0..63 by an inclusive scan of carry maps: within
  // each row of 16 lanes (row_shr 1, 2, 4, 8), then row 0's total into row
  // 1 and row 2's into row 3 (row_bcast:15), then rows 0-1's into rows 2-3
  // (row_bcast:31); lanes without a source compose with the identity map
  // (when no digit is -1 or 2^32, which is the common case, no digit
  // passes a carry on and the scan is skipped)
  unsigned int dA;
  long long cy;
  if (__ballot(A == -1ll || A == 0x100000000ll) == 0ull) {
    dA = (unsigned int)A;
    cy = 0;
  } else {
    constexpr unsigned int kId = 0u | (1u << 2) | (2u << 4);   // c -> c
    unsigned int F = carry_map(A);
    F = carry_compose(F, dpp_u32<0x111>(kId, F));
    F = carry_compose(F, dpp_u32<0x112>(kId, F));
    F = carry_compose(F, dpp_u32<0x114>(kId, F));
    F = carry_compose(F, dpp_u32<0x118>(kId, F));
    F = carry_compose(F, dpp_u32<0x142, 0xA>(kId, F));
    F = carry_compose(F, dpp_u32<0x143, 0xC>(kId, F));
    const unsigned int Fprev = dpp_u32<0x138>(kId, F);          // lane 0: the identity, carry in 0
    const int cin = carry_apply(Fprev, 0);
    dA = (unsigned int)(A + cin);
    cy = carry_apply((unsigned int)__builtin_amdgcn_readlane((int)F, 63), 0);
  }
  // digits 64, 65 and the top take the remaining carries in order
  const long long v64 = (long long)readlane_u64((unsigned long long)B, 0) + cy;
  cy = v64 >> 32;
  const long long v65 = (long long)readlane_u64((unsigned long long)B, 1) + cy;
  cy = v65 >> 32;
  const long long top = (long long)readlane_u64((unsigned long long)B, 2) + cy;
  unsigned int dB = (lane == 0) ? (unsigned int)v64 : (lane == 1 ? (unsigned int)v65 : 0u);
  long long mtop = top;
  m.neg = 0;
  if (top < 0) {
    // two's-complement negation: digits below the lowest nonzero one stay 0,
    // that digit becomes 2^32 - d, the digits above are complemented, and the
    // top becomes -top - 1 (or -top if every lower digit is zero)
    m.neg = 1;
    const unsigned long long nzA = __ballot(dA != 0u);
    const unsigned long long nzB = __ballot(lane < 2 && dB != 0u);
    int k;
    if (nzA) k = __ffsll((long long)nzA) - 1;
    else if (nzB) k = 64 + __ffsll((long long)nzB) - 1;
    else k = 66;
    const int iA = lane, iB = 64 + lane;
    dA = (iA < k) ? 0u : (iA == k ? 0u - dA : ~dA);
    if (lane < 2) dB = (iB < k) ? 0u : (iB == k ? 0u - dB : ~dB);
    mtop = (k == 66) ? -top : -top - 1;
  }
  m.dA = dA;
  m.dB = dB;
  m.mtop = mtop;
  m.mA = __ballot(dA != 0u);
  m.mB = __ballot(lane < 2 && dB != 0u);
  if (mtop != 0) m.t = 66;
  else if (m.mB) m.t = 64 + (63 - __clzll((long long)m.mB));
  else if (m.mA) m.t = 63 - __clzll((long long)m.mA);
  else m.t = -1;
  return m;
}

// Digit i (uniform i) of the magnitude.
__device__ __forceinline__ unsigned int wave_digit(const WaveMag &m, int i) {
  if (i < 0) return 0u;
  if (i < 64) return readlane_u32(m.dA, i);
  if (i < 66) return readlane_u32(m.dB, i - 64);
  if (i == 66) return (unsigned int)m.mtop;
  return 0u;
}

// 32 bits of the magnitude from bit position pos up (uniform pos >= 0).
__device__ __forceinline__ unsigned int wave_bits32(const WaveMag &m, int pos) {
  const int w = pos >> 5, o = pos & 31;
  const unsigned int lo = wave_digit(m, w);
  return o ? ((lo >> o) | (wave_digit(m, w + 1) << (32 - o))) : lo;
}

// Whether any bit of the magnitude below bit position pos (0 <= pos <
// 32 * 67) is set.
__device__ __forceinline__ bool wave_any_below(const WaveMag &m, int pos) {
  const int rw = pos >> 5;
  if ((wave_digit(m, rw) & ((1u << (pos & 31)) - 1u)) != 0u) return true;
  const unsigned long long belowA = (rw >= 64) ? m.mA : (rw > 0 ? (m.mA & ((1ull << rw) - 1ull)) : 0ull);
  const unsigned long long belowB = (rw > 64) ? (m.mB & ((1ull << (rw - 64)) - 1ull)) : 0ull;
  return belowA != 0ull || belowB != 0ull;
}

// Round sum c[i] 2^(32i-1075) (67 int64 chunks in LDS, |c[i]| < 2^62) to
// format F, ties to even; specials take precedence (Small: obtaining the
// correctly rounded result).  Called by one whole wavefront (all 64 lanes
// active); returns the same bits in every lane.
template <class F>
__device__ inline unsigned long long round_chunks_wave(const long long *c, unsigned long long pos_inf,
                                                       unsigned long long neg_inf, unsigned long long nan_bits,
                                                       int lane) {
  bool has;
  const unsigned long long sp = special_result<F>(pos_inf, neg_inf, nan_bits, &has);
  if (has) return sp;
  const WaveMag m = wave_magnitude(c, lane);
  if (m.t < 0) return 0;                           // exact zero -> +0.0
  const int Bl = 32 * m.t + 32 - __clz(wave_digit(m, m.t));   // bit length of X (units 2^-1075)
  int sh = Bl - F::P;
  if (sh < F::U) sh = F::U;
  unsigned long long q = (unsigned long long)wave_bits32(m, sh) | ((unsigned long long)wave_bits32(m, sh + 32) << 32);
  q &= (1ull << F::P) - 1;
  const int rpos = sh - 1;
  const unsigned int rbit = (wave_digit(m, rpos >> 5) >> (rpos & 31)) & 1u;
  const bool sticky = wave_any_below(m, rpos);
  if (rbit && (sticky || (q & 1))) q += 1;
  unsigned long long bits = ((unsigned long long)(sh - F::U) << (F::P - 1)) + q;
  if (bits == 0) return 0;                         // a nonzero sum that rounds to zero -> +0.0
  if ((bits >> (F::P - 1)) >= F::EMAX) bits = F::EMAX << (F::P - 1);
  return (m.neg << F::SIGN) | bits;
}

// The exact mean: the value sum c[i] 2^(32i-1075) divided by n >= 1,
// rounded once to binary64, ties to even (Discussion, on a correctly rounded
// mean); a mean that rounds to zero is +0.  Called by one whole wavefront.
// With A = X/2 in units of 2^-1074, Q = floor(A/n) and R = A mod n (the
// quotient is rounded on its 53 top bits, the bit below and the sticky OR
// of the rest and R), only Q's top bits matter: for j >= 0, floor(Q / 2^j) = floor(floor(A / 2^j) / n), and
// (Q mod 2^j, R) are both zero exactly when A mod (n 2^j) is, i.e. when the
// low j bits of A and floor(A / 2^j) mod n are.  j is chosen so that
// floor(A / 2^j) has at most 96 bits and its quotient at least 55, which
// leaves room for the 53 kept bits and the round bit.
__device__ inline unsigned long long round_mean_wave(const long long *c, unsigned long long pos_inf,
                                                     unsigned long long neg_inf, unsigned long long nan_bits,
                                                     unsigned long long n, int lane) {
  bool has;
  const unsigned long long sp = special_result<FmtF64>(pos_inf, neg_inf, nan_bits, &has);
  if (has) return sp;
  const WaveMag m = wave_magnitude(c, lane);
  if (m.t < 0) return 0;                           // exact zero -> +0.0
  const int bA = 32 * m.t + 31 - __clz(wave_digit(m, m.t));   // bit length of A = X / 2
  const int bn = 64 - __clzll((long long)n);
  const int j0 = (bA - bn - 55 > 0) ? bA - bn - 55 : 0;
  // A' = floor(A / 2^j0) = X >> (j0 + 1), below 2^96
  const unsigned int a0 = wave_bits32(m, j0 + 1), a1 = wave_bits32(m, j0 + 33), a2 = wave_bits32(m, j0 + 65);
  const unsigned int aw[3] = {a0, a1, a2};
  const long long nn = (long long)n;
  const double inv = 1.0 / (double)n;
  long long r = 0;
  unsigned long long T = 0;
#pragma unroll
  for (int k = 5; k >= 0; k--) {
    const long long cur = (r << 16) | (long long)((aw[k >> 1] >> (16 * (k & 1))) & 0xFFFFu);
    long long qe = (long long)((double)cur * inv);
    long long rem = cur - qe * nn;
    while (rem < 0) { qe -= 1; rem += nn; }
    while (rem >= nn) { qe += 1; rem -= nn; }
    r = rem;
    T = (T << 16) | (unsigned long long)qe;
  }
  const bool low = (j0 > 0) && wave_any_below(m, j0 + 1);   // bits of A below j0
  const int bT = T ? 64 - __clzll((long long)T) : 0;
  unsigned long long q;
  int sh;
  bool up;
  if (j0 == 0 && bT <= 53) {
    sh = 0;
    q = T;
    up = (2 * r > nn) || (2 * r == nn && (q & 1));
  } else {
    const int s2 = bT - 53;                        // >= 1
    q = T >> s2;
    const bool rb = (T >> (s2 - 1)) & 1ull;
    const bool sticky = (T & ((1ull << (s2 - 1)) - 1ull)) != 0ull || r != 0 || low;
    up = rb && (sticky || (q & 1));
    sh = j0 + s2;
  }
  if (up) q += 1;
  const unsigned long long sign = m.neg << 63;
  if (q == 0) return 0;                            // rounds to zero -> +0
  if (q < (1ull << 52)) return sign | q;           // denormal
  if (q == (1ull << 53)) {
    q = 1ull << 52;
    sh += 1;
  }
  const unsigned long long E = (unsigned long long)sh + 1;
  if (E >= 2047) return sign | 0x7FF0000000000000ull;
  return sign | (E << 52) | (q - (1ull << 52));
}

}  // namespace exsum
