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

// Merge workspace of one multi-workgroup sum.  Each workgroup writes its
// small accumulator as a row with plain stores; groups of kMergeGroup
// workgroups are summed by the group's last arrival, and the group sums by
// the last group to finish.  Only two small counters are atomic, so no
// address sees more than max(kMergeGroup, groups) atomic updates.  Row
// layout: words 0..66 chunks, 68 +Inf seen, 69 -Inf seen, 70 max NaN bits.
constexpr int kMergeGroup = 16;
constexpr int kRowWords = 72;
struct MergeRows {
  long long rows[kMaxGrid][kRowWords];
  long long grows[kMaxGrid / kMergeGroup][kRowWords];
  unsigned int gticket[kMaxGrid / kMergeGroup];
  unsigned int ticket;
  unsigned int pad[63];
};

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

// For a finite term: chunk index h = e_eff>>5, low piece (< 2^32) for chunk h
// and high piece (< 2^52) for chunk h+1, both already signed.
__device__ __forceinline__ void term_pieces(unsigned long long b, int &h, long long &plo, long long &phi) {
  const unsigned int e = (unsigned int)(b >> 52) & 2047u;
  const unsigned long long M = (b & ((1ull << 52) - 1)) | ((unsigned long long)(e != 0) << 52);
  const unsigned int e_eff = e ? e : 1u;
  const unsigned int lo = e_eff & 31u;
  h = (int)(e_eff >> 5);
  const long long low = (long long)((M << lo) & 0xFFFFFFFFull);
  const long long high = (long long)(M >> (32 - lo));
  const long long neg = (long long)b >> 63;          // branch-free conditional negate
  plo = (low ^ neg) - neg;
  phi = (high ^ neg) - neg;
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

// ---- carry propagation and rounding (one thread) ---------------------------

// Magnitude digits of sum c[i] 2^(32i) (i < 67, int64 chunks whose partial
// sums stay in range): D[0..66] in [0, 2^32), D[67..69] = 0; returns the
// sign (1 negative).  Serial, one lane; D is 70 words of scratch in LDS.
__device__ inline int magnitude_digits(const long long *c, unsigned int *D) {
  long long carry = 0;
  for (int i = 0; i < 66; i++) {
    const long long v = c[i] + carry;
    D[i] = (unsigned int)v;
    carry = v >> 32;
  }
  long long top = c[66] + carry;                      // |top| < 2^31 for any real input
  D[66] = (unsigned int)top;
  D[67] = D[68] = D[69] = 0;
  if (top >= 0) return 0;
  unsigned long long cy = 1;                          // magnitude by two's-complement negation
  for (int i = 0; i < 67; i++) {
    const unsigned long long t = (unsigned long long)(unsigned int)~D[i] + cy;
    D[i] = (unsigned int)t;
    cy = t >> 32;
  }
  return 1;
}

// Round the value sum c[i] 2^(32i-1075) to format F, round to nearest, ties
// to even (Small: obtaining the correctly rounded result); specials take
// precedence; an exact zero gives +0.  Serial code, run by a single lane.
template <class F>
__device__ inline unsigned long long round_chunks(const long long *c, unsigned long long pos_inf,
                                                  unsigned long long neg_inf, unsigned long long nan_bits,
                                                  unsigned int *D) {
  bool has;
  const unsigned long long sp = special_result<F>(pos_inf, neg_inf, nan_bits, &has);
  if (has) return sp;
  const unsigned long long sign = (unsigned long long)magnitude_digits(c, D) << F::SIGN;
  int t = 66;
  while (t >= 0 && D[t] == 0) t--;
  if (t < 0) return 0;                                // exact zero -> +0.0
  const int Bl = 32 * t + 32 - __builtin_clz(D[t]);  // bit length of X
  int sh = Bl - F::P;
  if (sh < F::U) sh = F::U;
  const int w = sh >> 5, o = sh & 31;
  unsigned long long q = ((unsigned long long)D[w] | ((unsigned long long)D[w + 1] << 32)) >> o;
  if (o) q |= (unsigned long long)D[w + 2] << (64 - o);
  q &= (1ull << F::P) - 1;
  const int rpos = sh - 1;                            // round bit position (>= 0)
  const unsigned int rbit = (D[rpos >> 5] >> (rpos & 31)) & 1u;
  unsigned int sticky = D[rpos >> 5] & ((1u << (rpos & 31)) - 1u);
  for (int i = 0; i < (rpos >> 5); i++) sticky |= D[i];
  if (rbit && (sticky || (q & 1))) q += 1;
  unsigned long long bits = ((unsigned long long)(sh - F::U) << (F::P - 1)) + q;
  if ((bits >> (F::P - 1)) >= F::EMAX) bits = F::EMAX << (F::P - 1);
  return sign | bits;
}

// The exact mean: the value sum c[i] 2^(32i-1075) divided by n >= 1, rounded
// once to binary64 (Discussion, on a correctly rounded mean).  With A the
// magnitude in units of 2^-1074 (X/2; X is even), Q = floor(A/n) and
// R = A mod n: a quotient below 2^53 rounds on R alone, a longer one on its
// bit below the 53 kept and the sticky OR of the bits further down and R.
// A mean that rounds to zero is +0.  Serial, one lane; D is 70 words of LDS.
__device__ inline unsigned long long round_mean_f64(const long long *c, unsigned long long pos_inf,
                                                    unsigned long long neg_inf, unsigned long long nan_bits,
                                                    unsigned int *D, unsigned long long n) {
  bool has;
  const unsigned long long sp = special_result<FmtF64>(pos_inf, neg_inf, nan_bits, &has);
  if (has) return sp;
  const unsigned long long sign = (unsigned long long)magnitude_digits(c, D) << 63;
  // A = X / 2, then Q = A / n in place, 16 bits at a time: each partial
  // dividend is below n * 2^16 <= 2^56, its quotient (below 2^16) is first
  // estimated with a binary64 multiply by 1/n and then made exact with
  // integer corrections of the remainder (the estimate is off by a few
  // units at most)
  for (int i = 0; i < 67; i++) D[i] = (D[i] >> 1) | (D[i + 1] << 31);
  const long long nn = (long long)n;
  const double inv = 1.0 / (double)n;
  unsigned long long r = 0;
  for (int i = 66; i >= 0; i--) {
    const unsigned int d = D[i];
    long long cur = (long long)((r << 16) | (d >> 16));
    long long qe = (long long)((double)cur * inv);
    long long rem = cur - qe * nn;
    while (rem < 0) { qe -= 1; rem += nn; }
    while (rem >= nn) { qe += 1; rem -= nn; }
    const unsigned long long qh = (unsigned long long)qe;
    cur = (rem << 16) | (long long)(d & 0xFFFFu);
    qe = (long long)((double)cur * inv);
    rem = cur - qe * nn;
    while (rem < 0) { qe -= 1; rem += nn; }
    while (rem >= nn) { qe += 1; rem -= nn; }
    r = (unsigned long long)rem;
    D[i] = (unsigned int)((qh << 16) | (unsigned long long)qe);
  }
  int t = 66;
  while (t >= 0 && D[t] == 0) t--;
  const int b = (t < 0) ? 0 : 32 * t + 32 - __builtin_clz(D[t]);
  unsigned long long q;
  int sh;
  bool up;
  if (b <= 53) {
    sh = 0;
    q = (unsigned long long)D[0] | ((unsigned long long)D[1] << 32);
    up = (2 * r > n) || (2 * r == n && (q & 1));
  } else {
    sh = b - 53;
    const int w = sh >> 5, o = sh & 31;
    q = ((unsigned long long)D[w] | ((unsigned long long)D[w + 1] << 32)) >> o;
    if (o) q |= (unsigned long long)D[w + 2] << (64 - o);
    q &= (1ull << 53) - 1;
    const int rpos = sh - 1;
    const unsigned int rbit = (D[rpos >> 5] >> (rpos & 31)) & 1u;
    unsigned int sticky = D[rpos >> 5] & ((1u << (rpos & 31)) - 1u);
    for (int i = 0; i < (rpos >> 5); i++) sticky |= D[i];
    up = rbit && (sticky || r != 0 || (q & 1));
  }
  if (up) q += 1;
  if (q == 0) return 0;                               // rounds to zero -> +0
  if (q < (1ull << 52)) return sign | q;              // denormal
  if (q == (1ull << 53)) {
    q = 1ull << 52;
    sh += 1;
  }
  const unsigned long long E = (unsigned long long)sh + 1;
  if (E >= 2047) return sign | 0x7FF0000000000000ull;
  return sign | (E << 52) | (q - (1ull << 52));
}

// ---- wave-parallel carry propagation and rounding -------------------------

__device__ __forceinline__ unsigned int readlane_u32(unsigned int v, int lane) {
  return (unsigned int)__builtin_amdgcn_readlane((int)v, lane);
}

// One parallel carry step on the 67 chunks held as digit i = A (lane i) for
// i < 64 and digit 64 + j = B (lane j) for j < 3:  c_i <- low32(c_i) +
// (c_{i-1} >> 32); the top digit (66) keeps its high part.  Value unchanged.
__device__ __forceinline__ void carry_step_regs(long long &A, long long &B, int lane) {
  const long long hiA = A >> 32, hiB = B >> 32;
  const long long loA = A & 0xFFFFFFFFll, loB = B & 0xFFFFFFFFll;
  long long cA = (long long)__shfl_up((unsigned long long)hiA, 1, 64);
  if (lane == 0) cA = 0;
  const long long hiA63 = (long long)readlane_u64((unsigned long long)hiA, 63);
  long long cB = (long long)__shfl_up((unsigned long long)hiB, 1, 64);
  if (lane == 0) cB = hiA63;
  A = loA + cA;
  if (lane < 2) B = loB + cB;
  else if (lane == 2) B = B + cB;
  else B = 0;
}

// Round sum c[i] 2^(32i-1075) (67 int64 chunks in LDS, |c[i]| < 2^62) to
// format F, ties to even; specials take precedence.  Called by one whole
// wavefront (all 64 lanes active); returns the same bits in every lane.  Two
// parallel carry steps leave every digit below the top in [-1, 2^32]; in
// the rare case that a digit sits exactly on a bound the serial routine
// finishes the job (lane 0, D = 70 words of scratch).
template <class F>
__device__ inline unsigned long long round_chunks_wave(const long long *c, unsigned long long pos_inf,
                                                       unsigned long long neg_inf, unsigned long long nan_bits,
                                                       unsigned int *D, int lane) {
  bool has;
  const unsigned long long sp = special_result<F>(pos_inf, neg_inf, nan_bits, &has);
  if (has) return sp;
  long long A = c[lane];
  long long B = (lane < 3) ? c[64 + lane] : 0;
  carry_step_regs(A, B, lane);
  carry_step_regs(A, B, lane);
  // digits 0..65 now in [-1, 2^32]; a digit on either bound would need a
  // longer carry chain
  const bool edgeA = (A < 0) || (A > 0xFFFFFFFFll);
  const bool edgeB = (lane < 2) && ((B < 0) || (B > 0xFFFFFFFFll));
  if (__ballot(edgeA || edgeB) != 0ull) {
    unsigned long long r = 0;
    if (lane == 0) r = round_chunks<F>(c, 0ull, 0ull, 0ull, D);
    return readlane_u64(r, 0);
  }
  const long long top = (long long)readlane_u64((unsigned long long)B, 2);
  unsigned int dA = (unsigned int)A;            // digits 0..63
  unsigned int dB = (lane < 2) ? (unsigned int)B : 0u;  // digits 64, 65
  long long mtop = top;
  unsigned long long sign = 0;
  if (top < 0) {
    // two's-complement negation: digits below the lowest nonzero one stay 0,
    // that digit becomes 2^32 - d, the digits above are complemented, and the
    // top becomes -top - 1 (or -top if every lower digit is zero)
    sign = 1ull << F::SIGN;
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
  // magnitude digits: dA (0..63), dB (64, 65), mtop (66, small, >= 0)
  const unsigned long long mA = __ballot(dA != 0u);
  const unsigned long long mB = __ballot(lane < 2 && dB != 0u);
  int t;
  if (mtop != 0) t = 66;
  else if (mB) t = 64 + (63 - __clzll((long long)mB));
  else if (mA) t = 63 - __clzll((long long)mA);
  else return 0;                                   // exact zero -> +0.0
  auto digit = [&](int i) -> unsigned int {
    if (i < 0) return 0u;
    if (i < 64) return readlane_u32(dA, i);
    if (i < 66) return readlane_u32(dB, i - 64);
    if (i == 66) return (unsigned int)mtop;
    return 0u;
  };
  const unsigned int Dt = digit(t);
  const int Bl = 32 * t + 32 - __clz(Dt);          // bit length of X (units 2^-1075)
  int sh = Bl - F::P;
  if (sh < F::U) sh = F::U;
  const int w = sh >> 5, o = sh & 31;
  unsigned long long q = ((unsigned long long)digit(w) | ((unsigned long long)digit(w + 1) << 32)) >> o;
  if (o) q |= (unsigned long long)digit(w + 2) << (64 - o);
  q &= (1ull << F::P) - 1;
  const int rpos = sh - 1;
  const int rw = rpos >> 5;
  const unsigned int rd = digit(rw);
  const unsigned int rbit = (rd >> (rpos & 31)) & 1u;
  bool sticky = (rd & ((1u << (rpos & 31)) - 1u)) != 0u;
  // any nonzero digit strictly below rw
  const unsigned long long belowA = (rw >= 64) ? mA : (rw > 0 ? (mA & ((1ull << rw) - 1ull)) : 0ull);
  const unsigned long long belowB = (rw > 64) ? (mB & ((1ull << (rw - 64)) - 1ull)) : 0ull;
  sticky = sticky || belowA || belowB;
  if (rbit && (sticky || (q & 1))) q += 1;
  unsigned long long bits = ((unsigned long long)(sh - F::U) << (F::P - 1)) + q;
  if ((bits >> (F::P - 1)) >= F::EMAX) bits = F::EMAX << (F::P - 1);
  return sign | bits;
}

}  // namespace exsum
