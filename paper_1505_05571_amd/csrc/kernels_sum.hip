// kernels_sum.hip -- one exact sum per launch: the large-accumulator kernel,
// its narrow form for binary32 inputs, the small-only kernel, the streaming
// accumulator's kernels and the inexact comparator (gfx950, wave64).
//
// Large kernel: workgroup b owns terms [n*b/G, n*(b+1)/G) and a private large
// superaccumulator in LDS; it transfers every used chunk into its small
// superaccumulator, adds that into one shared accumulator with 64-bit device
// atomics, and the workgroup that completes the grid applies the finisher
// once (Discussion: split the array, sum the parts exactly, add the small
// superaccumulators, round the total).  One workgroup per compute unit is the
// intended grid: each holds the whole LDS budget it needs and is never
// starved by a younger workgroup on the same unit.
#include <mutex>

#include "exsum_blocks.h"
#include "exsum_internal.h"

namespace exsum {
namespace {

template <int BLOCK, int VEC, int DEPTH, int MODE, class Src, class Fin>
__global__ __launch_bounds__(BLOCK) void large_kernel(Src src, long long n, GlobalAcc *__restrict__ M, Fin fin,
                                                      int precombine) {
  __shared__ LargeShared S;
  const int tid = threadIdx.x;
  large_init(S, tid, BLOCK);
  __syncthreads();
  const long long G = gridDim.x;
  const long long r0 = n * (long long)blockIdx.x / G;
  const long long r1 = n * (long long)(blockIdx.x + 1) / G;
  unsigned int tile = 0;
  accumulate_range<BLOCK, VEC, DEPTH, MODE>(S, src, r0, r1, precombine, tile);
  final_flush<BLOCK, false, MODE>(S);
  merge_grid_and_finish(S.small, S.spec, &S.ticket, M, fin);
}

// Narrow kernel (binary32 sums and dot products): the same grid and merge
// as the large kernel, with a narrow large accumulator (KC interleaved
// copies) in LDS.
template <int BLOCK, int VEC, int DEPTH, int KC, class T, class Fin>
__global__ __launch_bounds__(BLOCK) void narrow_kernel(T src, long long n, GlobalAcc *__restrict__ M, Fin fin) {
  __shared__ NarrowShared<T::kKeys, KC> S;
  const int tid = threadIdx.x;
  narrow_init(S, tid, BLOCK);
  __syncthreads();
  const long long G = gridDim.x;
  const long long r0 = n * (long long)blockIdx.x / G;
  const long long r1 = n * (long long)(blockIdx.x + 1) / G;
  narrow_accumulate_range<BLOCK, VEC, DEPTH, KC>(S, src, r0, r1);
  narrow_final_flush<BLOCK, KC, T>(S);
  merge_grid_and_finish(S.small, S.spec, &S.ticket, M, fin);
}

// Small-only kernel: every wavefront sums a contiguous part into its own
// small superaccumulator; the workgroup adds its wavefronts' accumulators
// (each below 2^33 per chunk after the final carry step) and merges.
template <int BLOCK, class Src, class Fin>
__global__ __launch_bounds__(BLOCK) void small_kernel(Src src, long long n, GlobalAcc *__restrict__ M, Fin fin) {
  constexpr int NW = BLOCK / 64;
  __shared__ long long s_acc[NW][small_acc_words<1>()];
  __shared__ long long s_tot[68];
  __shared__ unsigned long long s_spec[3];
  __shared__ unsigned int s_flag[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < NW * small_acc_words<1>(); i += BLOCK) (&s_acc[0][0])[i] = 0;
  if (tid < 3) s_spec[tid] = 0ull;
  __syncthreads();
  const long long G = gridDim.x;
  const long long r0 = n * (long long)blockIdx.x / G, r1 = n * (long long)(blockIdx.x + 1) / G;
  const long long len = r1 - r0;
  const long long w0 = r0 + len * wave / NW, w1 = r0 + len * (wave + 1) / NW;
  small_wave_accumulate<1>(s_acc[wave], s_spec, src, w0, w1, lane);
  __syncthreads();
  if (tid < 68) {
    long long t = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) t += s_acc[w][tid];
    s_tot[tid] = t;
  }
  merge_grid_and_finish(s_tot, s_spec, s_flag, M, fin);
}

// The streaming accumulator's own kernels (one wavefront each).
// Short sums (n <= kTinyMax) on one wavefront: no workgroup barrier, no
// cross-wave sum and no merge, and the first batch of loads is in flight
// while the accumulator is cleared.  A short sum is all fixed cost (Small:
// the small superaccumulator's per-call overhead), so the kernel keeps only
// what one wave needs: the small-superaccumulator body with 8 interleaved
// copies, then the finisher.
constexpr long long kTinyMax = 4096;
constexpr int kTinyCopies = 8;
template <class Src, class Fin>
__global__ __launch_bounds__(64) void tiny_kernel(Src src, long long n, Fin fin) {
  __shared__ long long acc[small_acc_words<kTinyCopies>()];
  __shared__ unsigned long long spec[4];
  const int lane = threadIdx.x;
  // `direct`: below 1024 terms the copies' sum stays below 2^62 without
  // carry steps, which the rounding accepts; the streaming finisher adds
  // the total to a state and carries it itself
  small_wave_accumulate<kTinyCopies, Src, true>(acc, spec, src, 0, n, lane, true);
  __builtin_amdgcn_wave_barrier();
  fin(acc, spec);
}

__global__ __launch_bounds__(64) void acc_zero_kernel(GlobalAcc *acc) {
  unsigned long long *w = reinterpret_cast<unsigned long long *>(acc);
  for (int i = threadIdx.x; i < (int)(sizeof(GlobalAcc) / 8); i += 64) w[i] = 0ull;
}

__global__ __launch_bounds__(64) void acc_merge_kernel(GlobalAcc *dst, const GlobalAcc *src) {
  __shared__ long long c[68];
  const int lane = threadIdx.x;
  c[lane] = (long long)(dst->chunk[lane] + src->chunk[lane]);
  if (lane < 4) c[64 + lane] = (long long)(dst->chunk[64 + lane] + src->chunk[64 + lane]);
  __builtin_amdgcn_wave_barrier();
  carry_step(c, lane);
  dst->chunk[lane] = (unsigned long long)c[lane];
  if (lane < 4) dst->chunk[64 + lane] = (unsigned long long)c[64 + lane];
  if (lane == 0) {
    dst->pos_inf |= src->pos_inf;
    dst->neg_inf |= src->neg_inf;
    if (src->nan_bits > dst->nan_bits) dst->nan_bits = src->nan_bits;
  }
}

__global__ __launch_bounds__(64) void acc_round_kernel(const GlobalAcc *acc, double *out) {
  __shared__ long long c[68];
  const int lane = threadIdx.x;
  c[lane] = (long long)acc->chunk[lane];
  if (lane < 4) c[64 + lane] = (long long)acc->chunk[64 + lane];
  __builtin_amdgcn_wave_barrier();
  const unsigned long long r =
      round_chunks_wave<FmtF64>(c, acc->pos_inf, acc->neg_inf, acc->nan_bits, lane);
  if (lane == 0) out[0] = __longlong_as_double((long long)r);
}

// Inexact comparator: ordinary binary64 additions on the exact kernel's load
// path (one workgroup per compute unit, per-wave contiguous streams, 16-byte
// non-temporal loads, DEPTH tiles in flight, past-the-end prefetches on the
// pad tile), 2*VEC independent accumulators per lane, then wave, block and a
// fixed-order tree over the per-workgroup partials in the last workgroup.
template <int BLOCK, int VEC, int DEPTH>
__global__ __launch_bounds__(BLOCK) void inexact_kernel(const double *__restrict__ x, long long n,
                                                        double *__restrict__ partials,
                                                        unsigned int *__restrict__ ticket,
                                                        double *__restrict__ out) {
  constexpr int NW = BLOCK / 64;
  constexpr int TILE_W = 64 * VEC;
  static_assert(VEC <= kMaxVec, "pad tile too small");
  __shared__ double s_red[BLOCK / 64];
  __shared__ unsigned int s_ticket;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long G = gridDim.x;
  const long long r0 = n * (long long)blockIdx.x / G, r1 = n * (long long)(blockIdx.x + 1) / G;
  double a[2 * VEC];
#pragma unroll
  for (int j = 0; j < 2 * VEC; j++) a[j] = 0.0;
  if (r1 > r0) {
    const long long head = (reinterpret_cast<uintptr_t>(x + r0) & 15) ? 1 : 0;
    const long long s0 = r0 + head;
    const long long nv = (r1 - s0) >> 1;
    if (tid == 0 && head) a[0] += x[r0];
    if (tid == 1 && s0 < r1 && ((r1 - s0) & 1)) a[1] += x[r1 - 1];
    const ulonglong2 *__restrict__ xv = reinterpret_cast<const ulonglong2 *>(x + s0);
    const long long q = nv / NW;
    const long long ws = (long long)wave * q;
    const long long we = (wave == NW - 1) ? nv : ws + q;
    const long long ntiles = q / TILE_W;
    ulonglong2 buf[DEPTH][VEC];
    auto load = [&](ulonglong2(&bf)[VEC], long long t) {
      const ulonglong2 *tp = (t < ntiles) ? xv + ws + t * TILE_W : g_pad_tile;
#pragma unroll
      for (int j = 0; j < VEC; j++) bf[j] = stream_load(tp + lane + j * 64);
      __builtin_amdgcn_sched_barrier(0);
    };
    auto process = [&](const ulonglong2(&bf)[VEC]) {
#pragma unroll
      for (int j = 0; j < VEC; j++) {
        a[2 * j] += __longlong_as_double((long long)bf[j].x);
        a[2 * j + 1] += __longlong_as_double((long long)bf[j].y);
      }
    };
    if (ntiles > 0) {
#pragma unroll
      for (int d = 0; d < DEPTH; d++) load(buf[d], d);
      for (long long t = 0; t < ntiles; t += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; d++) {
          if (d == 0 || t + d < ntiles) process(buf[d]);
          load(buf[d], t + d + DEPTH);
        }
      }
    }
    for (long long p = ws + ntiles * TILE_W + lane; p < we; p += 64) {
      const ulonglong2 v = xv[p];
      a[0] += __longlong_as_double((long long)v.x);
      a[1] += __longlong_as_double((long long)v.y);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < 2 * VEC; j++) s += a[j];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane == 0) s_red[wave] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < BLOCK / 64; w++) t += s_red[w];
    // a device-scope store, completed before the ticket (as in the exact
    // merge): no device-wide cache flush
    __hip_atomic_store((unsigned long long *)&partials[blockIdx.x], (unsigned long long)__double_as_longlong(t),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wait_memory();
    s_ticket = ticket_add(ticket);
  }
  __syncthreads();
  if (s_ticket != gridDim.x - 1) return;
  double t = 0.0;
  for (long long i = tid; i < G; i += BLOCK) {
    t += __longlong_as_double((long long)__hip_atomic_load((unsigned long long *)&partials[i], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT));
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
  __syncthreads();
  if (lane == 0) s_red[wave] = t;
  __syncthreads();
  if (tid == 0) {
    double r = 0.0;
    for (int w = 0; w < BLOCK / 64; w++) r += s_red[w];
    out[0] = r;
    atomicExch(ticket, 0u);
  }
}

}  // namespace

constexpr int kOpBlock = 1024;
constexpr int kInexactBlock = 1024;

// Built variants (block, vec, depth, mode).  Count mode needs
// 2*block*vec < 4096 (the count bound per tile); carry mode does not.
#define EXSUM_LARGE_VARIANTS(X) \
  X(256, 6, 3, kCountMode)      \
  X(256, 4, 3, kCountMode)      \
  X(256, 2, 4, kCountMode)      \
  X(512, 3, 2, kCountMode)      \
  X(512, 2, 2, kCountMode)      \
  X(256, 4, 3, kCarryMode)      \
  X(512, 4, 2, kCarryMode)      \
  X(512, 2, 4, kCarryMode)      \
  X(1024, 2, 2, kCarryMode)     \
  X(1024, 4, 2, kCarryMode)

hipError_t launch_large(const double *x, int64_t n, GlobalAcc *M, double *out, hipStream_t s, int block,
                        int vec, int depth, int mode, int grid, int precombine) {
  if (grid < 1) grid = 1;
#define EXSUM_LAUNCH(B, V, D, MD)                                                                             \
  if (block == B && vec == V && depth == D && mode == MD) {                                                   \
    hipLaunchKernelGGL((large_kernel<B, V, D, MD, SrcF64, FinF64>), dim3(grid), dim3(B), 0, s, SrcF64{x},     \
                       (long long)n, M, FinF64{out}, precombine);                                             \
    return hipGetLastError();                                                                                 \
  }
  EXSUM_LARGE_VARIANTS(EXSUM_LAUNCH)
#undef EXSUM_LAUNCH
  return hipErrorInvalidValue;
}

bool large_variant_exists(int block, int vec, int depth, int mode) {
#define EXSUM_EXISTS(B, V, D, MD) \
  if (block == B && vec == V && depth == D && mode == MD) return true;
  EXSUM_LARGE_VARIANTS(EXSUM_EXISTS)
#undef EXSUM_EXISTS
  return false;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free single sum: the one merge accumulator that
// the small and large kernels of exsum_f64 need (67 chunks, side words and
// ticket, 576 bytes), in static device memory, one copy per device, held
// until the process ends.  The kernels leave it zeroed when a call
// completes, as they leave a stream's workspace; it is also cleared once per
// device at set-up.  Host code never passes `scratch` itself to a kernel:
// its device address comes from hipGetSymbolAddress, per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) GlobalAcc scratch[1];

namespace {
std::mutex g_scratch_mu;
GlobalAcc *g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

hipError_t noalloc_scratch(int dev, hipStream_t s, GlobalAcc **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    // the calling thread's current device is `dev`
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    // clear it with a fill kernel on the caller's stream (no memset node, so
    // a first call under graph capture records only kernels)
    hipLaunchKernelGGL(acc_zero_kernel, dim3(1), dim3(64), 0, s, static_cast<GlobalAcc *>(p));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<GlobalAcc *>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int large_variants(int32_t *out, int64_t cap) {
  int k = 0;
#define EXSUM_LIST(B, V, D, MD)  \
  if (out && k < cap) {          \
    out[4 * k + 0] = B;          \
    out[4 * k + 1] = V;          \
    out[4 * k + 2] = D;          \
    out[4 * k + 3] = MD;         \
  }                              \
  k++;
  EXSUM_LARGE_VARIANTS(EXSUM_LIST)
#undef EXSUM_LIST
  return k;
}

// The small-only kernel, or for a short sum on one workgroup the one-wave
// kernel.
template <class Src, class Fin>
hipError_t launch_small_any(const Src &src, int64_t n, const Fin &fin, GlobalAcc *M, hipStream_t s, int grid) {
  if (grid < 1) grid = 1;
  if (grid == 1 && n <= kTinyMax)
    hipLaunchKernelGGL((tiny_kernel<Src, Fin>), dim3(1), dim3(64), 0, s, src, (long long)n, fin);
  else
    hipLaunchKernelGGL((small_kernel<256, Src, Fin>), dim3(grid), dim3(256), 0, s, src, (long long)n, M, fin);
  return hipGetLastError();
}

hipError_t launch_small(const double *x, int64_t n, GlobalAcc *M, double *out, hipStream_t s, int grid) {
  return launch_small_any(SrcF64{x}, n, FinF64{out}, M, s, grid);
}

// Other sources and finishers: the small kernel, or the large kernel in its
// default variant (1024 threads, 4 positions per thread per tile, 2 tiles in
// flight, carry-triggered transfers).
namespace {
template <int BLOCK, int VEC, class Src, class Fin>
hipError_t launch_op(const Src &src, int64_t n, const Fin &fin, GlobalAcc *M, hipStream_t s, int grid, bool small,
                     int precombine) {
  if (grid < 1) grid = 1;
  if (small)
    return launch_small_any(src, n, fin, M, s, grid);
  else
    hipLaunchKernelGGL((large_kernel<BLOCK, VEC, 2, kCarryMode, Src, Fin>), dim3(grid), dim3(BLOCK), 0, s, src,
                       (long long)n, M, fin, precombine);
  return hipGetLastError();
}
// Sources with more registers per position use shapes that fit their
// registers without spilling (measured best of 512x4 and 1024x2 for each).
constexpr int kDotBlock = 512, kDotVec = 4;      // two inputs per position
}  // namespace

hipError_t launch_sqnorm(const double *x, int64_t n, double *out, GlobalAcc *M, hipStream_t s, int grid, bool small,
                         int precombine) {
  return launch_op<kOpBlock, 4>(SrcSq{{x}}, n, FinF64{out}, M, s, grid, small, precombine);
}

hipError_t launch_dot(const double *x, const double *y, int64_t n, double *out, GlobalAcc *M, hipStream_t s,
                      int grid, bool small, int precombine) {
  if (((reinterpret_cast<uintptr_t>(x) ^ reinterpret_cast<uintptr_t>(y)) & 15) == 0)
    return launch_op<kDotBlock, kDotVec>(SrcDot<true>{x, y}, n, FinF64{out}, M, s, grid, small, precombine);
  return launch_op<kDotBlock, kDotVec>(SrcDot<false>{x, y}, n, FinF64{out}, M, s, grid, small, precombine);
}

hipError_t launch_mean(const double *x, int64_t n, double *out, GlobalAcc *M, hipStream_t s, int grid, bool small,
                       int precombine) {
  return launch_op<kOpBlock, 4>(SrcF64{x}, n, FinMean{out, (unsigned long long)n}, M, s, grid, small, precombine);
}

// binary32 sums and dot products on the large path take the narrow kernel
// (no pre-combine: its interleaved copies serve a hot chunk better); its
// chunks cannot wrap while a workgroup's range holds fewer than 2^40 terms,
// which any n below 2^40 (the entry points' bound) guarantees.
constexpr int kNarrowBlock = 1024, kNarrowVec = 4, kNarrowDepth = 2, kNarrowCopies = 8;
constexpr int kNarrowDotVec = 2;

template <class T>
hipError_t launch_narrow(const T &src, int64_t n, float *out, GlobalAcc *M, hipStream_t s, int grid) {
  if (n >= kNarrowMaxTerms) return hipErrorInvalidValue;
  constexpr int VEC = sizeof(typename T::Vec) > 16 ? kNarrowDotVec : kNarrowVec;
  hipLaunchKernelGGL((narrow_kernel<kNarrowBlock, VEC, kNarrowDepth, kNarrowCopies, T, FinF32>), dim3(grid),
                     dim3(kNarrowBlock), 0, s, src, (long long)n, M, FinF32{out});
  return hipGetLastError();
}

hipError_t launch_f32(const float *x, int64_t n, float *out, GlobalAcc *M, hipStream_t s, int grid, bool small,
                      int) {
  if (grid < 1) grid = 1;
  if (small) return launch_small_any(SrcF32{x}, n, FinF32{out}, M, s, grid);
  return launch_narrow(NarrowSumF32{x}, n, out, M, s, grid);
}

hipError_t launch_dot_f32(const float *x, const float *y, int64_t n, float *out, GlobalAcc *M, hipStream_t s,
                          int grid, bool small, int) {
  if (grid < 1) grid = 1;
  if (small) return launch_small_any(SrcDotF32{x, y}, n, FinF32{out}, M, s, grid);
  if (((reinterpret_cast<uintptr_t>(x) ^ reinterpret_cast<uintptr_t>(y)) & 15) == 0)
    return launch_narrow(NarrowDotF32<true>{x, y}, n, out, M, s, grid);
  return launch_narrow(NarrowDotF32<false>{x, y}, n, out, M, s, grid);
}

hipError_t launch_acc_add(const double *x, int64_t n, GlobalAcc *acc, GlobalAcc *M, hipStream_t s, int grid,
                          bool small, int precombine) {
  return launch_op<kOpBlock, 4>(SrcF64{x}, n, FinAcc{acc}, M, s, grid, small, precombine);
}

hipError_t launch_acc_zero(GlobalAcc *acc, hipStream_t s) {
  hipLaunchKernelGGL(acc_zero_kernel, dim3(1), dim3(64), 0, s, acc);
  return hipGetLastError();
}

hipError_t launch_acc_merge(GlobalAcc *dst, const GlobalAcc *src, hipStream_t s) {
  hipLaunchKernelGGL(acc_merge_kernel, dim3(1), dim3(64), 0, s, dst, src);
  return hipGetLastError();
}

hipError_t launch_acc_round(const GlobalAcc *acc, double *out, hipStream_t s) {
  hipLaunchKernelGGL(acc_round_kernel, dim3(1), dim3(64), 0, s, acc, out);
  return hipGetLastError();
}

int op_block() { return kOpBlock; }

int inexact_block() { return kInexactBlock; }

hipError_t launch_inexact(const double *x, int64_t n, double *partials, unsigned int *ticket, double *out,
                          hipStream_t s, int grid) {
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((inexact_kernel<kInexactBlock, 4, 2>), dim3(grid), dim3(kInexactBlock), 0, s, x, (long long)n,
                     partials, ticket, out);
  return hipGetLastError();
}

}  // namespace exsum
