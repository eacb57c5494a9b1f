// exsum_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exsum {

constexpr int kMaxGrid = 8192;       // most workgroups one single-sum launch may use
constexpr int kMaxDevices = 64;      // devices the per-device tables hold

struct GlobalAcc;

// Per-(device, stream) workspace.  Everything the kernels write here is left
// zeroed when a call completes.
struct Workspace {
  GlobalAcc *acc = nullptr;            // merge accumulator of the one-sum kernels
  double *partials = nullptr;          // per-workgroup partials of the inexact sum
  unsigned int *ticket = nullptr;      // ticket of the inexact sum
  int max_grid = 0;                    // capacity of `partials`
  // segmented calls: one accumulator per workgroup boundary (kMaxGrid), then
  // the short-segment partition's chunk weights (kMaxGrid words)
  GlobalAcc *seg_accs = nullptr;
  long long *seg_chunks = nullptr;
  void *seg_ctl = nullptr;             // the persistent launch's cursor (seg_ctl_bytes())
};

// Host helpers (api.cpp): EXSUM_* status of a HIP error (clearing the HIP
// error state), and the compute-unit count of a device (cached).
int status_of(hipError_t e);
int cu_count(int dev);

// Launchers (kernels_sum.hip).  Return a hipError_t.
hipError_t launch_large(const double *x, int64_t n, GlobalAcc *M, double *out, hipStream_t s,
                        int block, int vec, int depth, int mode, int grid, int precombine);
bool large_variant_exists(int block, int vec, int depth, int mode);
// The built (block, vec, depth, mode) variants, 4 ints each, up to cap of
// them into out (may be NULL); returns how many are built.
int large_variants(int32_t *out, int64_t cap);
hipError_t launch_small(const double *x, int64_t n, GlobalAcc *M, double *out, hipStream_t s,
                        int grid);
// The allocation-free single sum's scratch accumulator on device `dev` (the
// current device): its device address, found and cleared (on stream s) on
// the first call for that device.
hipError_t noalloc_scratch(int dev, hipStream_t s, GlobalAcc **out);
int inexact_block();
hipError_t launch_inexact(const double *x, int64_t n, double *partials, unsigned int *ticket,
                          double *out, hipStream_t s, int grid);

// Further sums over the same path (kernels_sum.hip): the small-only kernel
// when `small`, else the large kernel in its default variant (op_block()
// threads, 4 positions per thread per tile).
hipError_t launch_sqnorm(const double *x, int64_t n, double *out, GlobalAcc *M, hipStream_t s, int grid,
                         bool small, int precombine);
hipError_t launch_dot(const double *x, const double *y, int64_t n, double *out, GlobalAcc *M, hipStream_t s,
                      int grid, bool small, int precombine);
hipError_t launch_mean(const double *x, int64_t n, double *out, GlobalAcc *M, hipStream_t s, int grid, bool small,
                       int precombine);
hipError_t launch_f32(const float *x, int64_t n, float *out, GlobalAcc *M, hipStream_t s, int grid, bool small,
                      int precombine);
hipError_t launch_dot_f32(const float *x, const float *y, int64_t n, float *out, GlobalAcc *M, hipStream_t s,
                          int grid, bool small, int precombine);
hipError_t launch_acc_add(const double *x, int64_t n, GlobalAcc *acc, GlobalAcc *M, hipStream_t s, int grid,
                          bool small, int precombine);
hipError_t launch_acc_zero(GlobalAcc *acc, hipStream_t s);
hipError_t launch_acc_merge(GlobalAcc *dst, const GlobalAcc *src, hipStream_t s);
hipError_t launch_acc_round(const GlobalAcc *acc, double *out, hipStream_t s);
int op_block();

// Segmented sums (kernels_seg.hip).
size_t global_acc_bytes();
// Two launches: long segments (more than small_max terms) by `grid`
// workgroups, then short ones by `short_grid` workgroups of
// seg_short_block() threads.  chunks: short_grid words of scratch.
hipError_t launch_segmented(const double *x, const int64_t *offsets, int64_t nseg, double *out,
                            GlobalAcc *accs, long long *chunks, hipStream_t s, int grid, int short_grid,
                            int64_t small_max, int precombine);
// One persistent launch (block = 256, 512 or 1024 threads, `grid`
// workgroups): long segments by term range with the large accumulator, then
// short ones claimed by waves in units of `group` (1..64) segments from the
// cursor in `ctl` (seg_ctl_bytes() of zeroed workspace, left zeroed).
hipError_t launch_segmented_persistent(const double *x, const int64_t *offsets, int64_t nseg, double *out,
                                       GlobalAcc *accs, void *ctl, hipStream_t s, int grid, int block,
                                       int64_t small_max, int precombine, int group);
size_t seg_ctl_bytes();
hipError_t launch_check_offsets(const int64_t *offsets, int64_t nseg, int64_t n, int64_t *first_bad, hipStream_t s);
int seg_short_block();

// One piece of a served request (host and device layout).  `expected` is the
// request's total number of pieces when this piece belongs to the step that
// completes the request, kNotFinal otherwise; 1 means "round directly".
constexpr uint32_t kNotFinal = 0xFFFFFFFFu;
struct Piece {
  const double *x;
  int64_t n;
  double *out;
  int32_t slot;
  uint32_t expected;
};
static_assert(sizeof(Piece) == 32, "Piece layout");

// Served pieces (kernels_serve.hip): pieces [0, nshort) have at most
// short_max terms and are summed one per wavefront; the rest one per
// workgroup.  With host_pieces and at most kInlinePieces pieces the list
// travels in the kernel arguments (`pieces` is then not read); otherwise
// `pieces` is the device copy of the list.
constexpr int kInlinePieces = 32;
hipError_t launch_pieces(const Piece *pieces, const Piece *host_pieces, int nshort, int npieces, GlobalAcc *slots,
                         hipStream_t s, int grid, int precombine);
int pieces_block();

}  // namespace exsum
