// exsum_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exsum {

constexpr int kMaxGrid = 8192;       // most workgroups one single-sum launch may use

struct GlobalAcc;
struct MergeRows;

// Per-(device, stream) workspace.  Everything the kernels write here is left
// zeroed when a call completes.
struct Workspace {
  MergeRows *rows = nullptr;           // merge workspace of the single-sum kernels
  double *partials = nullptr;          // per-workgroup partials of the inexact sum
  unsigned int *ticket = nullptr;      // ticket of the inexact sum
  int max_grid = 0;                    // capacity of `partials`
  // segmented calls: one accumulator per workgroup boundary (kMaxGrid)
  GlobalAcc *seg_accs = nullptr;
};

// Launchers (kernels_sum.hip).  Return a hipError_t.
hipError_t launch_large(const double *x, int64_t n, MergeRows *M, double *out, hipStream_t s,
                        int block, int vec, int depth, int mode, int grid, int precombine);
bool large_variant_exists(int block, int vec, int depth, int mode);
hipError_t launch_small(const double *x, int64_t n, MergeRows *M, double *out, hipStream_t s,
                        int grid);
hipError_t launch_inexact(const double *x, int64_t n, double *partials, unsigned int *ticket,
                          double *out, hipStream_t s, int grid);

// Segmented sums (kernels_seg.hip).
size_t global_acc_bytes();
hipError_t launch_segmented(const double *x, const int64_t *offsets, int64_t nseg, double *out,
                            GlobalAcc *accs, hipStream_t s, int grid, int64_t small_max, int precombine);

size_t merge_rows_bytes();

}  // namespace exsum
