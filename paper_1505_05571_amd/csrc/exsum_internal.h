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
  // segmented calls
  void *seg = nullptr;                 // segment workspace (see kernels_seg.hip)
  size_t seg_bytes = 0;
  int64_t seg_cap = 0;                 // segments the workspace holds
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
size_t seg_workspace_bytes(int64_t cap);
hipError_t launch_segmented(const double *x, const int64_t *offsets, int64_t nseg, double *out,
                            void *ws, int64_t cap, hipStream_t s, int grid, int64_t small_max,
                            int64_t tile, int precombine);

size_t merge_rows_bytes();

}  // namespace exsum
