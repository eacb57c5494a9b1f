// api.cpp -- the C ABI of include/exsum.h: argument checks, per-stream
// workspaces, launch planning.  No arithmetic on terms happens here; every
// step of the sum runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "exsum.h"
#include "exsum_internal.h"

namespace exsum {

int status_of(hipError_t e) {
  if (e == hipSuccess) return EXSUM_OK;
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? EXSUM_ENOMEM : EXSUM_EDEVICE;
}

namespace {
std::mutex g_cu_mu;
int g_cu[64] = {0};
}  // namespace

int cu_count(int dev) {
  if (dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lk(g_cu_mu);
  if (g_cu[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) {
      (void)hipGetLastError();
      v = 256;
    }
    g_cu[dev] = v;
  }
  return g_cu[dev];
}

namespace {

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

exsum_config default_config() {
  exsum_config c;
  c.large_block = 1024;
  c.large_vec = 4;
  c.large_depth = 2;
  c.large_mode = 1;
  c.large_grid = 0;
  c.precombine = 16;
  c.small_max = 4096;
  c.small_grid = 0;
  c.seg_grid = 0;
  c.seg_small_max = 20480;
  c.seg_mode = 0;
  c.seg_block = 256;
  c.seg_group = 8;
  c.seg_pad = 0;
  return c;
}

exsum_config g_cfg = default_config();

constexpr int64_t kMaxN = int64_t(1) << 40;

bool config_ok(const exsum_config &c) {
  if (!large_variant_exists(c.large_block, c.large_vec, c.large_depth, c.large_mode)) return false;
  if (c.large_grid < 0 || c.large_grid > kMaxGrid) return false;
  if (c.small_grid > kMaxGrid) return false;
  if (c.precombine < 0 || c.precombine > 64) return false;
  if (c.small_max < 0 || c.small_grid < 0 || c.small_grid > kMaxGrid) return false;
  if (c.seg_grid < 0 || c.seg_grid > kMaxGrid) return false;
  if (c.seg_small_max < 0 || c.seg_small_max > (int64_t(1) << 20)) return false;
  if (c.seg_mode != 0 && c.seg_mode != 1) return false;
  if (c.seg_block != 256 && c.seg_block != 512 && c.seg_block != 1024) return false;
  if (c.seg_group < 1 || c.seg_group > 64 || c.seg_pad != 0) return false;
  return true;
}


// Workspace for (current device, stream); allocated and zeroed on first use.
int get_workspace(hipStream_t s, Workspace **out, int *dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return status_of(e);
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, s);
  auto it = g_ws.find(key);
  if (it == g_ws.end()) {
    Workspace w;
    w.max_grid = kMaxGrid;
    void *p = nullptr;
    const size_t mb = (global_acc_bytes() + 255) / 256 * 256;
    const size_t bytes = mb + sizeof(double) * kMaxGrid + 256;
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return status_of(e);
    e = hipMemset(p, 0, bytes);
    if (e != hipSuccess) { (void)hipFree(p); return status_of(e); }
    w.acc = reinterpret_cast<GlobalAcc *>(p);
    w.partials = reinterpret_cast<double *>(static_cast<char *>(p) + mb);
    w.ticket = reinterpret_cast<unsigned int *>(static_cast<char *>(p) + mb + sizeof(double) * kMaxGrid);
    it = g_ws.emplace(key, w).first;
  }
  *out = &it->second;
  if (dev_out) *dev_out = dev;
  return EXSUM_OK;
}

// Launch the single sum with merge accumulator `acc` (zeroed, left zeroed).
hipError_t launch_sum(const double *x, int64_t n, double *out, hipStream_t s, const exsum_config &c,
                      GlobalAcc *acc, int dev) {
  hipError_t e;
  if (n <= c.small_max) {
    int grid = c.small_grid;
    if (grid == 0) grid = (int)std::min<int64_t>(std::max<int64_t>((n + 8191) / 8192, 1), 64);
    e = launch_small(x, n, acc, out, s, grid);
  } else {
    int grid = c.large_grid;
    if (grid == 0) {
      // one workgroup per compute unit, each with at least a few tiles
      const int64_t tile_terms = int64_t(2) * c.large_block * c.large_vec;
      const int64_t want = (n + 4 * tile_terms - 1) / (4 * tile_terms);
      grid = (int)std::min<int64_t>(std::max<int64_t>(want, 1), int64_t(cu_count(dev)));
    }
    e = launch_large(x, n, acc, out, s, c.large_block, c.large_vec, c.large_depth, c.large_mode, grid,
                     c.precombine);
  }
  return e;
}

int run_sum(const double *x, int64_t n, double *out, hipStream_t s, const exsum_config &c) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
  if (!config_ok(c)) return EXSUM_EINVAL;
  Workspace *w = nullptr;
  int dev = 0;
  int st = get_workspace(s, &w, &dev);
  if (st != EXSUM_OK) return st;
  return status_of(launch_sum(x, n, out, s, c, w->acc, dev));
}

// Launch shape of a sum over the small-only kernel or the large kernel's
// default variant (op_block() threads, 4 positions per thread per tile, T
// terms per position).
struct OpPlan {
  bool small;
  int grid;
};
OpPlan plan_op(int64_t n, int64_t terms_per_position, const exsum_config &c, int dev) {
  OpPlan p;
  p.small = n <= c.small_max;
  if (p.small) {
    p.grid = c.small_grid ? c.small_grid : (int)std::min<int64_t>(std::max<int64_t>((n + 8191) / 8192, 1), 64);
  } else if (c.large_grid) {
    p.grid = c.large_grid;
  } else {
    const int64_t tile_terms = terms_per_position * op_block() * 4;
    const int64_t want = (n + 4 * tile_terms - 1) / (4 * tile_terms);
    p.grid = (int)std::min<int64_t>(std::max<int64_t>(want, 1), int64_t(cu_count(dev)));
  }
  return p;
}

// Common set-up of the entry points below: configuration, workspace.
int op_setup(hipStream_t s, exsum_config *c, Workspace **w, int *dev) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    *c = g_cfg;
  }
  return get_workspace(s, w, dev);
}

bool acc_ptr_ok(const void *acc) { return acc != nullptr && (reinterpret_cast<uintptr_t>(acc) & 63) == 0; }

}  // namespace

}  // namespace exsum

using namespace exsum;

extern "C" {

const char *exsum_status_string(int status) {
  switch (status) {
    case EXSUM_OK: return "ok";
    case EXSUM_EINVAL: return "invalid argument";
    case EXSUM_ENOMEM: return "out of device memory";
    case EXSUM_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

int exsum_f64(const double *x, int64_t n, double *out, void *stream) {
  exsum_config c;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    c = g_cfg;
  }
  return run_sum(x, n, out, static_cast<hipStream_t>(stream), c);
}

int exsum_f64_noalloc(const double *x, int64_t n, double *out, void *stream) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
  exsum_config c;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    c = g_cfg;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return status_of(e);
  if (dev < 0 || dev >= kMaxDevices) return EXSUM_EINVAL;
  GlobalAcc *acc = nullptr;
  e = noalloc_scratch(dev, s, &acc);
  if (e != hipSuccess) return status_of(e);
  return status_of(launch_sum(x, n, out, s, c, acc, dev));
}

int exsum_f64_cfg(const double *x, int64_t n, double *out, void *stream, const exsum_config *cfg) {
  if (cfg == nullptr) return EXSUM_EINVAL;
  return run_sum(x, n, out, static_cast<hipStream_t>(stream), *cfg);
}

int exsum_inexact_f64(const double *x, int64_t n, double *out, void *stream) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace *w = nullptr;
  int dev = 0;
  int st = get_workspace(s, &w, &dev);
  if (st != EXSUM_OK) return st;
  // the exact kernel's geometry: one workgroup per compute unit, fewer for
  // inputs under about four tiles per workgroup
  const int64_t tile_terms = int64_t(2) * inexact_block() * 4;
  const int64_t want = (n + 4 * tile_terms - 1) / (4 * tile_terms);
  const int grid = (int)std::min<int64_t>(std::max<int64_t>(want, 1),
                                          std::min<int64_t>(int64_t(cu_count(dev)), w->max_grid));
  return status_of(launch_inexact(x, n, w->partials, w->ticket, out, s, grid));
}

int exsum_segmented_f64(const double *x, const int64_t *offsets, int64_t nseg, double *out, void *stream) {
  if (nseg < 0 || nseg >= (int64_t(1) << 31)) return EXSUM_EINVAL;
  if (nseg == 0) return EXSUM_OK;
  // x may be NULL when every segment is empty (no term is read then)
  if (offsets == nullptr || out == nullptr) return EXSUM_EINVAL;
  exsum_config c;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    c = g_cfg;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace *w = nullptr;
  int dev = 0;
  int st = get_workspace(s, &w, &dev);
  if (st != EXSUM_OK) return st;
  GlobalAcc *accs = nullptr;
  long long *chunks = nullptr;
  void *ctl = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (w->seg_accs == nullptr) {
      void *p = nullptr;
      const size_t abytes = global_acc_bytes() * (size_t)kMaxGrid;
      const size_t cbytes = sizeof(long long) * (size_t)kMaxGrid;
      const size_t bytes = abytes + cbytes + seg_ctl_bytes();
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) return status_of(e);
      e = hipMemset(p, 0, bytes);
      if (e != hipSuccess) { (void)hipFree(p); return status_of(e); }
      w->seg_accs = reinterpret_cast<GlobalAcc *>(p);
      w->seg_chunks = reinterpret_cast<long long *>(static_cast<char *>(p) + abytes);
      w->seg_ctl = static_cast<char *>(p) + abytes + cbytes;
    }
    accs = w->seg_accs;
    chunks = w->seg_chunks;
    ctl = w->seg_ctl;
  }
  if (c.seg_mode == 1) {
    // one persistent launch, as many workgroups per compute unit as fit its
    // LDS and registers (three of 256 threads, two of 512, one of 1024); at
    // most kMaxGrid (one merge slot per workgroup)
    int pgrid = c.seg_grid;
    if (pgrid == 0) pgrid = (c.seg_block == 1024 ? 1 : (c.seg_block == 512 ? 2 : 3)) * cu_count(dev);
    return status_of(launch_segmented_persistent(x, offsets, nseg, out, accs, ctl, s, pgrid, c.seg_block,
                                                 c.seg_small_max, c.precombine, c.seg_group));
  }
  int grid = c.seg_grid;
  // long segments: eight workgroups (term ranges) per compute unit, three
  // of which fit at once, so that the dispatcher hands more ranges to
  // compute units whose ranges hold fewer long segments
  if (grid == 0) grid = std::min(8 * cu_count(dev), kMaxGrid);
  // short segments: one workgroup per compute unit
  const int short_grid = std::min(cu_count(dev), seg_short_block());
  return status_of(launch_segmented(x, offsets, nseg, out, accs, chunks, s, grid, short_grid, c.seg_small_max,
                                    c.precombine));
}

int exsum_check_offsets(const int64_t *offsets, int64_t nseg, int64_t n, int64_t *first_bad, void *stream) {
  if (nseg < 0 || nseg >= (int64_t(1) << 31) || first_bad == nullptr || (nseg > 0 && offsets == nullptr))
    return EXSUM_EINVAL;
  return status_of(launch_check_offsets(offsets, nseg, n, first_bad, static_cast<hipStream_t>(stream)));
}

int exsum_sqnorm_f64(const double *x, int64_t n, double *out, void *stream) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  exsum_config c;
  Workspace *w = nullptr;
  int dev = 0;
  int st = op_setup(s, &c, &w, &dev);
  if (st != EXSUM_OK) return st;
  const OpPlan p = plan_op(n, 2, c, dev);
  return status_of(launch_sqnorm(x, n, out, w->acc, s, p.grid, p.small, c.precombine));
}

int exsum_dot_f64(const double *x, const double *y, int64_t n, double *out, void *stream) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && (x == nullptr || y == nullptr))) return EXSUM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  exsum_config c;
  Workspace *w = nullptr;
  int dev = 0;
  int st = op_setup(s, &c, &w, &dev);
  if (st != EXSUM_OK) return st;
  const OpPlan p = plan_op(n, 2, c, dev);
  return status_of(launch_dot(x, y, n, out, w->acc, s, p.grid, p.small, c.precombine));
}

int exsum_mean_f64(const double *x, int64_t n, double *out, void *stream) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  exsum_config c;
  Workspace *w = nullptr;
  int dev = 0;
  int st = op_setup(s, &c, &w, &dev);
  if (st != EXSUM_OK) return st;
  const OpPlan p = plan_op(n, 2, c, dev);
  return status_of(launch_mean(x, n, out, w->acc, s, p.grid, p.small, c.precombine));
}

int exsum_f32(const float *x, int64_t n, float *out, void *stream) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  exsum_config c;
  Workspace *w = nullptr;
  int dev = 0;
  int st = op_setup(s, &c, &w, &dev);
  if (st != EXSUM_OK) return st;
  const OpPlan p = plan_op(n, 4, c, dev);
  return status_of(launch_f32(x, n, out, w->acc, s, p.grid, p.small, c.precombine));
}

int exsum_dot_f32(const float *x, const float *y, int64_t n, float *out, void *stream) {
  if (n < 0 || n >= kMaxN || out == nullptr || (n > 0 && (x == nullptr || y == nullptr))) return EXSUM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  exsum_config c;
  Workspace *w = nullptr;
  int dev = 0;
  int st = op_setup(s, &c, &w, &dev);
  if (st != EXSUM_OK) return st;
  const OpPlan p = plan_op(n, 4, c, dev);
  return status_of(launch_dot_f32(x, y, n, out, w->acc, s, p.grid, p.small, c.precombine));
}

int exsum_acc_zero(void *acc, void *stream) {
  if (!acc_ptr_ok(acc)) return EXSUM_EINVAL;
  return status_of(launch_acc_zero(static_cast<GlobalAcc *>(acc), static_cast<hipStream_t>(stream)));
}

int exsum_acc_add_f64(void *acc, const double *x, int64_t n, void *stream) {
  if (!acc_ptr_ok(acc) || n < 0 || n >= kMaxN || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
  if (n == 0) return EXSUM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  exsum_config c;
  Workspace *w = nullptr;
  int dev = 0;
  int st = op_setup(s, &c, &w, &dev);
  if (st != EXSUM_OK) return st;
  const OpPlan p = plan_op(n, 2, c, dev);
  return status_of(launch_acc_add(x, n, static_cast<GlobalAcc *>(acc), w->acc, s, p.grid, p.small, c.precombine));
}

int exsum_acc_merge(void *dst, const void *src, void *stream) {
  if (!acc_ptr_ok(dst) || !acc_ptr_ok(src) || dst == src) return EXSUM_EINVAL;
  return status_of(launch_acc_merge(static_cast<GlobalAcc *>(dst), static_cast<const GlobalAcc *>(src),
                                    static_cast<hipStream_t>(stream)));
}

int exsum_acc_round_f64(const void *acc, double *out, void *stream) {
  if (!acc_ptr_ok(acc) || out == nullptr) return EXSUM_EINVAL;
  return status_of(launch_acc_round(static_cast<const GlobalAcc *>(acc), out, static_cast<hipStream_t>(stream)));
}

int exsum_large_variants(int32_t *out, int64_t cap, int64_t *count) {
  if (count == nullptr || cap < 0 || (cap > 0 && out == nullptr)) return EXSUM_EINVAL;
  *count = large_variants(out, cap);
  return EXSUM_OK;
}

int exsum_get_config(exsum_config *cfg) {
  if (cfg == nullptr) return EXSUM_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  *cfg = g_cfg;
  return EXSUM_OK;
}

int exsum_set_config(const exsum_config *cfg) {
  if (cfg == nullptr || !config_ok(*cfg)) return EXSUM_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  g_cfg = *cfg;
  return EXSUM_OK;
}

int exsum_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  hipError_t first = hipSuccess;
  for (auto &kv : g_ws) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(kv.first.first);
    hipError_t e = hipFree(kv.second.acc);
    if (first == hipSuccess) first = e;
    if (kv.second.seg_accs) {
      e = hipFree(kv.second.seg_accs);
      if (first == hipSuccess) first = e;
    }
    (void)hipSetDevice(cur);
  }
  g_ws.clear();
  return status_of(first);
}

}  // extern "C"
