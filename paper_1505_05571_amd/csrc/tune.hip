// tune.hip -- the launch-configuration tuner.
//
// Every field of exsum_config changes only speed, never a result bit, so
// the tuner times candidate configurations on the current device with
// synthetic inputs shaped like the benchmark workloads, keeps the fastest,
// and checks on the way that all candidates give the same bits.  Decisions,
// in order (each uses the winners of the ones before):
//   1. large-accumulator variant (block, vec, depth, transfer mode), grid and
//      pre-combine threshold, timed on three input distributions and chosen
//      by its worst ratio to the fastest candidate;
//   2. small_max: the largest tested length at which the small-only kernel
//      still beats the large one;
//   3. the segmented call's launch: mode (two launches or one persistent
//      launch), threshold seg_small_max, workgroups, and for the persistent
//      launch its workgroup size and unit size, timed on two batches of
//      lognormal segment lengths (sigma 2 and 1.63, median 1000) and chosen
//      by the worst ratio to the fastest candidate.
// The result becomes the process configuration and can be written to a
// JSON file that exsum_load_tuning() reads back on the same kind of device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "exsum.h"
#include "exsum_internal.h"

namespace exsum {
namespace {

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  // the splitmix64 output function (Steele, Lea and Flood 2014)
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Synthetic terms.  kind 0: random sign, exponent uniform in [-300, 300],
// random mantissa; kind 1: positive, all in [1, 2) (one large-accumulator
// chunk); kind 2: random sign, exponent in [-30, 30] (few chunks).
__global__ void gen_kernel(double *x, long long n, unsigned long long seed, int kind) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long r = mix64(seed ^ mix64((unsigned long long)i));
    const unsigned long long m = r & ((1ull << 52) - 1);
    const unsigned long long s = kind == 1 ? 0ull : (r >> 63) << 63;
    const unsigned int span = kind == 0 ? 601u : (kind == 1 ? 1u : 61u);
    const unsigned int k = (unsigned int)((r >> 52) & 0x7FFu) % span;
    const unsigned long long e = kind == 0 ? 1023 - 300 + k : (kind == 1 ? 1023 : 1023 - 30 + k);
    x[i] = __longlong_as_double((long long)(s | (e << 52) | m));
  }
}

struct Timer {
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  explicit Timer(hipStream_t st) : s(st) {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  // average microseconds of `reps` back-to-back calls after one untimed call;
  // a negative value if a call failed
  template <class F>
  double time_us(F f, int reps) {
    if (f() != EXSUM_OK) return -1.0;
    if (hipEventRecord(a, s) != hipSuccess) return -1.0;
    for (int r = 0; r < reps; r++)
      if (f() != EXSUM_OK) return -1.0;
    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0;
    return 1000.0 * ms / reps;
  }
};

struct Variant {
  int block, vec, depth, mode;
};
// The large kernel's built shapes, from the library's one table.
std::vector<Variant> built_variants() {
  std::vector<int32_t> v(4 * (size_t)large_variants(nullptr, 0));
  const int n = large_variants(v.data(), (int64_t)(v.size() / 4));
  std::vector<Variant> out;
  for (int k = 0; k < n; k++) out.push_back(Variant{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]});
  return out;
}

std::string config_json(const exsum_config &c) {
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "{\"large_block\": %d, \"large_vec\": %d, \"large_depth\": %d, \"large_mode\": %d, "
                "\"large_grid\": %d, \"precombine\": %d, \"small_max\": %lld, \"small_grid\": %d, "
                "\"seg_grid\": %d, \"seg_small_max\": %lld, \"seg_mode\": %d, \"seg_block\": %d, "
                "\"seg_group\": %d}",
                c.large_block, c.large_vec, c.large_depth, c.large_mode, c.large_grid, c.precombine,
                (long long)c.small_max, c.small_grid, c.seg_grid, (long long)c.seg_small_max, c.seg_mode,
                c.seg_block, c.seg_group);
  return buf;
}

std::string json_escape(const char *s) {
  std::string o;
  for (; *s; s++) {
    if (*s == '"' || *s == '\\') o += '\\';
    if ((unsigned char)*s >= 0x20) o += *s;
  }
  return o;
}

// Integer value of "key": in text (after position `from`); false if absent.
bool json_int(const std::string &t, const char *key, long long *v, size_t from = 0) {
  const std::string k = std::string("\"") + key + "\":";
  size_t p = t.find(k, from);
  if (p == std::string::npos) return false;
  p += k.size();
  while (p < t.size() && (t[p] == ' ' || t[p] == '\t' || t[p] == '\n')) p++;
  char *end = nullptr;
  const long long x = std::strtoll(t.c_str() + p, &end, 10);
  if (end == t.c_str() + p) return false;
  *v = x;
  return true;
}

bool json_str(const std::string &t, const char *key, std::string *v) {
  const std::string k = std::string("\"") + key + "\":";
  size_t p = t.find(k);
  if (p == std::string::npos) return false;
  p += k.size();
  while (p < t.size() && (t[p] == ' ' || t[p] == '\t' || t[p] == '\n')) p++;
  if (p >= t.size() || t[p] != '"') return false;
  std::string o;
  for (p++; p < t.size() && t[p] != '"'; p++) {
    if (t[p] == '\\' && p + 1 < t.size()) p++;
    o += t[p];
  }
  *v = o;
  return true;
}

struct DeviceId {
  std::string name, arch;
  int cus = 0;
};

int device_id(DeviceId *d, std::string *why = nullptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e == hipSuccess) {
      d->name = p.name;
      d->arch = p.gcnArchName;
      d->cus = p.multiProcessorCount;
      return EXSUM_OK;
    }
  }
  if (why) *why = std::string("device query: ") + hipGetErrorName(e);
  return status_of(e);
}

// Lognormal segment lengths (median 1000, clipped to [1, 1e6]) as offsets;
// deterministic for a seed.
std::vector<int64_t> lognormal_offsets(int nseg, unsigned seed, double sigma) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> nd(std::log(1000.0), sigma);
  std::vector<int64_t> off(nseg + 1, 0);
  for (int i = 0; i < nseg; i++) {
    double L = std::rint(std::exp(nd(g)));
    L = std::min(std::max(L, 1.0), 1e6);
    off[i + 1] = off[i] + (int64_t)L;
  }
  return off;
}

struct Buffers {
  double *x = nullptr, *x2 = nullptr, *out = nullptr;
  int64_t *off = nullptr;
  ~Buffers() {
    if (x) (void)hipFree(x);
    if (x2) (void)hipFree(x2);
    if (out) (void)hipFree(out);
    if (off) (void)hipFree(off);
  }
};

}  // namespace
}  // namespace exsum

using namespace exsum;

namespace {
int autotune_body(const char *cache_path, std::string &js, std::string &err, void *stream);
}

extern "C" int exsum_autotune(const char *cache_path, char *report, int64_t report_len, void *stream) {
  if (report_len < 0 || (report_len > 0 && report == nullptr)) return EXSUM_EINVAL;
  std::string js, err;
  const int st = autotune_body(cache_path, js, err, stream);
  if (st != EXSUM_OK) js = "{\"error\": \"" + json_escape(err.c_str()) + "\"}\n";
  if (report_len > 0) {
    const size_t m = std::min((size_t)report_len - 1, js.size());
    std::memcpy(report, js.data(), m);
    report[m] = '\0';
  }
  return st;
}

namespace {
int autotune_body(const char *cache_path, std::string &js, std::string &err, void *stream) {
  auto fail = [&err](int code, const std::string &what) {
    err = what;
    return code;
  };
  hipStream_t s = static_cast<hipStream_t>(stream);
  DeviceId id;
  std::string why;
  int st = device_id(&id, &why);
  if (st != EXSUM_OK) return fail(st, why);
  exsum_config base;
  exsum_get_config(&base);
  // the process configuration is restored unless tuning completes
  struct Restore {
    exsum_config c;
    bool keep = false;
    ~Restore() {
      if (!keep) exsum_set_config(&c);
    }
  } restore{base};

  // inputs: 10^8 terms (800 MB, beyond the last-level cache; not a power of
  // two, so workgroup ranges do not all start on the same address bits) for
  // the single sums; two batches of 32768 segments with lognormal lengths,
  // sigma 2 and 1.63 (the benchmark batches' shapes at half their count)
  const int64_t n_single = 100000000;
  const int nseg = 32768;
  const std::vector<int64_t> offs[2] = {lognormal_offsets(nseg, 12345u, 2.0), lognormal_offsets(nseg, 54321u, 1.63)};
  const int64_t n_seg = std::max(offs[0][nseg], offs[1][nseg]);
  const int64_t n_buf = std::max(n_single, n_seg);
  Buffers B;
  hipError_t e = hipMalloc(&B.x, sizeof(double) * n_buf);
  if (e == hipSuccess) e = hipMalloc(&B.x2, sizeof(double) * n_single);
  if (e == hipSuccess) e = hipMalloc(&B.out, sizeof(double) * (nseg + 64));
  if (e == hipSuccess) e = hipMalloc(&B.off, sizeof(int64_t) * 2 * (nseg + 1));
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? EXSUM_ENOMEM : status_of(e), "allocating the inputs");
  Timer T(s);
  std::string log;
  char line[256];
  auto bits_of = [&](int count, std::vector<unsigned long long> *v) -> int {
    v->assign(count, 0);
    hipError_t er = hipMemcpyAsync(v->data(), B.out, sizeof(double) * count, hipMemcpyDeviceToHost, s);
    if (er == hipSuccess) er = hipStreamSynchronize(s);
    return er == hipSuccess ? EXSUM_OK : status_of(er);
  };
  auto gen = [&](int64_t n, int kind, unsigned long long seed) -> int {
    hipLaunchKernelGGL(gen_kernel, dim3(1024), dim3(256), 0, s, B.x, (long long)n, seed, kind);
    return status_of(hipGetLastError());
  };

  // 1. large-accumulator configuration
  exsum_config best = base;
  const int grids[] = {0, 2 * id.cus};
  const int pcs[] = {0, 8, 16, 32};
  std::vector<unsigned long long> want, got;
  std::vector<exsum_config> cands;
  for (const Variant &v : built_variants())
    for (int g : grids)
      for (int pc : pcs) {
        exsum_config c = base;
        c.large_block = v.block;
        c.large_vec = v.vec;
        c.large_depth = v.depth;
        c.large_mode = v.mode;
        c.large_grid = g;
        c.precombine = pc;
        c.small_max = 0;
        cands.push_back(c);
      }
  // Each candidate is timed on three inputs (wide exponents, one chunk,
  // narrow exponents), two copies alternated so that no call reads what the
  // previous one left in cache, best of two rounds.  Its score is its worst
  // ratio to the fastest candidate over the inputs: a configuration that is
  // fast on one distribution and slow on another (the count rule without
  // pre-combining, on one hot chunk) is not chosen.
  const int nk = 3;
  std::vector<double> tk[nk];
  for (int kind = 0; kind < nk; kind++) {
    tk[kind].assign(cands.size(), 1e300);
    if ((st = gen(n_single, kind, 7 + kind)) != EXSUM_OK) return fail(st, "generating an input");
    e = hipMemcpyAsync(B.x2, B.x, sizeof(double) * n_single, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(status_of(e), "copying an input");
    {
      exsum_config c = base;
      c.small_max = 0;
      if ((st = exsum_f64_cfg(B.x, n_single, B.out, s, &c)) != EXSUM_OK) return fail(st, "a reference call failed");
      if ((st = bits_of(1, &want)) != EXSUM_OK) return fail(st, "reading a result");
    }
    for (int round = 0; round < 2; round++)
      for (size_t i = 0; i < cands.size(); i++) {
        const exsum_config &c = cands[i];
        int flip = 0;
        const double t = T.time_us(
            [&] { return exsum_f64_cfg((flip++ & 1) ? B.x2 : B.x, n_single, B.out, s, &c); }, 6);
        if (t < 0) return fail(EXSUM_EDEVICE, "a timed call failed");
        if ((st = bits_of(1, &got)) != EXSUM_OK) return fail(st, "reading a result");
        if (got != want)
          return fail(EXSUM_EDEVICE, "candidate " + config_json(c) + " changed the bits of input " + std::to_string(kind));
        tk[kind][i] = std::min(tk[kind][i], t);
      }
  }
  std::vector<double> score(cands.size(), 0.0);
  for (int kind = 0; kind < nk; kind++) {
    const double m = *std::min_element(tk[kind].begin(), tk[kind].end());
    for (size_t i = 0; i < cands.size(); i++) score[i] = std::max(score[i], tk[kind][i] / m);
  }
  size_t bi = 0, si = cands.size();
  for (size_t i = 0; i < cands.size(); i++) {
    if (score[i] < score[bi] || (score[i] == score[bi] && tk[0][i] < tk[0][bi])) bi = i;
    const exsum_config &c = cands[i];
    if (c.large_block == base.large_block && c.large_vec == base.large_vec && c.large_depth == base.large_depth &&
        c.large_mode == base.large_mode && c.large_grid == base.large_grid && c.precombine == base.precombine)
      si = i;
  }
  best = cands[bi];
  best.small_max = base.small_max;
  {
    auto row = [&](size_t i) {
      char b2[160];
      std::snprintf(b2, sizeof b2, "{\"score\": %.4f, \"us\": [%.2f, %.2f, %.2f]}", score[i], tk[0][i], tk[1][i],
                    tk[2][i]);
      return std::string(b2);
    };
    log += "\"large_terms\": " + std::to_string((long long)n_single) + ", \"large_chosen\": " + row(bi) +
           (si < cands.size() ? ", \"large_start\": " + row(si) : std::string()) + ", ";
  }

  // 2. small-only versus large crossover
  {
    if ((st = gen(n_single, 2, 11)) != EXSUM_OK) return fail(st, "generating an input");
    const int64_t lens[] = {512, 1024, 2048, 4096, 8192, 16384, 32768, 65536};
    int64_t chosen = lens[0] / 2;
    log += "\"crossover\": [";
    for (size_t k = 0; k < sizeof lens / sizeof lens[0]; k++) {
      const int64_t n = lens[k];
      exsum_config cs = best, cl = best;
      cs.small_max = int64_t(1) << 40;
      cl.small_max = 0;
      const double ts = T.time_us([&] { return exsum_f64_cfg(B.x, n, B.out, s, &cs); }, 20);
      if (ts < 0) return fail(EXSUM_EDEVICE, "a timed call failed (crossover)");
      std::vector<unsigned long long> a, b;
      if ((st = bits_of(1, &a)) != EXSUM_OK) return fail(st, "reading a result");
      const double tl = T.time_us([&] { return exsum_f64_cfg(B.x, n, B.out, s, &cl); }, 20);
      if (tl < 0) return fail(EXSUM_EDEVICE, "a timed call failed (crossover)");
      if ((st = bits_of(1, &b)) != EXSUM_OK) return fail(st, "reading a result");
      if (a != b) return fail(EXSUM_EDEVICE, "small and large paths differ at n=" + std::to_string(n));
      std::snprintf(line, sizeof line, "%s[%lld, %.2f, %.2f]", k ? ", " : "", (long long)n, ts, tl);
      log += line;
      // the small-only kernel keeps every length up to the first it loses at
      if (ts <= tl && chosen == (k ? lens[k - 1] : lens[0] / 2)) chosen = n;
    }
    log += "], ";
    best.small_max = chosen;
  }

  // 3. segmented launch: candidates over the mode, the short/long threshold,
  // the workgroups and the persistent launch's shapes; each timed on both
  // batches (best of two rounds), scored by its worst ratio to the fastest
  // on either, and every candidate's bits compared with the first's
  {
    for (int b = 0; b < 2; b++) {
      e = hipMemcpyAsync(B.off + b * (nseg + 1), offs[b].data(), sizeof(int64_t) * (nseg + 1),
                         hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return fail(status_of(e), "copying the offsets");
    }
    if ((st = gen(n_seg, 2, 13)) != EXSUM_OK) return fail(st, "generating an input");
    std::vector<exsum_config> sc;
    for (int64_t sm : {12288, 16384, 20480})
      for (int g : {0, 6 * id.cus, 12 * id.cus}) {
        exsum_config c = best;
        c.seg_mode = 0;
        c.seg_small_max = sm;
        c.seg_grid = g;
        sc.push_back(c);
      }
    for (int blk : {256, 512})
      for (int grp : {8, 16})
        for (int64_t sm : {8192, 12288}) {
          exsum_config c = best;
          c.seg_mode = 1;
          c.seg_block = blk;
          c.seg_group = grp;
          c.seg_small_max = sm;
          c.seg_grid = 0;
          sc.push_back(c);
        }
    std::vector<double> ts[2];
    std::vector<unsigned long long> ref[2];
    for (int b = 0; b < 2; b++) ts[b].assign(sc.size(), 1e300);
    for (int round = 0; round < 2; round++)
      for (int b = 0; b < 2; b++)
        for (size_t i = 0; i < sc.size(); i++) {
          if ((st = exsum_set_config(&sc[i])) != EXSUM_OK) return fail(st, "setting a candidate configuration");
          const int64_t *o = B.off + b * (nseg + 1);
          const double t = T.time_us([&] { return exsum_segmented_f64(B.x, o, nseg, B.out, s); }, 5);
          if (t < 0) return fail(EXSUM_EDEVICE, "a timed call failed (segmented)");
          if ((st = bits_of(nseg, &got)) != EXSUM_OK) return fail(st, "reading a result");
          if (ref[b].empty()) ref[b] = got;
          if (got != ref[b]) return fail(EXSUM_EDEVICE, "segmented candidate " + config_json(sc[i]) + " changed the bits");
          ts[b][i] = std::min(ts[b][i], t);
        }
    const double m0 = *std::min_element(ts[0].begin(), ts[0].end());
    const double m1 = *std::min_element(ts[1].begin(), ts[1].end());
    size_t bi = 0;
    std::vector<double> sscore(sc.size());
    for (size_t i = 0; i < sc.size(); i++) {
      sscore[i] = std::max(ts[0][i] / m0, ts[1][i] / m1);
      if (sscore[i] < sscore[bi]) bi = i;
    }
    log += "\"segmented\": [";
    for (size_t i = 0; i < sc.size(); i++) {
      std::snprintf(line, sizeof line, "%s{\"mode\": %d, \"small_max\": %lld, \"grid\": %d, \"block\": %d, "
                    "\"group\": %d, \"us\": [%.2f, %.2f], \"score\": %.4f}", i ? ", " : "", sc[i].seg_mode,
                    (long long)sc[i].seg_small_max, sc[i].seg_grid, sc[i].seg_block, sc[i].seg_group, ts[0][i],
                    ts[1][i], sscore[i]);
      log += line;
    }
    log += "]";
    best = sc[bi];
  }
  if ((st = exsum_set_config(&best)) != EXSUM_OK) return fail(st, "setting a candidate configuration");
  restore.keep = true;

  js = "{\"exsum_tuning\": 1, \"device\": \"" + json_escape(id.name.c_str()) + "\", \"arch\": \"" +
                   json_escape(id.arch.c_str()) + "\", \"cus\": " + std::to_string(id.cus) +
                   ", \"config\": " + config_json(best) + ", \"measured\": {" + log + "}}\n";
  if (cache_path) {
    FILE *f = std::fopen(cache_path, "w");
    if (!f) return fail(EXSUM_EINVAL, "cannot open the cache file");
    const bool ok = std::fwrite(js.data(), 1, js.size(), f) == js.size();
    if (std::fclose(f) != 0 || !ok) return fail(EXSUM_EINVAL, "cannot write the cache file");
  }
  return EXSUM_OK;
}
}  // namespace

extern "C" int exsum_load_tuning(const char *cache_path) {
  if (cache_path == nullptr) return EXSUM_EINVAL;
  FILE *f = std::fopen(cache_path, "r");
  if (!f) return EXSUM_EINVAL;
  std::string t;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, k);
  std::fclose(f);
  long long ver = 0, cus = 0;
  std::string name, arch;
  if (!json_int(t, "exsum_tuning", &ver) || ver != 1 || !json_int(t, "cus", &cus) || !json_str(t, "device", &name) ||
      !json_str(t, "arch", &arch))
    return EXSUM_EINVAL;
  const size_t cpos = t.find("\"config\":");
  if (cpos == std::string::npos) return EXSUM_EINVAL;
  exsum_config c;
  (void)exsum_get_config(&c);
  long long v[13];
  const char *keys[13] = {"large_block", "large_vec",  "large_depth", "large_mode", "large_grid",
                          "precombine",  "small_max",  "small_grid",  "seg_grid",   "seg_small_max",
                          "seg_mode",    "seg_block",  "seg_group"};
  for (int i = 0; i < 13; i++)
    if (!json_int(t, keys[i], &v[i], cpos)) return EXSUM_EINVAL;
  c.large_block = (int32_t)v[0];
  c.large_vec = (int32_t)v[1];
  c.large_depth = (int32_t)v[2];
  c.large_mode = (int32_t)v[3];
  c.large_grid = (int32_t)v[4];
  c.precombine = (int32_t)v[5];
  c.small_max = v[6];
  c.small_grid = (int32_t)v[7];
  c.seg_grid = (int32_t)v[8];
  c.seg_small_max = v[9];
  c.seg_mode = (int32_t)v[10];
  c.seg_block = (int32_t)v[11];
  c.seg_group = (int32_t)v[12];
  c.seg_pad = 0;
  DeviceId id;
  const int st = device_id(&id);
  if (st != EXSUM_OK) return st;
  if (name != id.name || arch != id.arch || cus != id.cus) return EXSUM_EINVAL;   // tuned elsewhere
  return exsum_set_config(&c);
}
