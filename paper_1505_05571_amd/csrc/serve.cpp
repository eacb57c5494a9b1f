// serve.cpp -- the serving loop of include/exsum.h: a continuous-batching
// scheduler on the host, a server that turns its steps into piece-kernel
// launches on one stream, and real-time trace replays (batched and serial).
// No arithmetic on terms happens here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <chrono>
#include <deque>
#include <list>
#include <unordered_map>
#include <utility>
#include <vector>

#include "exsum.h"
#include "exsum_internal.h"

namespace exsum {
namespace {

constexpr int64_t kMaxTerms = int64_t(1) << 40;

exsum_server_config default_server_config() {
  exsum_server_config c;
  c.step_terms = int64_t(1) << 27;
  c.piece_terms = int64_t(1) << 16;
  c.short_max = 4096;
  c.max_slots = 4096;
  c.max_pieces = 16384;
  c.max_inflight = 2;
  c.precombine = 16;
  c.mem_budget = 0;
  return c;
}

// Device bytes a request holds while admitted: an accumulator slot if it is
// cut into pieces, and one piece descriptor per piece of a step in flight.
constexpr int64_t kSlotBytes = 576;
constexpr int64_t kPieceBytes = (int64_t)sizeof(Piece);
constexpr int64_t kNoBudget = INT64_MAX;

bool server_config_ok(const exsum_server_config &c) {
  if (c.piece_terms < 1 || c.piece_terms >= kMaxTerms) return false;
  if (c.step_terms < c.piece_terms || c.step_terms >= kMaxTerms) return false;
  if (c.short_max < 0) return false;
  if (c.max_slots < 1 || c.max_slots > (1 << 20)) return false;
  if (c.max_pieces < 1 || c.max_pieces > (1 << 20)) return false;
  if (c.max_inflight < 1 || c.max_inflight > 64) return false;
  if (c.precombine < 0 || c.precombine > 64) return false;
  // a budget must hold at least one slot and one piece, or a long request
  // could never be admitted
  if (c.mem_budget != 0 && c.mem_budget < kSlotBytes + kPieceBytes) return false;
  return true;
}

// ---- scheduler (host logic only) -------------------------------------------

struct PlannedPiece {
  int64_t id;
  int64_t off;
  int64_t len;
  int32_t slot;
  uint32_t expected;
};

class Scheduler {
 public:
  explicit Scheduler(const exsum_server_config &c) : cfg_(c), budget_(c.mem_budget ? c.mem_budget : kNoBudget) {
    free_slots_.reserve(c.max_slots);
    for (int32_t i = c.max_slots - 1; i >= 0; i--) free_slots_.push_back(i);
  }

  void submit(int64_t id, int64_t n) { pending_.push_back(Req{id, n, 0, 0, -1}); }

  void release_slot(int32_t slot) {
    if (slot >= 0) {
      free_slots_.push_back(slot);
      held_ -= kSlotBytes;
    }
  }

  bool idle() const { return pending_.empty() && active_.empty(); }

  // Plan one step.  `finals` receives (id, slot) of the requests whose last
  // piece is in this step.  `inflight_bytes`: piece descriptors of the steps
  // still queued on the device, which count against the memory budget.
  void plan(std::vector<PlannedPiece> &out, std::vector<std::pair<int64_t, int32_t>> &finals,
            int64_t inflight_bytes = 0) {
    out.clear();
    finals.clear();
    admit(inflight_bytes);
    int64_t budget = cfg_.step_terms;
    // pieces this step may describe: max_pieces, and what the memory budget
    // leaves after the slots held and the steps in flight
    int64_t cap = cfg_.max_pieces;
    if (budget_ != kNoBudget) cap = std::min(cap, std::max<int64_t>(0, (budget_ - held_ - inflight_bytes) / kPieceBytes));
    // pass 1: one piece for every active request, oldest first (a request
    // that fits in one piece is scheduled whole or not at all)
    for (auto &r : active_) {
      if ((int64_t)out.size() >= cap) break;
      const int64_t len = std::min(r.n - r.next, cfg_.piece_terms);
      if (r.next > 0 && len == 0) continue;
      if (len > budget) continue;
      add(r, len, out);
      budget -= len;
    }
    // pass 2: the rest of the budget to the oldest requests that hold a slot
    for (auto &r : active_) {
      if (budget <= 0 || (int64_t)out.size() >= cap) break;
      if (r.slot < 0) continue;
      while (r.next < r.n && budget > 0 && (int64_t)out.size() < cap) {
        const int64_t len = std::min(std::min(r.n - r.next, cfg_.piece_terms), budget);
        add(r, len, out);
        budget -= len;
      }
    }
    // the step completes every request whose terms are now all scheduled
    std::unordered_map<int64_t, uint32_t> total;
    for (auto it = active_.begin(); it != active_.end();) {
      if (it->pieces > 0 && it->next == it->n) {
        total[it->id] = it->pieces;
        finals.emplace_back(it->id, it->slot);
        it = active_.erase(it);
      } else {
        ++it;
      }
    }
    for (auto &p : out) {
      auto t = total.find(p.id);
      p.expected = (t == total.end()) ? kNotFinal : t->second;
    }
  }

 private:
  struct Req {
    int64_t id;
    int64_t n;
    int64_t next;     // terms scheduled so far
    uint32_t pieces;  // pieces scheduled so far
    int32_t slot;     // accumulator slot (requests of more than one piece), else -1
  };

  // Requests that fit in one piece are admitted at once (they hold device
  // memory only as a piece descriptor while their step is in flight, which
  // the step's piece cap accounts for).  A longer one needs a free
  // accumulator slot and room in the memory budget for the slot and at least
  // one piece beside everything already held and in flight; otherwise it
  // waits, and the ones behind it keep their order.
  void admit(int64_t inflight_bytes) {
    for (auto it = pending_.begin(); it != pending_.end();) {
      if (it->n <= cfg_.piece_terms) {
        active_.push_back(*it);
        it = pending_.erase(it);
      } else if (!free_slots_.empty() &&
                 (budget_ == kNoBudget || held_ + kSlotBytes + kPieceBytes + inflight_bytes <= budget_)) {
        it->slot = free_slots_.back();
        free_slots_.pop_back();
        held_ += kSlotBytes;
        active_.push_back(*it);
        it = pending_.erase(it);
      } else {
        ++it;
      }
    }
  }

  void add(Req &r, int64_t len, std::vector<PlannedPiece> &out) {
    out.push_back(PlannedPiece{r.id, r.next, len, r.slot, kNotFinal});
    r.next += len;
    r.pieces += 1;
  }

  exsum_server_config cfg_;
  int64_t budget_;         // bytes of slots and in-flight piece descriptors allowed
  int64_t held_ = 0;       // bytes of the slots held by admitted requests
  std::list<Req> pending_;
  std::list<Req> active_;
  std::vector<int32_t> free_slots_;
};

}  // namespace

// ---- server ---------------------------------------------------------------

struct ServerImpl {
  struct Step {
    hipEvent_t ev = nullptr;
    Piece *host = nullptr;   // pinned
    Piece *dev = nullptr;
    int64_t npieces = 0;
    std::vector<std::pair<int64_t, int32_t>> finals;
  };
  struct ReqInfo {
    const double *x;
    double *out;
  };

  explicit ServerImpl(const exsum_server_config &c) : cfg(c), sched(c) {}

  exsum_server_config cfg;
  Scheduler sched;
  hipStream_t stream = nullptr;
  int device = 0;
  int grid_cap = 256;
  GlobalAcc *slots = nullptr;
  Piece *dev_tables = nullptr;
  std::vector<Step> ring;
  int head = 0, tail = 0, inflight = 0;
  int64_t inflight_pieces = 0;       // pieces of the steps queued on the stream
  std::unordered_map<int64_t, ReqInfo> reqs;
  std::deque<int64_t> done;
  int64_t next_id = 0;
  std::vector<PlannedPiece> plan;
  std::vector<std::pair<int64_t, int32_t>> finals;

  void free_all() {
    for (auto &st : ring) {
      if (st.ev) (void)hipEventDestroy(st.ev);
      if (st.host) (void)hipHostFree(st.host);
    }
    ring.clear();
    if (dev_tables) (void)hipFree(dev_tables);
    if (slots) (void)hipFree(slots);
    dev_tables = nullptr;
    slots = nullptr;
  }

  int init(hipStream_t s) {
    stream = s;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return status_of(e);
    grid_cap = cu_count(device);
    const size_t slot_bytes = global_acc_bytes() * (size_t)cfg.max_slots;
    e = hipMalloc(&slots, slot_bytes);
    if (e == hipSuccess) e = hipMemset(slots, 0, slot_bytes);
    const size_t table = sizeof(Piece) * (size_t)cfg.max_pieces;
    if (e == hipSuccess) e = hipMalloc(&dev_tables, table * (size_t)cfg.max_inflight);
    ring.resize(cfg.max_inflight);
    for (int i = 0; i < cfg.max_inflight && e == hipSuccess; i++) {
      e = hipHostMalloc(&ring[i].host, table, hipHostMallocDefault);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ring[i].ev, hipEventDisableTiming);
      ring[i].dev = dev_tables + (size_t)i * cfg.max_pieces;
    }
    if (e != hipSuccess) {
      const int st = status_of(e);
      free_all();
      return st;
    }
    return EXSUM_OK;
  }

  int submit(const double *x, int64_t n, double *out, int64_t *id) {
    if (n < 0 || n >= kMaxTerms || out == nullptr || (n > 0 && x == nullptr)) return EXSUM_EINVAL;
    const int64_t i = next_id++;
    reqs[i] = ReqInfo{x, out};
    sched.submit(i, n);
    if (id) *id = i;
    return EXSUM_OK;
  }

  // Retire completed steps, in stream order.
  int retire() {
    while (inflight > 0) {
      Step &st = ring[tail];
      const hipError_t e = hipEventQuery(st.ev);
      if (e == hipErrorNotReady) {
        (void)hipGetLastError();
        break;
      }
      if (e != hipSuccess) return status_of(e);
      for (auto &f : st.finals) {
        sched.release_slot(f.second);
        reqs.erase(f.first);
        done.push_back(f.first);
      }
      st.finals.clear();
      inflight_pieces -= st.npieces;
      st.npieces = 0;
      tail = (tail + 1) % (int)ring.size();
      inflight--;
    }
    return EXSUM_OK;
  }

  int step(int64_t *launched) {
    if (launched) *launched = 0;
    int st = retire();
    if (st != EXSUM_OK) return st;
    if (inflight == (int)ring.size() || sched.idle()) return EXSUM_OK;
    sched.plan(plan, finals, inflight_pieces * kPieceBytes);
    if (plan.empty()) return EXSUM_OK;
    Step &s = ring[head];
    // short pieces first, then long ones
    int n = 0;
    for (int pass = 0; pass < 2; pass++) {
      for (const auto &p : plan) {
        const bool is_short = p.len <= cfg.short_max;
        if (is_short != (pass == 0)) continue;
        const ReqInfo &r = reqs[p.id];
        s.host[n++] = Piece{r.x + p.off, p.len, r.out, p.slot < 0 ? 0 : p.slot, p.expected};
      }
    }
    int nshort = 0;
    for (const auto &p : plan) nshort += (p.len <= cfg.short_max) ? 1 : 0;
    const int nlong = n - nshort;
    const int per_wg = pieces_block() / 64;
    const int want = std::max(nlong, (nshort + per_wg - 1) / per_wg);
    const int grid = std::max(1, std::min(want, grid_cap));
    (void)hipGetLastError();
    // a few pieces travel in the kernel arguments; more go through the
    // device copy of the step's table
    hipError_t e = hipSuccess;
    if (n > kInlinePieces)
      e = hipMemcpyAsync(s.dev, s.host, sizeof(Piece) * (size_t)n, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_pieces(s.dev, s.host, nshort, n, slots, stream, grid, cfg.precombine);
    if (e == hipSuccess) e = hipEventRecord(s.ev, stream);
    if (e != hipSuccess) return status_of(e);
    s.finals = finals;
    s.npieces = n;
    inflight_pieces += n;
    head = (head + 1) % (int)ring.size();
    inflight++;
    if (launched) *launched = n;
    return EXSUM_OK;
  }

  int drain() {
    while (true) {
      int64_t launched = 0;
      int st = step(&launched);
      if (st != EXSUM_OK) return st;
      if (sched.idle() && inflight == 0) return EXSUM_OK;
      if (launched == 0 && inflight > 0) {
        const hipError_t e = hipEventSynchronize(ring[tail].ev);
        if (e != hipSuccess) return status_of(e);
      }
    }
  }
};

}  // namespace exsum

struct exsum_server {
  exsum::ServerImpl impl;
  explicit exsum_server(const exsum_server_config &c) : impl(c) {}
};

using namespace exsum;

namespace {

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool trace_ok(const double *pool, const int64_t *starts, const int64_t *lens, const double *arrival_s, int64_t nreq,
              const double *out, const double *latency_s) {
  if (nreq < 0) return false;
  if (nreq == 0) return true;
  if (!starts || !lens || !arrival_s || !out || !latency_s) return false;
  for (int64_t i = 0; i < nreq; i++) {
    if (lens[i] < 0 || lens[i] >= kMaxTerms || starts[i] < 0) return false;
    if (lens[i] > 0 && pool == nullptr) return false;
    if (i > 0 && arrival_s[i] < arrival_s[i - 1]) return false;
  }
  return true;
}

}  // namespace

extern "C" {

int exsum_server_default_config(exsum_server_config *cfg) {
  if (cfg == nullptr) return EXSUM_EINVAL;
  *cfg = default_server_config();
  return EXSUM_OK;
}

int exsum_server_create(const exsum_server_config *cfg, void *stream, exsum_server **out) {
  if (out == nullptr) return EXSUM_EINVAL;
  *out = nullptr;
  const exsum_server_config c = cfg ? *cfg : default_server_config();
  if (!server_config_ok(c)) return EXSUM_EINVAL;
  exsum_server *srv = new exsum_server(c);
  const int st = srv->impl.init(static_cast<hipStream_t>(stream));
  if (st != EXSUM_OK) {
    delete srv;
    return st;
  }
  *out = srv;
  return EXSUM_OK;
}

int exsum_server_destroy(exsum_server *srv) {
  if (srv == nullptr) return EXSUM_OK;
  const hipError_t e = hipStreamSynchronize(srv->impl.stream);
  srv->impl.free_all();
  delete srv;
  return status_of(e);
}

int exsum_server_submit(exsum_server *srv, const double *x, int64_t n, double *out, int64_t *id) {
  if (srv == nullptr) return EXSUM_EINVAL;
  return srv->impl.submit(x, n, out, id);
}

int exsum_server_step(exsum_server *srv, int64_t *launched) {
  if (srv == nullptr) return EXSUM_EINVAL;
  return srv->impl.step(launched);
}

int exsum_server_poll(exsum_server *srv, int64_t *ids, int64_t max, int64_t *count) {
  if (srv == nullptr || count == nullptr || max < 0 || (max > 0 && ids == nullptr)) return EXSUM_EINVAL;
  *count = 0;
  const int st = srv->impl.retire();
  if (st != EXSUM_OK) return st;
  auto &d = srv->impl.done;
  int64_t k = 0;
  while (k < max && !d.empty()) {
    ids[k++] = d.front();
    d.pop_front();
  }
  *count = k;
  return EXSUM_OK;
}

int exsum_server_drain(exsum_server *srv) {
  if (srv == nullptr) return EXSUM_EINVAL;
  return srv->impl.drain();
}

int exsum_server_pending(exsum_server *srv, int64_t *count) {
  if (srv == nullptr || count == nullptr) return EXSUM_EINVAL;
  *count = (int64_t)srv->impl.reqs.size();
  return EXSUM_OK;
}

int exsum_server_replay(exsum_server *srv, const double *pool, const int64_t *starts, const int64_t *lens,
                        const double *arrival_s, int64_t nreq, double *out, double *latency_s,
                        double *makespan_s) {
  if (srv == nullptr || makespan_s == nullptr) return EXSUM_EINVAL;
  if (!trace_ok(pool, starts, lens, arrival_s, nreq, out, latency_s)) return EXSUM_EINVAL;
  ServerImpl &S = srv->impl;
  if (!S.reqs.empty()) return EXSUM_EINVAL;          // the server must be idle
  std::unordered_map<int64_t, int64_t> index;        // request id -> trace position
  std::vector<int64_t> ids(1024);
  const auto t0 = std::chrono::steady_clock::now();
  int64_t next = 0, completed = 0;
  double last = 0.0;
  while (completed < nreq) {
    const double now = seconds_since(t0);
    while (next < nreq && arrival_s[next] <= now) {
      int64_t id = 0;
      const int st = S.submit(lens[next] > 0 ? pool + starts[next] : pool, lens[next], out + next, &id);
      if (st != EXSUM_OK) return st;
      index[id] = next++;
    }
    int64_t launched = 0;
    int st = S.step(&launched);
    if (st != EXSUM_OK) return st;
    int64_t cnt = 0;
    st = exsum_server_poll(srv, ids.data(), (int64_t)ids.size(), &cnt);
    if (st != EXSUM_OK) return st;
    if (cnt > 0) {
      const double t = seconds_since(t0);
      for (int64_t k = 0; k < cnt; k++) {
        auto it = index.find(ids[k]);
        if (it == index.end()) continue;
        latency_s[it->second] = t - arrival_s[it->second];
        index.erase(it);
        completed++;
      }
      last = t;
    }
  }
  *makespan_s = last;
  return EXSUM_OK;
}

int exsum_serial_replay(const double *pool, const int64_t *starts, const int64_t *lens, const double *arrival_s,
                        int64_t nreq, double *out, void *stream, double *latency_s, double *makespan_s) {
  if (makespan_s == nullptr) return EXSUM_EINVAL;
  if (!trace_ok(pool, starts, lens, arrival_s, nreq, out, latency_s)) return EXSUM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int R = 4096;
  std::vector<hipEvent_t> ev(R, nullptr);
  for (int i = 0; i < R; i++) {
    const hipError_t e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      for (int j = 0; j < i; j++) (void)hipEventDestroy(ev[j]);
      return status_of(e);
    }
  }
  int st = EXSUM_OK;
  const auto t0 = std::chrono::steady_clock::now();
  int64_t next = 0, oldest = 0;
  double last = 0.0;
  while (oldest < nreq && st == EXSUM_OK) {
    const double now = seconds_since(t0);
    while (next < nreq && arrival_s[next] <= now && next - oldest < R) {
      st = exsum_f64(lens[next] > 0 ? pool + starts[next] : pool, lens[next], out + next, stream);
      if (st != EXSUM_OK) break;
      const hipError_t e = hipEventRecord(ev[next % R], s);
      if (e != hipSuccess) {
        st = status_of(e);
        break;
      }
      next++;
    }
    while (oldest < next && st == EXSUM_OK) {
      const hipError_t e = hipEventQuery(ev[oldest % R]);
      if (e == hipErrorNotReady) {
        (void)hipGetLastError();
        break;
      }
      if (e != hipSuccess) {
        st = status_of(e);
        break;
      }
      last = seconds_since(t0);
      latency_s[oldest] = last - arrival_s[oldest];
      oldest++;
    }
  }
  if (st == EXSUM_OK) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = status_of(e);
  }
  for (int i = 0; i < R; i++) (void)hipEventDestroy(ev[i]);
  *makespan_s = last;
  return st;
}

int exsum_server_plan(const exsum_server_config *cfg, const int64_t *lens, int64_t nreq, int64_t cap,
                      int64_t *req, int64_t *off, int64_t *len, int64_t *step, int32_t *slot, uint32_t *expected,
                      int64_t *count) {
  if (count == nullptr || nreq < 0 || cap < 0 || (nreq > 0 && lens == nullptr)) return EXSUM_EINVAL;
  if (cap > 0 && (!req || !off || !len || !step || !slot || !expected)) return EXSUM_EINVAL;
  const exsum_server_config c = cfg ? *cfg : default_server_config();
  if (!server_config_ok(c)) return EXSUM_EINVAL;
  for (int64_t i = 0; i < nreq; i++)
    if (lens[i] < 0 || lens[i] >= kMaxTerms) return EXSUM_EINVAL;
  Scheduler sched(c);
  for (int64_t i = 0; i < nreq; i++) sched.submit(i, lens[i]);
  std::vector<PlannedPiece> plan;
  std::vector<std::pair<int64_t, int32_t>> finals;
  int64_t k = 0, s = 0;
  while (!sched.idle()) {
    sched.plan(plan, finals);
    if (plan.empty()) return EXSUM_EINVAL;            // cannot happen with a valid configuration
    for (const auto &p : plan) {
      if (k < cap) {
        req[k] = p.id;
        off[k] = p.off;
        len[k] = p.len;
        step[k] = s;
        slot[k] = p.slot;
        expected[k] = p.expected;
      }
      k++;
    }
    for (const auto &f : finals) sched.release_slot(f.second);
    s++;
  }
  *count = k;
  return EXSUM_OK;
}

}  // extern "C"
