// Per-kernel event timing (see prof.h).
#include "prof.h"

#include <atomic>
#include <mutex>
#include <sstream>

namespace mfh {
namespace {

const char* const kNames[PK_COUNT] = {
    "gemm_kernel<double>",        "gemm_kernel<float>",
    "gemm_narrow_kernel<double>", "gemm_narrow_kernel<float>",
    "gemm_reduce_kernel<double>", "gemm_reduce_kernel<float>",
    "gemm_narrow_fold_kernel<double>", "gemm_narrow_fold_kernel<float>",
    "potrf_blk_kernel<double, 64>",   "potrf_blk_kernel<float, 64>",
    "potrf_kernel<double, 128, 512>", "potrf_blk_kernel<float, 128>",
    "skreg_kernel<double, 2, 16, true, 1024>", "skreg_kernel<float, 4, 16, true, 1024>",
    "skreg_kernel<double, 2, 8, false, 1024>", "skreg_kernel<float, 3, 24, false, 512>",
    "skelfac_kernel<double>",     "skelfac_kernel<float>",
    "phase2_kernel<double>",      "phase2_kernel<float>",
    "phase2_coop_kernel<double, true>", "phase2_coop_kernel<float, true>",
    "phase2_coop_kernel<double, false>", "phase2_coop_kernel<float, false>",
    "extadd_kernel<double>",      "extadd_kernel<float>",
    "gj_kernel<1, 16, 256>", "gj_kernel<2, 16, 512>", "gj_kernel<3, 16, 768>", "gj_wide_kernel",
    "spmv_kernel",
};

struct Rec {
  int kind;
  hipEvent_t a, b;
  double flops, bytes;
  int state;        // 0 waiting for a launch, 1 events taken by a launch, 2 recorded here, 3 dropped
};
thread_local int t_pending = -1;   // record whose events the next MFH_LAUNCH takes
thread_local bool t_suspended = false;

struct State {
  std::mutex mu;
  std::atomic<uint64_t> mask{0};
  int session = 0;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};
State& S() {
  static State s;
  return s;
}

constexpr int kIdxBits = 24;

hipEvent_t take(State& s) {
  if (!s.pool.empty()) {
    hipEvent_t e = s.pool.back();
    s.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

Rec* find(State& s, int id) {
  if (id < 0 || (id >> kIdxBits) != (s.session & 0x3F)) return nullptr;
  const size_t i = (size_t)(id & ((1 << kIdxBits) - 1));
  return i < s.recs.size() ? &s.recs[i] : nullptr;
}

}  // namespace

const char* prof_name(int kind) { return (kind >= 0 && kind < PK_COUNT) ? kNames[kind] : "?"; }

bool prof_selected(int kind) { return ((S().mask.load(std::memory_order_relaxed) >> kind) & 1) != 0; }
void prof_suspend(bool on) { t_suspended = on; }

int prof_begin(int kind, hipStream_t st, double flops, double bytes) {
  State& s = S();
  if (t_suspended || !((s.mask.load(std::memory_order_relaxed) >> kind) & 1)) return -1;
  std::lock_guard<std::mutex> g(s.mu);
  if (s.recs.size() >= (size_t(1) << kIdxBits)) return -1;
  Rec r{kind, take(s), take(s), flops, bytes, 0};
  (void)st;
  if (!r.a || !r.b) {
    if (r.a) s.pool.push_back(r.a);
    if (r.b) s.pool.push_back(r.b);
    return -1;
  }
  s.recs.push_back(r);
  t_pending = (int)(s.recs.size() - 1);
  return ((s.session & 0x3F) << kIdxBits) | t_pending;
}

bool prof_take(hipEvent_t* start, hipEvent_t* stop) {
  if (t_pending < 0) return false;
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  const int i = t_pending;
  t_pending = -1;
  if (i >= (int)s.recs.size() || s.recs[i].state != 0) return false;
  s.recs[i].state = 1;
  *start = s.recs[i].a;
  *stop = s.recs[i].b;
  return true;
}

void prof_stream_start(int id, hipStream_t st) {
  if (id < 0) return;
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  Rec* r = find(s, id);
  if (!r || r->state != 0) return;
  if ((int)(r - s.recs.data()) == t_pending) t_pending = -1;
  r->state = 2;
  (void)hipEventRecord(r->a, st);
}

void prof_end(int id, hipStream_t st) {
  if (id < 0) return;
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  Rec* r = find(s, id);
  if (!r) return;
  if ((int)(r - s.recs.data()) == t_pending) t_pending = -1;
  if (r->state == 2) (void)hipEventRecord(r->b, st);
  else if (r->state == 0) r->state = 3;   // nothing was launched
}

void prof_add(int id, double flops, double bytes) {
  if (id < 0) return;
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  if (Rec* r = find(s, id)) {
    r->flops += flops;
    r->bytes += bytes;
  }
}

void prof_start(const std::string& names) {
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  uint64_t m = 0;
  if (names.empty()) {
    m = (uint64_t(1) << PK_COUNT) - 1;
  } else {
    std::stringstream ss(names);
    std::string tok;
    while (std::getline(ss, tok, ';'))
      for (int k = 0; k < PK_COUNT; ++k)
        if (tok == kNames[k]) m |= uint64_t(1) << k;
  }
  for (Rec& r : s.recs) {
    s.pool.push_back(r.a);
    s.pool.push_back(r.b);
  }
  s.recs.clear();
  t_pending = -1;
  ++s.session;
  s.mask.store(m);
}

std::vector<ProfTotal> prof_stop() {
  State& s = S();
  std::lock_guard<std::mutex> g(s.mu);
  s.mask.store(0);
  std::vector<ProfTotal> t(PK_COUNT);
  for (int k = 0; k < PK_COUNT; ++k) t[k] = ProfTotal{k, 0, 0.0, 0.0, 0.0};
  for (Rec& r : s.recs) {
    float ms = 0.f;
    double sec = -1.0;
    if ((r.state == 1 || r.state == 2) && hipEventSynchronize(r.b) == hipSuccess &&
        hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      sec = 1e-3 * ms;
    }
    if (sec >= 0.0) {
      ProfTotal& x = t[r.kind];
      x.launches += 1;
      x.seconds += sec;
      x.flops += r.flops;
      x.bytes += r.bytes;
    }
    s.pool.push_back(r.a);
    s.pool.push_back(r.b);
  }
  s.recs.clear();
  ++s.session;
  std::vector<ProfTotal> out;
  for (auto& x : t)
    if (x.launches > 0) out.push_back(x);
  return out;
}

}  // namespace mfh
