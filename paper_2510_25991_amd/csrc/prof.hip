// Per-kernel-class timing with HIP events on the launching stream.
//
// When enabled, every launch of an instrumented kernel class is bracketed by
// two events recorded on its own stream; elapsed times are collected lazily
// (when many pairs are pending and when the counters are read), together
// with the algorithmic work (flops or bytes) the launch performs.
#include <mutex>
#include <vector>

#include "internal.h"

namespace ddst {
namespace {

struct Pending {
  hipEvent_t a, b;
  int kind;
  double work;
};

struct Prof {
  std::mutex mu;
  bool on = false;
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  double ms[KK_COUNT] = {};
  long long n[KK_COUNT] = {};
  double work[KK_COUNT] = {};
};

Prof &prof() {
  static Prof p;
  return p;
}

thread_local hipEvent_t t_open = nullptr;

hipEvent_t take(Prof &p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain(Prof &p) {
  for (Pending &q : p.pend) {
    float ms = 0.f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      p.ms[q.kind] += ms;
      p.n[q.kind] += 1;
      p.work[q.kind] += q.work;
    }
    p.pool.push_back(q.a);
    p.pool.push_back(q.b);
  }
  p.pend.clear();
}

}  // namespace

bool prof_on() { return prof().on; }

void prof_begin(int kind, hipStream_t s) {
  (void)kind;
  Prof &p = prof();
  if (!p.on) return;
  std::lock_guard<std::mutex> g(p.mu);
  t_open = take(p);
  if (t_open) (void)hipEventRecord(t_open, s);
}

void prof_end(int kind, hipStream_t s, double work) {
  Prof &p = prof();
  if (!p.on || !t_open) return;
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t b = take(p);
  if (!b) return;
  (void)hipEventRecord(b, s);
  p.pend.push_back({t_open, b, kind, work});
  t_open = nullptr;
  if (p.pend.size() > 4096) drain(p);
}

}  // namespace ddst

extern "C" int ddst_profile_enable(int32_t on) {
  ddst::Prof &p = ddst::prof();
  std::lock_guard<std::mutex> g(p.mu);
  ddst::drain(p);
  if (on) {
    for (int k = 0; k < ddst::KK_COUNT; ++k) {
      p.ms[k] = 0;
      p.n[k] = 0;
      p.work[k] = 0;
    }
  }
  p.on = on != 0;
  return DDST_OK;
}

extern "C" int ddst_profile_read(int32_t kind, int64_t *launches, double *total_ms,
                                 double *work) {
  if (kind < 0 || kind >= ddst::KK_COUNT) return DDST_EINVAL;
  ddst::Prof &p = ddst::prof();
  std::lock_guard<std::mutex> g(p.mu);
  ddst::drain(p);
  if (launches) *launches = p.n[kind];
  if (total_ms) *total_ms = p.ms[kind];
  if (work) *work = p.work[kind];
  return DDST_OK;
}
