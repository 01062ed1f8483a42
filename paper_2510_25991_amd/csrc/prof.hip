// Per-kernel-class timing with HIP events on the launching stream.
//
// When a class is enabled, each of its launches carries a start and a stop
// event: single-kernel launches attach them to the dispatch itself
// (hipExtLaunchKernelGGL), which adds no packets to the stream; launches that
// span several kernels record them around the sequence.  Elapsed times are
// collected lazily (when many pairs are pending and when the counters are
// read), together with the algorithmic work (flops or bytes) of the launch,
// and each launch's start and end relative to a reference event recorded
// when timing starts: launches of one class that overlap (on different
// streams) are then also measured by the union of their intervals.
#include <algorithm>
#include <mutex>
#include <utility>
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
  unsigned mask = 0;  // bit k: class k is timed
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  double ms[KK_COUNT] = {};
  long long n[KK_COUNT] = {};
  double work[KK_COUNT] = {};
  hipEvent_t ref = nullptr;  // recorded when timing starts
  std::vector<std::pair<float, float>> iv[KK_COUNT];  // launch intervals, ms after ref
};

Prof &prof() {
  static Prof p;
  return p;
}

thread_local ProfSpan t_open;

hipEvent_t take(Prof &p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Collects the elapsed times of the first `count` pending pairs (all by
// default) and returns their events to the pool.
void drain(Prof &p, size_t count = (size_t)-1) {
  count = std::min(count, p.pend.size());
  for (size_t j = 0; j < count; ++j) {
    Pending &q = p.pend[j];
    float ms = 0.f, t0 = 0.f, t1 = 0.f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      p.ms[q.kind] += ms;
      p.n[q.kind] += 1;
      p.work[q.kind] += q.work;
      if (p.ref && hipEventElapsedTime(&t0, p.ref, q.a) == hipSuccess &&
          hipEventElapsedTime(&t1, p.ref, q.b) == hipSuccess)
        p.iv[q.kind].push_back({t0, t1});
    }
    p.pool.push_back(q.a);
    p.pool.push_back(q.b);
  }
  p.pend.erase(p.pend.begin(), p.pend.begin() + count);
}

}  // namespace

ProfSpan prof_open(int kind) {
  Prof &p = prof();
  if (!(p.mask >> kind & 1u)) return {};
  std::lock_guard<std::mutex> g(p.mu);
  ProfSpan sp{take(p), take(p)};
  if (!sp.a || !sp.b) {
    if (sp.a) p.pool.push_back(sp.a);
    if (sp.b) p.pool.push_back(sp.b);
    return {};
  }
  return sp;
}

void prof_close(const ProfSpan &sp, int kind, double work) {
  if (!sp.a) return;
  Prof &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.pend.push_back({sp.a, sp.b, kind, work});
  // Launch schedules wait on the stop events of recent launches; only the
  // older half is recycled here, far older than any event still waited on.
  if (p.pend.size() > 4096) drain(p, 2048);
}

void prof_begin(int kind, hipStream_t s) {
  t_open = prof_open(kind);
  if (t_open.a) (void)hipEventRecord(t_open.a, s);
}

void prof_end(int kind, hipStream_t s, double work) {
  if (!t_open.a) return;
  (void)hipEventRecord(t_open.b, s);
  prof_close(t_open, kind, work);
  t_open = {};
}

}  // namespace ddst

extern "C" int ddst_profile_select(uint32_t kinds) {
  ddst::Prof &p = ddst::prof();
  std::lock_guard<std::mutex> g(p.mu);
  ddst::drain(p);
  if (kinds) {
    for (int k = 0; k < ddst::KK_COUNT; ++k) {
      p.ms[k] = 0;
      p.n[k] = 0;
      p.work[k] = 0;
      p.iv[k].clear();
    }
    if (!p.ref && hipEventCreateWithFlags(&p.ref, hipEventDisableSystemFence) != hipSuccess)
      p.ref = nullptr;
    // the common time origin of the launch intervals
    if (p.ref && hipEventRecord(p.ref, nullptr) != hipSuccess) return DDST_EHIP;
  }
  p.mask = kinds & ((1u << ddst::KK_COUNT) - 1);
  return DDST_OK;
}

extern "C" int ddst_profile_enable(int32_t on) {
  return ddst_profile_select(on ? (1u << ddst::KK_COUNT) - 1 : 0u);
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

extern "C" int ddst_profile_busy(int32_t kind, double *busy_ms) {
  if (kind < 0 || kind >= ddst::KK_COUNT || !busy_ms) return DDST_EINVAL;
  ddst::Prof &p = ddst::prof();
  std::lock_guard<std::mutex> g(p.mu);
  ddst::drain(p);
  std::vector<std::pair<float, float>> v = p.iv[kind];
  std::sort(v.begin(), v.end());
  double total = 0, end = -1e300, start = 0;
  bool open = false;
  for (const auto &x : v) {
    if (!open || x.first > end) {
      if (open) total += end - start;
      start = x.first;
      end = x.second;
      open = true;
    } else if (x.second > end) {
      end = x.second;
    }
  }
  if (open) total += end - start;
  *busy_ms = total;
  return DDST_OK;
}
