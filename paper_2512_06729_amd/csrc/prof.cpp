// Event-based launch timing for the benchmark and tuning: HIP events are
// recorded on the launching stream around each profiled launch, and
// xod_profile_read() sums their elapsed times.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "xod_internal.h"

namespace xod {
namespace {

struct Pair {
  hipEvent_t a, b;
};
struct Prof {
  std::mutex mu;
  std::vector<hipEvent_t> pool;
  std::vector<Pair> rec[kProfNum];
  hipEvent_t pending[kProfNum] = {};
};
Prof &prof() {
  static Prof p;
  return p;
}
hipEvent_t get_event(Prof &p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
const char *kNames[kProfNum] = {"panel", "update", "prologue", "solve", "jacobian", "rates",
                                "rhs", "gemm", "photolysis"};

}  // namespace

void prof_begin(int kind, hipStream_t s) {
  Prof &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t e = get_event(p);
  (void)hipEventRecord(e, s);
  p.pending[kind] = e;
}

void prof_end(int kind, hipStream_t s) {
  Prof &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t e = get_event(p);
  (void)hipEventRecord(e, s);
  p.rec[kind].push_back({p.pending[kind], e});
  p.pending[kind] = nullptr;
}

}  // namespace xod

using namespace xod;

extern "C" xod_status xod_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
  if (!kernel || !total_ms || !launches) {
    set_error("xod_profile_read: null argument");
    return XOD_EINVAL;
  }
  int kind = -1;
  for (int i = 0; i < kProfNum; ++i)
    if (std::strcmp(kernel, kNames[i]) == 0) kind = i;
  if (kind < 0) {
    set_error(std::string("xod_profile_read: unknown kernel ") + kernel);
    return XOD_EINVAL;
  }
  Prof &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  double sum = 0.0;
  for (auto &pr : p.rec[kind]) {
    XOD_HIP(hipEventSynchronize(pr.b));
    float ms = 0.f;
    XOD_HIP(hipEventElapsedTime(&ms, pr.a, pr.b));
    sum += ms;
  }
  *total_ms = sum;
  *launches = (int64_t)p.rec[kind].size();
  return XOD_OK;
}

extern "C" xod_status xod_profile_reset(void) {
  Prof &p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  for (int i = 0; i < kProfNum; ++i) {
    for (auto &pr : p.rec[i]) {
      (void)hipEventSynchronize(pr.b);
      p.pool.push_back(pr.a);
      p.pool.push_back(pr.b);
    }
    p.rec[i].clear();
  }
  return XOD_OK;
}
