// Optional per-kernel timing: when enabled, instrumented launch sites record
// a pair of HIP events on their own stream around the kernel; the totals are
// read back (synchronising on the events) through tc_timing_read.  Disabled
// by default: no events are created or recorded then.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tc_internal.h"

namespace tc {

namespace {
struct Registry {
  std::mutex mu;
  bool on = false;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> ev;
};
Registry& reg() {
  static Registry r;
  return r;
}
}  // namespace

bool timing_on() { return reg().on; }

TimedLaunch::TimedLaunch(const char* name, hipStream_t st) : name_(name), st_(st) {
  if (!reg().on) return;
  if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
    a_ = b_ = nullptr;
    return;
  }
  if (hipEventRecord(a_, st_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
    a_ = b_ = nullptr;
  }
}

TimedLaunch::~TimedLaunch() {
  if (!a_) return;
  if (hipEventRecord(b_, st_) != hipSuccess) return;
  std::lock_guard<std::mutex> g(reg().mu);
  reg().ev[name_].emplace_back(a_, b_);
}

}  // namespace tc

extern "C" {

tc_status tc_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> g(tc::reg().mu);
  tc::reg().on = on != 0;
  return TC_OK;
}

tc_status tc_timing_reset(void) {
  std::lock_guard<std::mutex> g(tc::reg().mu);
  for (auto& kv : tc::reg().ev)
    for (auto& p : kv.second) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  tc::reg().ev.clear();
  return TC_OK;
}

tc_status tc_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return TC_E_ARG;
  std::lock_guard<std::mutex> g(tc::reg().mu);
  *total_ms = 0.0;
  *launches = 0;
  auto it = tc::reg().ev.find(kernel);
  if (it == tc::reg().ev.end()) return TC_OK;
  for (auto& p : it->second) {
    if (hipEventSynchronize(p.second) != hipSuccess) return TC_E_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess) return TC_E_HIP;
    *total_ms += ms;
    *launches += 1;
  }
  return TC_OK;
}

}  // extern "C"
