// mgr_timing.hpp -- optional per-kernel HIP-event timing (instrumentation).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

namespace mgr {

bool timing_enabled();

// While one lives on a thread, launches from that thread are not timed (no
// events are created or recorded).
class TimingOff {
 public:
  TimingOff();
  ~TimingOff();
  TimingOff(const TimingOff &) = delete;
  TimingOff &operator=(const TimingOff &) = delete;
};

// Brackets one kernel launch with HIP events on its stream when timing is
// enabled; `alg_bytes` is the launch's algorithmic traffic (bytes the method
// must move), accumulated per kernel name.
class TimedLaunch {
 public:
  TimedLaunch(hipStream_t s, const std::string &name, double alg_bytes);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch &) = delete;
  TimedLaunch &operator=(const TimedLaunch &) = delete;

 private:
  hipStream_t stream_;
  int slot_ = -1;
};

}  // namespace mgr
