// Scoped HIP-event bracket around a kernel launch (active only when timing is on).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace jtfs {
bool timing_on();
// While an object of this type lives, launches of the calling thread record no
// stage events (for paths that must not create any).
struct TimingSuppressed {
    TimingSuppressed();
    ~TimingSuppressed();
};
class TimedLaunch {
  public:
    TimedLaunch(int stage, hipStream_t st);
    ~TimedLaunch();
  private:
    int stage_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};
}  // namespace jtfs

// Runs the statement (a kernel launch) between two events of `stage` on stream `st`.
#define JTFS_TIMED(stage, st, ...) do { ::jtfs::TimedLaunch tl_((stage), (st)); __VA_ARGS__; } while (0)
