// Optional timing of one kernel launch with HIP events attached to the
// dispatch itself (hipExtLaunchKernelGGL).  The API arms a pair for the next
// launch made on this thread; the first launch through HOPU_LAUNCH takes it.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

namespace hopu {
struct LaunchEvents {
  hipEvent_t start, stop;
};
LaunchEvents* take_launch_events();
void arm_launch_events(hipEvent_t start, hipEvent_t stop);
void disarm_launch_events();
}  // namespace hopu

#define HOPU_LAUNCH(K, G, B, SH, S, ...)                                               \
  do {                                                                                 \
    ::hopu::LaunchEvents* ev_ = ::hopu::take_launch_events();                          \
    if (ev_) hipExtLaunchKernelGGL(K, G, B, SH, S, ev_->start, ev_->stop, 0, __VA_ARGS__); \
    else hipLaunchKernelGGL(K, G, B, SH, S, __VA_ARGS__);                              \
  } while (0)
