// Optional timing of kernel launches with HIP events (host side).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <cstdint>

namespace rve {

// Kernel families whose launches can be timed (the numbering is part of the C ABI).
enum KernelFamily {
  KF_SLIP_FAST = 0,      // local Newton, first pass
  KF_SLIP_SLOW = 1,      // local Newton, continuation pass over the work list
  KF_STRESS_TANGENT = 2, // stress and consistent tangent
  KF_CG_PREP = 3,        // CG vector update, r.r and K : r
  KF_PLANE_FWD = 4,      // x and y forward transforms of one component plane
  KF_MID = 5,            // z transforms and the Green operator
  KF_PLANE_INV = 6,      // y and x inverse transforms and the CG epilogue
  KF_CG_GRAD = 7,        // gradient stencil of the factorised projection and the CG epilogue
  KF_PLANE_DIV = 8,      // divergence stencil and x and y forward transforms (factorised)
  KF_MID3 = 9,           // z transforms and 1 / |k|^2 on three components (factorised)
  KF_PLANE_W = 10,       // y and x inverse transforms of three components (factorised)
  KF_COUNT = 11
};

// Receives a mark before and after every launch of a family (the launch itself goes
// through launch()); units is what the launch covers (bytes or voxels).
struct LaunchTimer {
  virtual void begin(int family, hipStream_t st) = 0;
  virtual void end(int family, int64_t units, hipStream_t st) = 0;
  virtual ~LaunchTimer() = default;
};

// Events that the next launch through launch() on this thread records; set by the timer.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchEvents& pending_launch_events() {
  thread_local LaunchEvents e;
  return e;
}

// Kernel launch for the timed families: when events are pending on the calling thread, the
// dispatch itself records them at the kernel's start and end (AMD's extended launch), so
// that their difference is the kernel's own duration; otherwise an ordinary launch (which a
// stream capture records as a graph node).  Errors are left for hipGetLastError.
template <typename F, typename... Args>
inline void launch(F kernel, dim3 grid, dim3 block, uint32_t shared_bytes, hipStream_t st, Args... args) {
  LaunchEvents& ev = pending_launch_events();
  if (ev.start || ev.stop) {
    hipExtLaunchKernelGGL(kernel, grid, block, shared_bytes, st, ev.start, ev.stop, 0u, args...);
    ev = LaunchEvents{};
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shared_bytes, st, args...);
  }
}

// Brackets one launch: begin() in the constructor, end() in the destructor.
struct TimedLaunch {
  LaunchTimer* t;
  int family;
  int64_t units;
  hipStream_t st;
  TimedLaunch(LaunchTimer* t_, int f, int64_t u, hipStream_t s) : t(t_), family(f), units(u), st(s) {
    if (t) t->begin(family, st);
  }
  ~TimedLaunch() {
    if (t) t->end(family, units, st);
  }
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;
};

}  // namespace rve
