// Live per-kernel timing with HIP events on the launching stream.
//
// A few kernel classes (the finest-level red-black sweeps, the outer Arnoldi
// passes, the outer Stokes stencil) sample every stride-th launch: the sampled
// launch goes through hipExtLaunchKernelGGL with a start and a stop event,
// which the runtime stamps with the kernel's own start and end (the same
// interval a kernel trace reports), and its algorithmic bytes are
// accumulated.  The "vcycle" class times whole V-cycles instead, with events
// recorded on the stream before the first and after the last of their kernels.
// Disabled timers cost one branch per launch.
#include <cstring>
#include <vector>

#include "ibr.h"
#include "kernels.h"

namespace ibr {

namespace {

struct TimerState {
  int stride = 0;        // 0 = off; otherwise every stride-th launch is timed
  long seen = 0;         // launches of the class since enabling
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  double bytes = 0.0;
  long launches = 0;     // timed launches
};

TimerState g_timers[kTimerCount];

const char* const kTimerNames[kTimerCount] = {"rb_fine", "ortho_dot",    "ortho_axpy",    "stokes_apply",
                                              "vcycle",  "wall_rb_fine", "rb_red_prolong"};

int timer_index(const char* name) {
  if (!name) return -1;
  for (int i = 0; i < kTimerCount; ++i)
    if (std::strcmp(name, kTimerNames[i]) == 0) return i;
  return -1;
}

hipEvent_t next_event(TimerState& t) {
  if (t.used == t.pool.size()) {
    hipEvent_t e = nullptr;
    // timing only: no system-scope fence when the event is recorded (the
    // fence's cache write-back would lengthen the timed interval and slow the
    // kernels after it); the readout follows a device synchronisation
    if (hipEventCreateWithFlags(&e, hipEventDefault | hipEventDisableSystemFence) != hipSuccess) return nullptr;
    t.pool.push_back(e);
  }
  return t.pool[t.used++];
}

}  // namespace

TimerEvents timer_sample(int id, double bytes) {
  TimerEvents ev;
  if (id < 0 || id >= kTimerCount) return ev;
  TimerState& t = g_timers[id];
  if (t.stride <= 0) return ev;
  if ((t.seen++ % t.stride) != 0) return ev;
  ev.start = next_event(t);
  ev.stop = next_event(t);
  if (!ev.start || !ev.stop) return TimerEvents();
  t.bytes += bytes;
  t.launches += 1;
  return ev;
}

bool timers_any() {
  for (int i = 0; i < kTimerCount; ++i)
    if (g_timers[i].stride > 0) return true;
  return false;
}

}  // namespace ibr

extern "C" {

int ibr_timer_enable(const char* kernel, int stride) {
  const int i = ibr::timer_index(kernel);
  if (i < 0 || stride < 0) return IBR_EINVAL;
  ibr::TimerState& t = ibr::g_timers[i];
  t.stride = stride;
  t.seen = 0;
  t.used = 0;
  t.bytes = 0.0;
  t.launches = 0;
  return IBR_OK;
}

int ibr_timer_read(const char* kernel, double* ms, long* launches, double* bytes) {
  const int i = ibr::timer_index(kernel);
  if (i < 0) return IBR_EINVAL;
  ibr::TimerState& t = ibr::g_timers[i];
  double tot = 0.0;
  for (size_t k = 0; k + 1 < t.used; k += 2) {
    if (hipEventSynchronize(t.pool[k + 1]) != hipSuccess) return IBR_EDEVICE;
    float e = 0.0f;
    if (hipEventElapsedTime(&e, t.pool[k], t.pool[k + 1]) != hipSuccess) return IBR_EDEVICE;
    tot += e;
  }
  if (ms) *ms = tot;
  if (launches) *launches = t.launches;
  if (bytes) *bytes = t.bytes;
  return IBR_OK;
}

}  // extern "C"
