// Per-kernel timing with HIP events recorded on the box's stream.
#include <string>

#include "runtime.hpp"

namespace dhit {

TimedLaunch::TimedLaunch(dhit_box &box, int kind) : b(box) {
  KernelTimer *t = b.timer;
  if (!t || !t->enabled) return;
  slot = (int)(t->count % KernelTimer::kCap);
  t->kind[slot] = kind;
  DHIT_HIP(hipEventRecord(t->start[slot], b.stream));
}

void TimedLaunch::done() {
  if (slot < 0) return;
  KernelTimer *t = b.timer;
  DHIT_HIP(hipEventRecord(t->stop[slot], b.stream));
  t->count++;
}

}  // namespace dhit

namespace {

int32_t timer_error(const dhit::Error &e) {
  dhit::set_last_error(e.what());
  return e.code;
}

void destroy_events(dhit::KernelTimer *t) {
  if (!t->created) return;
  for (int i = 0; i < dhit::KernelTimer::kCap; ++i) {
    (void)hipEventDestroy(t->start[i]);
    (void)hipEventDestroy(t->stop[i]);
  }
  t->created = false;
}

}  // namespace

namespace dhit {

void timer_free(dhit_box &b) {
  if (!b.timer) return;
  destroy_events(b.timer);
  delete b.timer;
  b.timer = nullptr;
}

}  // namespace dhit

extern "C" int32_t set_kernel_timing(dhit_box *b, int32_t enable) {
  try {
    (void)hipGetLastError();
    if (!b) return DHIT_EINVAL;
    DHIT_HIP(hipStreamSynchronize(b->stream));
    if (!b->timer) b->timer = new dhit::KernelTimer();
    dhit::KernelTimer *t = b->timer;
    if (enable && !t->created) {
      for (int i = 0; i < dhit::KernelTimer::kCap; ++i) {
        DHIT_HIP(hipEventCreate(&t->start[i]));
        DHIT_HIP(hipEventCreate(&t->stop[i]));
      }
      t->created = true;
    }
    t->enabled = enable != 0;
    t->count = 0;
    return DHIT_OK;
  } catch (const dhit::Error &e) {
    return timer_error(e);
  } catch (...) {
    return DHIT_ENOMEM;
  }
}

extern "C" int32_t read_kernel_timings(dhit_box *b, double *ms, int64_t *launches) {
  try {
    (void)hipGetLastError();
    if (!b || !ms || !launches) return DHIT_EINVAL;
    for (int k = 0; k < DHIT_NKERNEL; ++k) {
      ms[k] = 0.0;
      launches[k] = 0;
    }
    dhit::KernelTimer *t = b->timer;
    if (!t || !t->created) return DHIT_OK;
    DHIT_HIP(hipStreamSynchronize(b->stream));
    const int64_t kept = t->count < dhit::KernelTimer::kCap ? t->count : dhit::KernelTimer::kCap;
    for (int64_t i = 0; i < kept; ++i) {
      const int slot = (int)((t->count - kept + i) % dhit::KernelTimer::kCap);
      float e = 0.f;
      DHIT_HIP(hipEventElapsedTime(&e, t->start[slot], t->stop[slot]));
      ms[t->kind[slot]] += e;
      launches[t->kind[slot]] += 1;
    }
    t->count = 0;
    return DHIT_OK;
  } catch (const dhit::Error &e) {
    return timer_error(e);
  }
}
