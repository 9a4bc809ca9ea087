// step_batch: many boxes of one method and precision advanced together.
#include <vector>

#include "runtime.hpp"

namespace {

template <class F>
int32_t guarded_batch(F &&f) {
  try {
    (void)hipGetLastError();  // clear a pending error of a call outside this library
    return f();
  } catch (const dhit::Error &e) {
    return e.code;
  } catch (...) {
    return DHIT_EINVAL;
  }
}

}  // namespace

extern "C" int32_t step_batch(dhit_box **boxes, int32_t nbox, int32_t nsteps) {
  return guarded_batch([&]() -> int32_t {
    if (!boxes || nbox <= 0 || nsteps < 0) throw dhit::Error(DHIT_EINVAL, "bad batch arguments");
    for (int32_t i = 0; i < nbox; ++i) {
      if (!boxes[i]) throw dhit::Error(DHIT_EINVAL, "null box in batch");
      if (boxes[i]->p.method != boxes[0]->p.method || boxes[i]->p.precision != boxes[0]->p.precision)
        throw dhit::Error(DHIT_EINVAL, "all boxes of a batch must share method and precision");
    }
    const bool lbe = boxes[0]->p.method != DHIT_DUGKS;
    for (int32_t s = 0; s < nsteps; ++s) {
      for (int32_t i = 0; i < nbox; ++i) {
        dhit_box &b = *boxes[i];
        double *slot = b.hist + (b.steps % dhit::kHistoryCap) * 5;
        if (lbe)
          dhit::launch_lbe_step(b, b.f[b.cur], b.f[1 - b.cur], slot);
        else
          dhit::launch_dugks_step(b, b.f[b.cur], b.f[1 - b.cur], slot);
        b.cur = 1 - b.cur;
        b.steps++;
      }
    }
    return DHIT_OK;
  });
}
