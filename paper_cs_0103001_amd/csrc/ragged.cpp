// ragged.cpp -- ragged batches of square images of mixed power-of-two sizes.
#include "../../include/fftmi.h"
#include "plan.hpp"

namespace fftmi {
void destroy_ragged_state(fftmi_plan*) {}
}  // namespace fftmi

extern "C" {
int fft_plan_ragged(fft_plan_t* out, int64_t count, const int64_t* sizes, uint32_t flags) {
  (void)count;
  (void)sizes;
  (void)flags;
  if (out) *out = nullptr;
  return FFT_ERR_UNSUPPORTED;
}
int fft2d_filter_ragged(fft_plan_t p, const void*, void*, const fft_mask*, void*, void*) {
  if (!fftmi::plan_live(p)) return FFT_ERR_ARG;
  return FFT_ERR_UNSUPPORTED;
}
}
