// Smoother kernels with the general (any PSF) blur policy, FP32 and FP64, for
// radius classes R <= 3, 6 and 12 (radius passed at run time), and on short
// tiles for R <= 3 (small levels).
#include "eecmg_device.h"

namespace eecmg {

template <typename T>
static hipError_t gen_t(Stage st, int rclass, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  if (rclass <= 3) return launch_policy<T, ConvGeneral<T, 3>>(st, ll, descs, s);
  if (rclass <= 6) return launch_policy<T, ConvGeneral<T, 6>>(st, ll, descs, s);
  return launch_policy<T, ConvGeneral<T, 12>>(st, ll, descs, s);
}

template <typename T>
static hipError_t gen_short_t(Stage st, int rclass, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  if (rclass <= 3) return launch_policy<T, ConvGeneral<T, 3, kTHShort>>(st, ll, descs, s);
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t gen_op_t(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  if (R <= 3) return launch_op_conv<T, ConvGeneral<T, 3>>(x, y, H, W, taps, R, s);
  if (R <= 6) return launch_op_conv<T, ConvGeneral<T, 6>>(x, y, H, W, taps, R, s);
  return launch_op_conv<T, ConvGeneral<T, 12>>(x, y, H, W, taps, R, s);
}

hipError_t sm_gen(Stage st, bool f64, int rclass, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  return f64 ? gen_t<double>(st, rclass, ll, descs, s) : gen_t<float>(st, rclass, ll, descs, s);
}

hipError_t sm_gen_short(Stage st, bool f64, int rclass, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  return f64 ? gen_short_t<double>(st, rclass, ll, descs, s) : gen_short_t<float>(st, rclass, ll, descs, s);
}

hipError_t opc_gen(bool f64, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  return f64 ? gen_op_t<double>(x, y, H, W, taps, R, s) : gen_op_t<float>(x, y, H, W, taps, R, s);
}

}  // namespace eecmg
