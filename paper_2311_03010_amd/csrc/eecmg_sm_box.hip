// Smoother kernels with the uniform-disk blur policy (psf(a,b) = w on
// a^2 + b^2 <= R^2): FP32 for R = 1..8 (also on tall strips), FP64 for R = 1..6.
#include "eecmg_device.h"

namespace eecmg {

#define EECMG_BOX_CASE(T, R) \
  case R: return launch_policy<T, ConvBox<T, R>>(st, ll, descs, s);
#define EECMG_BOX_TALL(R) \
  case R: return launch_policy<float, ConvBox<float, R, true>>(st, ll, descs, s);
#define EECMG_BOX_OP(T, R) \
  case R: return launch_op_conv<T, ConvBox<T, R>>(x, y, H, W, taps, R, s);

hipError_t sm_box_short(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);

// sm: strip mode (0 usual, 1 tall, 2 short; tall and short FP32 only)
hipError_t sm_box(Stage st, bool f64, int R, int sm, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  if (sm == 2) return f64 ? hipErrorInvalidValue : sm_box_short(st, R, ll, descs, s);
  if (sm == 1) {
    if (f64) return hipErrorInvalidValue;
    switch (R) {
      EECMG_BOX_TALL(1) EECMG_BOX_TALL(2) EECMG_BOX_TALL(3) EECMG_BOX_TALL(4)
      EECMG_BOX_TALL(5) EECMG_BOX_TALL(6) EECMG_BOX_TALL(7) EECMG_BOX_TALL(8)
      default: return hipErrorInvalidValue;
    }
  }
  if (f64) {
    switch (R) {
      EECMG_BOX_CASE(double, 1) EECMG_BOX_CASE(double, 2) EECMG_BOX_CASE(double, 3)
      EECMG_BOX_CASE(double, 4) EECMG_BOX_CASE(double, 5) EECMG_BOX_CASE(double, 6)
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    EECMG_BOX_CASE(float, 1) EECMG_BOX_CASE(float, 2) EECMG_BOX_CASE(float, 3) EECMG_BOX_CASE(float, 4)
    EECMG_BOX_CASE(float, 5) EECMG_BOX_CASE(float, 6) EECMG_BOX_CASE(float, 7) EECMG_BOX_CASE(float, 8)
    default: return hipErrorInvalidValue;
  }
}

hipError_t opc_box(bool f64, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  if (f64) {
    switch (R) {
      EECMG_BOX_OP(double, 1) EECMG_BOX_OP(double, 2) EECMG_BOX_OP(double, 3)
      EECMG_BOX_OP(double, 4) EECMG_BOX_OP(double, 5) EECMG_BOX_OP(double, 6)
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    EECMG_BOX_OP(float, 1) EECMG_BOX_OP(float, 2) EECMG_BOX_OP(float, 3) EECMG_BOX_OP(float, 4)
    EECMG_BOX_OP(float, 5) EECMG_BOX_OP(float, 6) EECMG_BOX_OP(float, 7) EECMG_BOX_OP(float, 8)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace eecmg
