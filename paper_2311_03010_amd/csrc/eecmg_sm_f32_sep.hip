// FP32 smoother kernels with the rank-one (separable) blur policy, R = 0..12,
// on short and on tall strips.
#include "eecmg_device.h"

namespace eecmg {

#define EECMG_SEP_CASE(R) \
  case R: return launch_policy<float, ConvSep<float, R>>(st, ll, descs, s);
#define EECMG_SEP_TALL(R) \
  case R: return launch_policy<float, ConvSep<float, R, true>>(st, ll, descs, s);
#define EECMG_SEP_OP(R) \
  case R: return launch_op_conv<float, ConvSep<float, R>>(x, y, H, W, taps, R, s);

hipError_t sm_f32_sep_short(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);

// sm: strip mode (0 usual, 1 tall, 2 short)
hipError_t sm_f32_sep(Stage st, int R, int sm, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  if (sm == 2) return sm_f32_sep_short(st, R, ll, descs, s);
  if (sm == 1) {
    switch (R) {
      EECMG_SEP_TALL(0) EECMG_SEP_TALL(1) EECMG_SEP_TALL(2) EECMG_SEP_TALL(3) EECMG_SEP_TALL(4)
      EECMG_SEP_TALL(5) EECMG_SEP_TALL(6) EECMG_SEP_TALL(7) EECMG_SEP_TALL(8) EECMG_SEP_TALL(9)
      EECMG_SEP_TALL(10) EECMG_SEP_TALL(11) EECMG_SEP_TALL(12)
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    EECMG_SEP_CASE(0) EECMG_SEP_CASE(1) EECMG_SEP_CASE(2) EECMG_SEP_CASE(3) EECMG_SEP_CASE(4)
    EECMG_SEP_CASE(5) EECMG_SEP_CASE(6) EECMG_SEP_CASE(7) EECMG_SEP_CASE(8) EECMG_SEP_CASE(9)
    EECMG_SEP_CASE(10) EECMG_SEP_CASE(11) EECMG_SEP_CASE(12)
    default: return hipErrorInvalidValue;
  }
}

hipError_t opc_f32_sep(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  switch (R) {
    EECMG_SEP_OP(0) EECMG_SEP_OP(1) EECMG_SEP_OP(2) EECMG_SEP_OP(3) EECMG_SEP_OP(4) EECMG_SEP_OP(5)
    EECMG_SEP_OP(6) EECMG_SEP_OP(7) EECMG_SEP_OP(8) EECMG_SEP_OP(9) EECMG_SEP_OP(10) EECMG_SEP_OP(11)
    EECMG_SEP_OP(12)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace eecmg
