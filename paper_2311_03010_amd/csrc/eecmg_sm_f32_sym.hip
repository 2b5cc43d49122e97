// FP32 smoother kernels with the doubly-symmetric blur policy: square support
// R = 1..6, disk support R = 1..8, on short and on tall strips.
#include "eecmg_device.h"

namespace eecmg {

#define EECMG_SYM_CASE(R, D) \
  case R: return launch_policy<float, ConvSym<float, R, D>>(st, ll, descs, s);
#define EECMG_SYM_TALL(R, D) \
  case R: return launch_policy<float, ConvSym<float, R, D, true>>(st, ll, descs, s);
#define EECMG_SYM_OP(R, D) \
  case R: return launch_op_conv<float, ConvSym<float, R, D>>(x, y, H, W, taps, R, s);

hipError_t sm_f32_sym_short(Stage st, bool disk, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s);

// sm: strip mode (0 usual, 1 tall, 2 short)
hipError_t sm_f32_sym(Stage st, bool disk, int R, int sm, const LaunchList& ll, const JobDesc* descs,
                      hipStream_t s) {
  if (sm == 2) return sm_f32_sym_short(st, disk, R, ll, descs, s);
  const bool tall = sm == 1;
  if (tall && disk) {
    switch (R) {
      EECMG_SYM_TALL(1, true) EECMG_SYM_TALL(2, true) EECMG_SYM_TALL(3, true) EECMG_SYM_TALL(4, true)
      EECMG_SYM_TALL(5, true) EECMG_SYM_TALL(6, true) EECMG_SYM_TALL(7, true) EECMG_SYM_TALL(8, true)
      default: return hipErrorInvalidValue;
    }
  }
  if (tall) {
    switch (R) {
      EECMG_SYM_TALL(1, false) EECMG_SYM_TALL(2, false) EECMG_SYM_TALL(3, false) EECMG_SYM_TALL(4, false)
      EECMG_SYM_TALL(5, false) EECMG_SYM_TALL(6, false)
      default: return hipErrorInvalidValue;
    }
  }
  if (disk) {
    switch (R) {
      EECMG_SYM_CASE(1, true) EECMG_SYM_CASE(2, true) EECMG_SYM_CASE(3, true) EECMG_SYM_CASE(4, true)
      EECMG_SYM_CASE(5, true) EECMG_SYM_CASE(6, true) EECMG_SYM_CASE(7, true) EECMG_SYM_CASE(8, true)
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    EECMG_SYM_CASE(1, false) EECMG_SYM_CASE(2, false) EECMG_SYM_CASE(3, false) EECMG_SYM_CASE(4, false)
    EECMG_SYM_CASE(5, false) EECMG_SYM_CASE(6, false)
    default: return hipErrorInvalidValue;
  }
}

hipError_t opc_f32_sym(bool disk, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  if (disk) {
    switch (R) {
      EECMG_SYM_OP(1, true) EECMG_SYM_OP(2, true) EECMG_SYM_OP(3, true) EECMG_SYM_OP(4, true)
      EECMG_SYM_OP(5, true) EECMG_SYM_OP(6, true) EECMG_SYM_OP(7, true) EECMG_SYM_OP(8, true)
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    EECMG_SYM_OP(1, false) EECMG_SYM_OP(2, false) EECMG_SYM_OP(3, false) EECMG_SYM_OP(4, false)
    EECMG_SYM_OP(5, false) EECMG_SYM_OP(6, false)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace eecmg
