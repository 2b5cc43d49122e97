// FP64 smoother kernels: separable R = 0..12, doubly-symmetric square and disk
// support R = 1..6.
#include "eecmg_device.h"

namespace eecmg {

#define EECMG_SEP_CASE(R) \
  case R: return launch_policy<double, ConvSep<double, R>>(st, ll, descs, s);
#define EECMG_SEP_OP(R) \
  case R: return launch_op_conv<double, ConvSep<double, R>>(x, y, H, W, taps, R, s);
#define EECMG_SYM_CASE(R, D) \
  case R: return launch_policy<double, ConvSym<double, R, D>>(st, ll, descs, s);
#define EECMG_SYM_OP(R, D) \
  case R: return launch_op_conv<double, ConvSym<double, R, D>>(x, y, H, W, taps, R, s);

hipError_t sm_f64_sep(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  switch (R) {
    EECMG_SEP_CASE(0) EECMG_SEP_CASE(1) EECMG_SEP_CASE(2) EECMG_SEP_CASE(3) EECMG_SEP_CASE(4)
    EECMG_SEP_CASE(5) EECMG_SEP_CASE(6) EECMG_SEP_CASE(7) EECMG_SEP_CASE(8) EECMG_SEP_CASE(9)
    EECMG_SEP_CASE(10) EECMG_SEP_CASE(11) EECMG_SEP_CASE(12)
    default: return hipErrorInvalidValue;
  }
}

hipError_t opc_f64_sep(const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  switch (R) {
    EECMG_SEP_OP(0) EECMG_SEP_OP(1) EECMG_SEP_OP(2) EECMG_SEP_OP(3) EECMG_SEP_OP(4) EECMG_SEP_OP(5)
    EECMG_SEP_OP(6) EECMG_SEP_OP(7) EECMG_SEP_OP(8) EECMG_SEP_OP(9) EECMG_SEP_OP(10) EECMG_SEP_OP(11)
    EECMG_SEP_OP(12)
    default: return hipErrorInvalidValue;
  }
}

hipError_t sm_f64_sym(Stage st, bool disk, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  if (disk) {
    switch (R) {
      EECMG_SYM_CASE(1, true) EECMG_SYM_CASE(2, true) EECMG_SYM_CASE(3, true) EECMG_SYM_CASE(4, true)
      EECMG_SYM_CASE(5, true) EECMG_SYM_CASE(6, true)
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    EECMG_SYM_CASE(1, false) EECMG_SYM_CASE(2, false) EECMG_SYM_CASE(3, false) EECMG_SYM_CASE(4, false)
    EECMG_SYM_CASE(5, false) EECMG_SYM_CASE(6, false)
    default: return hipErrorInvalidValue;
  }
}

hipError_t opc_f64_sym(bool disk, const void* x, void* y, int H, int W, const void* taps, int R, hipStream_t s) {
  if (disk) {
    switch (R) {
      EECMG_SYM_OP(1, true) EECMG_SYM_OP(2, true) EECMG_SYM_OP(3, true) EECMG_SYM_OP(4, true)
      EECMG_SYM_OP(5, true) EECMG_SYM_OP(6, true)
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
