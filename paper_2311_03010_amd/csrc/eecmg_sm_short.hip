// FP32 smoother kernels on short strips (strip mode 2): the separable policy
// for R = 0..12, the doubly-symmetric one for square support R = 1..6 and disk
// support R = 1..8, the uniform-disk one for R = 1..8.  Mid-size levels whose
// usual strips would leave the chip with few waves take these.
#include "eecmg_device.h"

namespace eecmg {

#define EECMG_SEP_SHORT(R) \
  case R: return launch_policy<float, ConvSep<float, R, 2>>(st, ll, descs, s);
#define EECMG_SYM_SHORT(R, D) \
  case R: return launch_policy<float, ConvSym<float, R, D, 2>>(st, ll, descs, s);
#define EECMG_BOX_SHORT(R) \
  case R: return launch_policy<float, ConvBox<float, R, 2>>(st, ll, descs, s);

hipError_t sm_f32_sep_short(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  switch (R) {
    EECMG_SEP_SHORT(0) EECMG_SEP_SHORT(1) EECMG_SEP_SHORT(2) EECMG_SEP_SHORT(3) EECMG_SEP_SHORT(4)
    EECMG_SEP_SHORT(5) EECMG_SEP_SHORT(6) EECMG_SEP_SHORT(7) EECMG_SEP_SHORT(8) EECMG_SEP_SHORT(9)
    EECMG_SEP_SHORT(10) EECMG_SEP_SHORT(11) EECMG_SEP_SHORT(12)
    default: return hipErrorInvalidValue;
  }
}

hipError_t sm_f32_sym_short(Stage st, bool disk, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  if (disk) {
    switch (R) {
      EECMG_SYM_SHORT(1, true) EECMG_SYM_SHORT(2, true) EECMG_SYM_SHORT(3, true) EECMG_SYM_SHORT(4, true)
      EECMG_SYM_SHORT(5, true) EECMG_SYM_SHORT(6, true) EECMG_SYM_SHORT(7, true) EECMG_SYM_SHORT(8, true)
      default: return hipErrorInvalidValue;
    }
  }
  switch (R) {
    EECMG_SYM_SHORT(1, false) EECMG_SYM_SHORT(2, false) EECMG_SYM_SHORT(3, false) EECMG_SYM_SHORT(4, false)
    EECMG_SYM_SHORT(5, false) EECMG_SYM_SHORT(6, false)
    default: return hipErrorInvalidValue;
  }
}

hipError_t sm_box_short(Stage st, int R, const LaunchList& ll, const JobDesc* descs, hipStream_t s) {
  switch (R) {
    EECMG_BOX_SHORT(1) EECMG_BOX_SHORT(2) EECMG_BOX_SHORT(3) EECMG_BOX_SHORT(4)
    EECMG_BOX_SHORT(5) EECMG_BOX_SHORT(6) EECMG_BOX_SHORT(7) EECMG_BOX_SHORT(8)
    default: return hipErrorInvalidValue;
  }
}

}  // namespace eecmg
