// Instantiations of the recomposition sweep in threshold mode (all precisions).
// Every precision uses two row tiles per wave (each lane owns a whole row), so
// that a row's candidates come out in ascending column order.
#include "recompose_sweep.h"

namespace gmgm_rc {

SweepFn pick_sweep_thr(int prec, int kpad) {
  if (prec == P_F32) {
    switch (kpad) {
      case 32: return sweep_kernel<P_F32, 4, 2, 16, true>;
      case 64: return sweep_kernel<P_F32, 8, 2, 16, true>;
      case 104: return sweep_kernel<P_F32, 13, 2, 16, true>;
      case 128: return sweep_kernel<P_F32, 16, 2, 16, true>;
    }
  } else if (prec == P_BF16) {
    switch (kpad) {
      case 32: return sweep_kernel<P_BF16, 2, 2, 16, true>;
      case 64: return sweep_kernel<P_BF16, 4, 2, 16, true>;
      case 112: return sweep_kernel<P_BF16, 7, 2, 16, true>;
      case 128: return sweep_kernel<P_BF16, 8, 2, 16, true>;
    }
  } else {
    switch (kpad) {
      case 64: return sweep_kernel<P_FP8, 2, 2, 16, true>;
      case 128: return sweep_kernel<P_FP8, 4, 2, 16, true>;
    }
  }
  return nullptr;
}

}  // namespace gmgm_rc
