// Instantiations of the recomposition sweep: split BF16 operands (hi + lo,
// three MFMAs per K step), the re-sweep of rows a BF16 / FP8 sweep left
// uncertified.
#include "recompose_sweep.h"

namespace gmgm_rc {

SweepFn pick_sweep_bf16x3(int kpad, int C) {
  const int TI = ti_for(P_BF16X3, C);
  static_assert(ti_for(P_BF16X3, 16) == 1 && ti_for(P_BF16X3, 32) == 1, "half-row lists");
  (void)TI;
  if (C == 16) {
    switch (kpad) {
      case 32: return sweep_kernel<P_BF16X3, 4, 1, 16>;
      case 64: return sweep_kernel<P_BF16X3, 8, 1, 16>;
      case 112: return sweep_kernel<P_BF16X3, 14, 1, 16>;
      case 128: return sweep_kernel<P_BF16X3, 16, 1, 16>;
    }
  } else if (C == 32) {
    switch (kpad) {
      case 32: return sweep_kernel<P_BF16X3, 4, 1, 32>;
      case 64: return sweep_kernel<P_BF16X3, 8, 1, 32>;
      case 112: return sweep_kernel<P_BF16X3, 14, 1, 32>;
      case 128: return sweep_kernel<P_BF16X3, 16, 1, 32>;
    }
  }
  return nullptr;
}

}  // namespace gmgm_rc
