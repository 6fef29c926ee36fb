// Instantiations of the recomposition sweep: fp8 operands, top-32 lists.
#include "recompose_sweep.h"

namespace gmgm_rc {

SweepFn pick_sweep_fp8_c32(int kpad) {
  switch (kpad) {
    case 64: return sweep_kernel<P_FP8, 2, ti_for(P_FP8, 32), 32>;
    case 128: return sweep_kernel<P_FP8, 4, ti_for(P_FP8, 32), 32>;
  }
  return nullptr;
}

}  // namespace gmgm_rc
