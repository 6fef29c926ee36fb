// Instantiations of the recomposition sweep: f32 operands, top-32 lists.
#include "recompose_sweep.h"

namespace gmgm_rc {

SweepFn pick_sweep_f32_c32(int kpad) {
  switch (kpad) {
    case 32: return sweep_kernel<P_F32, 4, ti_for(P_F32, 32), 32>;
    case 64: return sweep_kernel<P_F32, 8, ti_for(P_F32, 32), 32>;
    case 104: return sweep_kernel<P_F32, 13, ti_for(P_F32, 32), 32>;
    case 128: return sweep_kernel<P_F32, 16, ti_for(P_F32, 32), 32>;
  }
  return nullptr;
}

}  // namespace gmgm_rc
