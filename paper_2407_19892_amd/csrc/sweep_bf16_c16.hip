// Instantiations of the recomposition sweep: bf16 operands, top-16 lists.
#include "recompose_sweep.h"

namespace gmgm_rc {

SweepFn pick_sweep_bf16_c16(int kpad) {
  switch (kpad) {
    case 32: return sweep_kernel<P_BF16, 2, ti_for(P_BF16, 16), 16>;
    case 64: return sweep_kernel<P_BF16, 4, ti_for(P_BF16, 16), 16>;
    case 112: return sweep_kernel<P_BF16, 7, ti_for(P_BF16, 16), 16>;
    case 128: return sweep_kernel<P_BF16, 8, ti_for(P_BF16, 16), 16>;
  }
  return nullptr;
}

}  // namespace gmgm_rc
