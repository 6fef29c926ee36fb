// Instantiations of the recomposition sweep: bf16 operands, symmetric form,
// and the column-sample sweep that gives its per-row bounds.
#include "recompose_sweep.h"

namespace gmgm_rc {

template <int C, bool SYM, bool STRIDED>
static SweepFn pick_c(int kpad) {
  switch (kpad) {
    case 32: return sweep_kernel<P_BF16, 2, 2, C, false, SYM, STRIDED>;
    case 64: return sweep_kernel<P_BF16, 4, 2, C, false, SYM, STRIDED>;
    case 112: return sweep_kernel<P_BF16, 7, 2, C, false, SYM, STRIDED>;
    case 128: return sweep_kernel<P_BF16, 8, 2, C, false, SYM, STRIDED>;
  }
  return nullptr;
}

SweepFn pick_sweep_bf16_sym(int kpad, int C) {
  return C == 16 ? pick_c<16, true, false>(kpad) : pick_c<32, true, false>(kpad);
}

SweepFn pick_sweep_bf16_sample(int kpad, int C) {
  return C == 16 ? pick_c<16, false, true>(kpad) : pick_c<32, false, true>(kpad);
}

}  // namespace gmgm_rc
