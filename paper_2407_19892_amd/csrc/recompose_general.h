// Recomposition + top-k beyond the register-resident sweep: ranks above 128
// (the contraction streamed in K chunks) and k up to 64.  Kernels in
// recompose_general.hip; the host pipeline is in recompose.hip.
#pragma once

#include "recompose_sweep.h"

namespace gmgm_rc {

constexpr int KL_WAVES = 4;                  // waves per workgroup, 64 rows each
constexpr int KL_THREADS = 64 * KL_WAVES;

struct KloopArgs {
  const u32x4* Vp;          // repacked V (all n_vtiles tiles, `units` units each)
  const u32x4* Wp;          // repacked W (one tile per 32 local rows)
  float* cval;              // candidates: [slot][split][C]
  int* cidx;
  const int* row_list;      // list mode: local row -> global row (nullptr: contiguous)
  const int* row_count;
  int64_t n;
  int n_vtiles, n_wtiles, units;
  int64_t row0, row_begin, row_end;
  int S, tiles_per_split;
  const double* wnorm;      // ||W_i||, indexed by global row - w_lo
  const unsigned* vmax_bits;
  int64_t w_lo;
  double cprec;
  int k;
};

struct FinalGenArgs {
  const float* cval;
  const int* cidx;
  const float* V;
  const double* psi;
  const double* wnorm;
  const unsigned* vmax_bits;
  int64_t n;
  int r, k, C, S;
  int64_t row_begin, rows;
  int64_t w_lo;
  const int* row_list;
  const int* row_count;
  double cprec;
  int32_t* col_out;
  float* val_out;
  int* fail_list;
  int* fail_count;
  unsigned long long* counters;
};

void launch_sweep_kloop(int prec, int C, int64_t gx, int S, hipStream_t st, const KloopArgs& a);
void launch_finalize_gen(int64_t nrows, hipStream_t st, const FinalGenArgs& a);
void launch_exact_panel(const float* V, const double* psi, int64_t n, int r, const int* list, int q0, int pr,
                        double* P, hipStream_t st);
void launch_panel_topk(const double* P, int64_t n, const int* list, int q0, int pr, int k, int64_t row_begin,
                       int32_t* col_out, float* val_out, hipStream_t st);

}  // namespace gmgm_rc
