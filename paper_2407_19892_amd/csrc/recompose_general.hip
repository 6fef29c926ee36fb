// Fused recomposition + per-row top-k for ranks beyond the register-resident
// sweep (r > 128) and for k up to 64 (Algorithm 1, final loop, over every
// axis: the gene axis is recomposed at its full rank; Computational
// complexity, O(sum_l r_l d_l^2)).
//
// Pipeline (host side in recompose.hip):
//   sweep_kloop   MFMA sweep with the contraction streamed in K chunks: each
//                 wave holds the accumulators of 64 rows x 128 columns and
//                 reads the W and V operand chunks from memory (L2-resident
//                 panels); every lane keeps a sorted top-C list of its own
//                 row (approximate |Psi|), as the register-resident sweep does
//   finalize_gen  one wave per row: exact FP64 rescoring of the candidates
//                 within the rounding band of the k-th, the certificate, CSR
//   exact_panel   rows no list could certify: exact FP64 values of the whole
//                 row block (FP64 FMA tiles through LDS), then top-k per row
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "recompose_general.h"

namespace gmgm_rc {

// ------------------------------------------------------------------ K-loop sweep
// Chunk of the contraction per step: 32 k (F32: 4 operand units of 8 k,
// BF16: 2 units of 16 k).
template <int PREC>
__host__ __device__ constexpr int kl_units() { return PREC == P_F32 ? 4 : 2; }

template <int C>
__device__ inline void kl_insert(float (&lv)[C], int (&li)[C], float v, int j) {
  bool g_hi = v > lv[C - 1];
#pragma unroll
  for (int s = C - 1; s > 0; --s) {
    const bool g_lo = v > lv[s - 1];
    const float nv = g_lo ? lv[s - 1] : (g_hi ? v : lv[s]);
    const int nj = g_lo ? li[s - 1] : (g_hi ? j : li[s]);
    lv[s] = nv;
    li[s] = nj;
    g_hi = g_lo;
  }
  lv[0] = g_hi ? v : lv[0];
  li[0] = g_hi ? j : li[0];
}

// One workgroup = KL_WAVES waves; wave w owns W tiles 2w, 2w+1 of the
// workgroup's 8 (rows wg*256 + 64 w .. + 63): after each MFMA the halves of
// the two accumulators are exchanged so that lane l holds 32 values of its own
// row (tile l / 32, row l % 32).  Column tiles are taken NT at a time (4, or
// 2 with the longest lists, to stay within the register file).
template <int PREC, int C>
__global__ void __launch_bounds__(KL_THREADS) sweep_kloop_kernel(KloopArgs a) {
  constexpr int KU = kl_units<PREC>();
  constexpr int KL_NT = C >= 128 ? 2 : 4;
  // per lane, the 32 values of its row in the current column tile: entry-major,
  // lane-minor (no bank conflicts), each lane reading back only its own
  __shared__ float stage[KL_WAVES][32][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int h = lane >> 5;
  const int l32 = lane & 31;
  const bool listed = a.row_list != nullptr;
  const int nrows_list = listed ? *a.row_count : 0;
  const int n_wt = listed ? (nrows_list + 31) / 32 : a.n_wtiles;
  const int wt0 = (blockIdx.x * KL_WAVES + wave) * 2;
  if (wt0 >= n_wt) return;                       // wave-uniform; no workgroup barrier below
  const int n32 = (int)a.n;
  const int units = a.units;                     // operand units per tile (kpad / (2 ECH))
  const int nchunks = units / KU;

  // the row this lane owns, and its candidate slot
  const int wt_own = wt0 + h;
  const int w_own = wt_own * 32 + l32;
  int myrow = -1, slot = -1;
  if (wt_own < n_wt) {
    if (listed) {
      if (w_own < nrows_list) {
        myrow = a.row_list[w_own];
        slot = w_own;
      }
    } else {
      myrow = (int)(a.row0 + w_own);
      if (myrow >= a.row_begin && myrow < a.row_end) slot = (int)(myrow - a.row_begin);
      else myrow = myrow < n32 ? myrow : -1;
    }
  }
  const double beta = slot >= 0
      ? a.cprec * a.wnorm[(int64_t)myrow - a.w_lo] * (double)__uint_as_float(*a.vmax_bits)
      : 0.0;
  const float beta2 = (float)(2.0 * beta);

  float lv[C];
  int li[C];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    lv[s] = -1.0f;
    li[s] = INVALID_J;
  }
  float tau = slot >= 0 ? -1.0f : INFINITY;       // lanes without a written row take nothing

  const int jt0 = blockIdx.y * a.tiles_per_split;
  const int jt1 = min(a.n_vtiles, jt0 + a.tiles_per_split);
  const u32x4* __restrict__ Wp = a.Wp;
  const u32x4* __restrict__ Vp = a.Vp;
  const bool t1ok = wt0 + 1 < n_wt;

  for (int jt = jt0; jt < jt1; jt += KL_NT) {
    v16f acc[2][KL_NT];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int q = 0; q < KL_NT; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[t][q][v] = 0.0f;
    u32x4 wb[2][KU], vb[KL_NT][KU];
    auto load = [&](int kc) {
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int64_t uu = (int64_t)kc * KU + u;
        wb[0][u] = Wp[((int64_t)wt0 * units + uu) * 64 + lane];
        wb[1][u] = t1ok ? Wp[((int64_t)(wt0 + 1) * units + uu) * 64 + lane] : u32x4{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < KL_NT; ++q)
          vb[q][u] = jt + q < jt1 ? Vp[((int64_t)(jt + q) * units + uu) * 64 + lane] : u32x4{0, 0, 0, 0};
      }
    };
    load(0);
    for (int kc = 0; kc < nchunks; ++kc) {
      u32x4 wc[2][KU], vc[KL_NT][KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        wc[0][u] = wb[0][u];
        wc[1][u] = wb[1][u];
#pragma unroll
        for (int q = 0; q < KL_NT; ++q) vc[q][u] = vb[q][u];
      }
      if (kc + 1 < nchunks) load(kc + 1);         // in flight during the MFMAs
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int q = 0; q < KL_NT; ++q) acc[t][q] = mfma_chunk<PREC>(vc[q], wc[t], acc[t][q], u);
    }

    // own-row values of each column tile, then the list
#pragma unroll
    for (int q = 0; q < KL_NT; ++q) {
      if (jt + q < jt1) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float p0 = acc[0][q][v], p1 = acc[1][q][v];
          swap_halves(p0, p1);
          acc[0][q][v] = p0;
          acc[1][q][v] = p1;
        }
        const int j0 = (jt + q) * 32;
        float mx = -1.0f;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int j = j0 + acc_row(v, hh);
            const float y = (j >= n32 || j == myrow) ? -1.0f : fabsf(acc[hh][q][v]);
            stage[wave][acc_row(v, hh)][lane] = y;       // entry = column within the tile
            mx = fmaxf(mx, y);
          }
        if (__ballot(mx > tau)) {
          // ascending columns (ties keep the smaller j); the lane reads back
          // only what it wrote
#pragma unroll 1
          for (int e = 0; e < 32; ++e) {
            const float xv = stage[wave][e][lane];
            if (__ballot(xv > tau)) {
              if (xv > tau) kl_insert<C>(lv, li, xv, j0 + e);
            }
          }
          // refreshed threshold: max(C-th entry, k-th entry - 2 beta)
          float kth = lv[0];
#pragma unroll
          for (int s = 1; s < C; ++s) kth = (s < a.k && lv[s] < kth) ? lv[s] : kth;
          if (slot >= 0) tau = fmaxf(lv[C - 1], kth - beta2);
        }
      }
    }
  }
  if (slot >= 0) {
    const int64_t base = ((int64_t)slot * a.S + blockIdx.y) * C;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      a.cval[base + s] = lv[s];
      a.cidx[base + s] = li[s];
    }
  }
}

// ------------------------------------------------------------------ finalize
// One wave per row, as finalize_kernel of the register-resident path, for any
// rank: candidate values are rescored exactly in FP64 with the lanes striding
// the contraction (coalesced row reads), then summed across the wave in a
// fixed order.
constexpr int GEN_MAXK = 64;
constexpr int GEN_RCAP = 512;

__device__ inline unsigned long long gen_key(float v, int j) {
  return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned)(0x7fffffff - j);
}

__device__ inline bool gen_greater(double av, int aj, double bv, int bj) {
  return av > bv || (av == bv && aj < bj);
}

__global__ void __launch_bounds__(256) finalize_gen_kernel(FinalGenArgs a) {
  __shared__ double rv[4][GEN_RCAP];
  __shared__ int rj[4][GEN_RCAP];
  __shared__ double sel_v[4][GEN_MAXK + 1];
  __shared__ int sel_j[4][GEN_MAXK + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t slotv = (int64_t)blockIdx.x * 4 + wave;
  int64_t i;
  if (a.row_list) {
    if (slotv >= *a.row_count) return;
    i = a.row_list[slotv];
  } else {
    if (slotv >= a.rows) return;
    i = a.row_begin + slotv;
  }
  const int64_t loc = i - a.row_begin;
  const int M = a.S * a.C;
  const int64_t cbase = slotv * M;
  const double vmax = (double)__uint_as_float(*a.vmax_bits);
  const double beta = a.cprec * a.wnorm[i - a.w_lo] * vmax;

  double mout = -1.0;
  for (int q = lane; q < a.S; q += 64) {
    const int64_t e = cbase + (int64_t)q * a.C;
    if (a.cidx[e + a.C - 1] != INVALID_J) mout = fmax(mout, (double)a.cval[e + a.C - 1]);
    if (a.cidx[e + a.k - 1] != INVALID_J)
      mout = fmax(mout, (double)(a.cval[e + a.k - 1] - (float)(2.0 * beta)));
  }
  mout = wave_max_f64(mout);

  unsigned long long prev = ~0ull;
  int found = 0;
  for (int t = 0; t < a.k; ++t) {
    unsigned long long best = 0;
    for (int q = lane; q < M; q += 64) {
      const int j = a.cidx[cbase + q];
      if (j == INVALID_J) continue;
      const unsigned long long key = gen_key(a.cval[cbase + q], j);
      if (key < prev && key > best) best = key;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long w = __shfl_xor(best, o, 64);
      best = w > best ? w : best;
    }
    if (best == 0) break;
    prev = best;
    found++;
  }
  const float ak = found == a.k ? __uint_as_float((unsigned)(prev >> 32)) : -1.0f;
  const double thr = (double)ak - 2.0 * beta;

  int rc = 0;
  for (int base = 0; base < M; base += 64) {
    const int q = base + lane;
    bool take = false;
    int j = INVALID_J;
    if (q < M) {
      j = a.cidx[cbase + q];
      take = j != INVALID_J && (double)a.cval[cbase + q] >= thr;
    }
    const unsigned long long mask = __ballot(take);
    const int pos = rc + __popcll(mask & ((1ull << lane) - 1ull));
    if (take && pos < GEN_RCAP) rj[wave][pos] = j;
    rc += __popcll(mask);
  }
  __builtin_amdgcn_wave_barrier();
  const bool overflow = rc > GEN_RCAP;
  const int nr = rc < GEN_RCAP ? rc : GEN_RCAP;
  const float* vi = a.V + i * a.r;
  for (int c = 0; c < nr; ++c) {
    const float* vj = a.V + (int64_t)rj[wave][c] * a.r;
    double s = 0.0;
    for (int t = lane; t < a.r; t += 64) s = fma((double)vi[t] * a.psi[t], (double)vj[t], s);
    s = wave_sum_f64(s);
    if (lane == 0) rv[wave][c] = s;
  }
  __builtin_amdgcn_wave_barrier();

  double pv = __builtin_inf();
  int pj = -1;
  int nsel = 0;
  for (int t = 0; t <= a.k; ++t) {
    double bv = -1.0, bs = 0.0;
    int bj = INVALID_J;
    for (int q = lane; q < nr; q += 64) {
      const double av = fabs(rv[wave][q]);
      const int j = rj[wave][q];
      if (gen_greater(pv, pj, av, j) && gen_greater(av, j, bv, bj)) {
        bv = av;
        bj = j;
        bs = rv[wave][q];
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oj = __shfl_xor(bj, o, 64);
      const double os = __shfl_xor(bs, o, 64);
      if (gen_greater(ov, oj, bv, bj)) {
        bv = ov;
        bj = oj;
        bs = os;
      }
    }
    if (bj == INVALID_J) break;
    if (lane == 0) {
      sel_v[wave][t] = bs;
      sel_j[wave][t] = bj;
    }
    pv = bv;
    pj = bj;
    nsel++;
  }
  __builtin_amdgcn_wave_barrier();
  bool ok = !overflow && nsel >= a.k;
  double tk = 0.0;
  if (ok) {
    tk = fabs(sel_v[wave][a.k - 1]);
    if (mout >= 0.0) ok = mout + beta < tk;
  }
  if (lane == 0) {
    if (a.counters) {
      int nvalid = 0;
      for (int q = 0; q < M; ++q) nvalid += a.cidx[cbase + q] != INVALID_J;
      atomicAdd(&a.counters[0], (unsigned long long)nvalid);
      if (ok && nsel > a.k && tk - fabs(sel_v[wave][a.k]) <= 1e-6 * tk) atomicAdd(&a.counters[1], 1ull);
    }
    if (!ok) {
      const int pos = atomicAdd(a.fail_count, 1);
      a.fail_list[pos] = (int)i;
    }
  }
  if (!ok) return;
  for (int t = lane; t < a.k; t += 64) {
    const int jt = sel_j[wave][t];
    int rank = 0;
    for (int u = 0; u < a.k; ++u) rank += sel_j[wave][u] < jt;
    a.col_out[loc * a.k + rank] = jt;
    a.val_out[loc * a.k + rank] = (float)sel_v[wave][t];
  }
}

// ------------------------------------------------------------------ exact panel
// P[q][j] = sum_t (V[row_q][t] psi[t]) V[j][t] in FP64 for the listed rows
// q in [q0, q0 + pr) and all columns: 64 x 64 output tiles, 256 threads of
// 4 x 4, the contraction in chunks of 16 through LDS, FMAs in ascending t.
__global__ void __launch_bounds__(256) exact_panel_kernel(const float* __restrict__ V, const double* __restrict__ psi,
                                                          int64_t n, int r, const int* __restrict__ list, int q0,
                                                          int pr, double* __restrict__ P) {
  __shared__ double Ws[16][65], Vs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int m0 = blockIdx.y * 64;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < r; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;                 // 0..1023 over a 64 x 16 tile
      const int mm = e >> 4, kk = e & 15;
      const int k = k0 + kk;
      double wv = 0.0, vv = 0.0;
      if (m0 + mm < pr && k < r) wv = (double)V[(int64_t)list[q0 + m0 + mm] * r + k] * psi[k];
      if (j0 + mm < n && k < r) vv = (double)V[(j0 + mm) * r + k];
      Ws[kk][mm] = wv;
      Vs[kk][mm] = vv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double wa[4], vb[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) wa[s] = Ws[kk][ty * 4 + s];
#pragma unroll
      for (int s = 0; s < 4; ++s) vb[s] = Vs[kk][tx * 4 + s];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[s][t] = fma(wa[s], vb[t], acc[s][t]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int m = m0 + ty * 4 + s;
      const int64_t j = j0 + tx * 4 + t;
      if (m < pr && j < n) P[(int64_t)m * n + j] = acc[s][t];
    }
}

// Top k of one panel row (j != the row, |value| descending, ties to the
// smaller j): k rounds of a workgroup argmax below the previous key.
__global__ void __launch_bounds__(256) panel_topk_kernel(const double* __restrict__ P, int64_t n,
                                                         const int* __restrict__ list, int q0, int pr, int k,
                                                         int64_t row_begin, int32_t* __restrict__ col_out,
                                                         float* __restrict__ val_out) {
  __shared__ double bv_s[4];
  __shared__ int bj_s[4];
  __shared__ double bs_s[4];
  __shared__ double sel_v[GEN_MAXK];
  __shared__ int sel_j[GEN_MAXK];
  const int q = blockIdx.x;
  if (q >= pr) return;
  const int64_t i = list[q0 + q];
  const double* row = P + (int64_t)q * n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double pv = __builtin_inf();
  int pj = -1;
  for (int t = 0; t < k; ++t) {
    double bv = -1.0, bs = 0.0;
    int bj = INVALID_J;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
      if (j == i) continue;
      const double s = row[j];
      const double av = fabs(s);
      if (gen_greater(pv, pj, av, (int)j) && gen_greater(av, (int)j, bv, bj)) {
        bv = av;
        bj = (int)j;
        bs = s;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oj = __shfl_xor(bj, o, 64);
      const double os = __shfl_xor(bs, o, 64);
      if (gen_greater(ov, oj, bv, bj)) {
        bv = ov;
        bj = oj;
        bs = os;
      }
    }
    if (lane == 0) {
      bv_s[wave] = bv;
      bj_s[wave] = bj;
      bs_s[wave] = bs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 4; ++w)
        if (gen_greater(bv_s[w], bj_s[w], bv_s[0], bj_s[0])) {
          bv_s[0] = bv_s[w];
          bj_s[0] = bj_s[w];
          bs_s[0] = bs_s[w];
        }
      sel_v[t] = bs_s[0];
      sel_j[t] = bj_s[0];
    }
    __syncthreads();
    pv = fabs(sel_v[t]);
    pj = sel_j[t];
    __syncthreads();
  }
  if (threadIdx.x < k) {
    const int jt = sel_j[threadIdx.x];
    int rank = 0;
    for (int u = 0; u < k; ++u) rank += sel_j[u] < jt;
    const int64_t loc = i - row_begin;
    col_out[loc * k + rank] = jt;
    val_out[loc * k + rank] = (float)sel_v[threadIdx.x];
  }
}

// ------------------------------------------------------------------ launchers
template <int PREC>
static void launch_kloop_c(int C, dim3 grid, hipStream_t st, const KloopArgs& a) {
  if (C == 32) hipLaunchKernelGGL((sweep_kloop_kernel<PREC, 32>), grid, dim3(KL_THREADS), 0, st, a);
  else if (C == 64) hipLaunchKernelGGL((sweep_kloop_kernel<PREC, 64>), grid, dim3(KL_THREADS), 0, st, a);
  else hipLaunchKernelGGL((sweep_kloop_kernel<PREC, 128>), grid, dim3(KL_THREADS), 0, st, a);
}

void launch_sweep_kloop(int prec, int C, int64_t gx, int S, hipStream_t st, const KloopArgs& a) {
  const dim3 grid((unsigned)gx, (unsigned)S);
  if (prec == P_F32) launch_kloop_c<P_F32>(C, grid, st, a);
  else launch_kloop_c<P_BF16>(C, grid, st, a);
}

void launch_finalize_gen(int64_t nrows, hipStream_t st, const FinalGenArgs& a) {
  hipLaunchKernelGGL(finalize_gen_kernel, dim3((unsigned)ceil_div(nrows, 4)), dim3(256), 0, st, a);
}

void launch_exact_panel(const float* V, const double* psi, int64_t n, int r, const int* list, int q0, int pr,
                        double* P, hipStream_t st) {
  hipLaunchKernelGGL(exact_panel_kernel, dim3((unsigned)ceil_div(n, 64), (unsigned)ceil_div(pr, 64)), dim3(256),
                     0, st, V, psi, n, r, list, q0, pr, P);
}

void launch_panel_topk(const double* P, int64_t n, const int* list, int q0, int pr, int k, int64_t row_begin,
                       int32_t* col_out, float* val_out, hipStream_t st) {
  hipLaunchKernelGGL(panel_topk_kernel, dim3((unsigned)pr), dim3(256), 0, st, P, n, list, q0, pr, k, row_begin,
                     col_out, val_out);
}

}  // namespace gmgm_rc
