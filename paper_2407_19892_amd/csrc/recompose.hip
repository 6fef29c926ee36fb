// Fused eigen-recomposition Psi = V diag(psi) V^T with per-row top-k into CSR
// (Algorithm 1, final loop: threshold while recomposing; per-row strongest
// edges as in the experiments).  Psi is never materialised.
//
// Pipeline of one call (all on the context stream):
//   prep      row norms, row maxima, non-finite check           (HBM, reads V once)
//   repack    W = V diag(psi) and V into MFMA operand tiles      (HBM)
//   sweep     each wave keeps W for 32*TI rows in registers and streams all
//             32-row tiles of V through MFMA; every lane keeps a sorted top-C
//             list (approximate |Psi|) per row it holds      (MFMA-bound)
//   finalize  one wave per row: rescore the candidates exactly (FP64), take
//             the top k, certify that no column outside the candidates can
//             beat the k-th with the precision's rounding bound, emit CSR
//   re-sweep  rows that fail the certificate: the sweep again over their rows
//             with finer operands (FP32, or split BF16 after a BF16 / FP8 sweep)
//   fallback  rows that fail again: exact FP64 scan of the whole row
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "recompose_general.h"

namespace gmgm_rc {

// ------------------------------------------------------------------ prep
// One wave per row (grid-stride): ||V_j|| max-reduced into vmax_bits (one
// atomic per workgroup), max|V_j|, and for rows in [w_lo, w_hi) the norm and
// max of W_i = V_i * psi.  Flags non-finite inputs.
__global__ void __launch_bounds__(256) prep_kernel(const float* __restrict__ V,
                                                   const double* __restrict__ psi, int64_t n,
                                                   int r, int64_t w_lo, int64_t w_hi,
                                                   float* __restrict__ vrowmax,
                                                   double* __restrict__ wnorm,
                                                   float* __restrict__ wrowmax,
                                                   unsigned* __restrict__ vmax_bits,
                                                   int* __restrict__ status) {
  __shared__ float bmax[4];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float nmax = 0.0f;
  bool bad = false;
  for (int64_t j = (int64_t)blockIdx.x * 4 + wave; j < n; j += (int64_t)gridDim.x * 4) {
    double s = 0.0, sw = 0.0;
    float mx = 0.0f, mw = 0.0f;
    const bool inw = j >= w_lo && j < w_hi;
    for (int k = lane; k < r; k += 64) {
      const float x = V[j * r + k];
      bad |= !isfinite(x);
      s += (double)x * (double)x;
      mx = fmaxf(mx, fabsf(x));
      if (inw) {
        const double pk = psi[k];
        bad |= !isfinite(pk);
        const double w = (double)x * pk;
        sw += w * w;
        mw = fmaxf(mw, fabsf((float)w));
      }
    }
    s = wave_sum_f64(s);
    mx = wave_max_f32(mx);
    nmax = fmaxf(nmax, (float)sqrt(s));
    if (!(s == s)) nmax = __builtin_nanf("");
    if (lane == 0) vrowmax[j] = mx;
    if (inw) {
      sw = wave_sum_f64(sw);
      mw = wave_max_f32(mw);
      if (lane == 0) {
        wnorm[j - w_lo] = sqrt(sw);
        wrowmax[j - w_lo] = mw;
      }
    }
  }
  if (__ballot(bad) && lane == 0) atomicCAS(status, 0, DEV_NONFINITE);
  if (lane == 0) bmax[wave] = nmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = fmaxf(fmaxf(bmax[0], bmax[1]), fmaxf(bmax[2], bmax[3]));
    // non-negative floats order like their bit patterns; NaN (0x7fc...) wins
    atomicMax(vmax_bits, __float_as_uint(m));
  }
}

// Smallest e with maxabs <= 448 * 2^e (power-of-two scale of an FP8 e4m3 row / tile).
__device__ inline int fp8_exp(float maxabs) {
  if (!(maxabs > 0.0f) || !isfinite(maxabs)) return 0;
  int e;
  frexpf(maxabs / 448.0f, &e);
  if (__builtin_ldexpf(maxabs, -(e - 1)) <= 448.0f) e -= 1;
  while (__builtin_ldexpf(maxabs, -e) > 448.0f) e += 1;
  return e;
}

__global__ void fp8_exps_kernel(const float* __restrict__ vrowmax, int64_t n, int n_vtiles,
                                const float* __restrict__ wrowmax, int64_t n_wrows,
                                int* __restrict__ ev, int* __restrict__ ew) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_vtiles) {
    float m = 0.0f;
    for (int q = 0; q < 32; ++q) {
      int64_t j = t * 32 + q;
      if (j < n) m = fmaxf(m, vrowmax[j]);
    }
    ev[t] = fp8_exp(m);
  }
  if (t < n_wrows) ew[t] = fp8_exp(wrowmax[t]);
}

// ------------------------------------------------------------------ repack
// One thread per (local row, 16-byte chunk) of `rows` local rows.  Local row w
// is global row row0 + w, or row_list[w] (w < *row_count) in list mode; rows
// outside [0, n) and k >= r are zero.
template <int PREC>
__global__ void repack_kernel(const float* __restrict__ V, const double* __restrict__ psi,
                              int64_t row0, int64_t n, int64_t rows, int r, int kpad,
                              bool fold_psi, const int* __restrict__ exps, bool exp_per_tile,
                              const int* __restrict__ row_list, const int* __restrict__ row_count,
                              u32x4* __restrict__ out) {
  constexpr int ECH = chunk_elems(PREC);
  const int nch = kpad / ECH;
  const int units = nch / 2;     // chunks per lane per tile
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= rows * nch) return;
  const int64_t w = gid / nch;
  int64_t row;
  if (row_list) {
    const int cnt = *row_count;
    if (w >= ((int64_t)cnt + 31) / 32 * 32) return;   // beyond the listed tiles
    row = w < cnt ? row_list[w] : -1;
  } else {
    row = row0 + w;
  }
  const int ch = (int)(gid % nch);
  const int k0 = ch * ECH;
  int u, h;
  if (PREC == P_F32) { u = k0 / 8; h = (k0 / 4) & 1; }
  else if (PREC == P_BF16 || PREC == P_BF16X3) { u = k0 / 16; h = (k0 / 8) & 1; }
  else { u = 2 * (k0 / 64) + ((k0 / 16) & 1); h = (k0 / 32) & 1; }
  float x[ECH];
#pragma unroll
  for (int e = 0; e < ECH; ++e) {
    const int k = k0 + e;
    float v = 0.0f;
    if (row >= 0 && row < n && k < r) {
      const float vv = V[row * r + k];
      v = fold_psi ? (float)((double)vv * psi[k]) : vv;
    }
    x[e] = v;
  }
  u32x4 o, olo = u32x4{0, 0, 0, 0};
  if (PREC == P_F32) {
    o = u32x4{__float_as_uint(x[0]), __float_as_uint(x[1]), __float_as_uint(x[2]),
              __float_as_uint(x[3])};
  } else if (PREC == P_BF16 || PREC == P_BF16X3) {
    unsigned q[4], ql[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint16_t h0 = f32_to_bf16_bits(x[2 * e]), h1 = f32_to_bf16_bits(x[2 * e + 1]);
      q[e] = (unsigned)h0 | ((unsigned)h1 << 16);
      // x - hi is exact in FP32; its BF16 rounding is the low part
      const float r0 = x[2 * e] - __uint_as_float((unsigned)h0 << 16);
      const float r1 = x[2 * e + 1] - __uint_as_float((unsigned)h1 << 16);
      ql[e] = (unsigned)f32_to_bf16_bits(r0) | ((unsigned)f32_to_bf16_bits(r1) << 16);
    }
    o = u32x4{q[0], q[1], q[2], q[3]};
    olo = u32x4{ql[0], ql[1], ql[2], ql[3]};
  } else {
    const int sc = exp_per_tile ? exps[w / 32] : exps[w];
    unsigned q[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      unsigned b = 0;
#pragma unroll
      for (int z = 0; z < 4; ++z) {
        float y = __builtin_ldexpf(x[4 * e + z], -sc);
        y = isfinite(y) ? y : 0.0f;          // non-finite inputs are already flagged
        b |= (unsigned)f32_to_e4m3_bits(fminf(fmaxf(y, -448.0f), 448.0f)) << (8 * z);
      }
      q[e] = b;
    }
    o = u32x4{q[0], q[1], q[2], q[3]};
  }
  const int64_t tile = w / 32;
  if (PREC == P_BF16X3) {
    // units: the high parts, then the low parts
    out[(tile * 2 * units + u) * 64 + (w % 32) + 32 * h] = o;
    out[(tile * 2 * units + units + u) * 64 + (w % 32) + 32 * h] = olo;
  } else {
    out[(tile * units + u) * 64 + (w % 32) + 32 * h] = o;
  }
}

// ------------------------------------------------------------------ finalize
// One wave per row.  The row's candidates are S*nsub sublists of C entries
// (descending approximate |Psi|, INVALID_J padded), one per column split and,
// when the sweep kept half rows, lane half.  With beta = cprec ||W_i|| max_j ||V_j|| bounding |approx - exact|:
//   A_k   = k-th largest approximate value among the candidates;
//   R     = candidates with approx >= A_k - 2 beta, rescored exactly (FP64);
//   T     = k-th largest exact |Psi| in R (ties to smaller j);
//   m_out = largest approximate value any non-candidate can have (the last
//           entry of every full sublist).
// Certified when m_out + beta < T: every column outside R has exact < T.
// Uncertified rows are appended (as global rows) to fail_list.
struct FinalArgs {
  const float* cval;
  const int* cidx;
  const float* V;
  const double* psi;
  const double* wnorm;       // per W row, indexed by global row - w_lo
  const unsigned* vmax_bits;
  int64_t n;
  int r, k, C, S, nsub;
  int64_t row_begin, rows;   // contiguous mode: slot s is row row_begin + s
  int64_t w_lo;
  const int* row_list;       // list mode: slot s is row row_list[s], s < *row_count
  const int* row_count;
  double cprec;
  int32_t* col_out;
  float* val_out;
  int* fail_list;
  int* fail_count;
  unsigned long long* counters;   // [0] candidates, [1] near ties (certified rows); null: not counted
  // symmetric form (contiguous rows from 0): further candidates of row i at
  // [xoff[i], xoff[i + 1]) of (xidx, xval), every value above tau[i], the
  // bound the row's list started from (null: none)
  const long long* xoff;
  const int* xidx;
  const float* xval;
  const float* tau;
};

constexpr int MAXK = 32;
constexpr int RCAP = 256;   // exact rescoring capacity per row

__device__ inline bool key_greater(double av, int aj, double bv, int bj) {
  return av > bv || (av == bv && aj < bj);
}

__device__ inline unsigned long long approx_key(float v, int j) {
  return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned)(0x7fffffff - j);
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__global__ void __launch_bounds__(256) finalize_kernel(FinalArgs a) {
  __shared__ double wrow[4][128];
  __shared__ double rv[4][RCAP];
  __shared__ int rj[4][RCAP];
  __shared__ double sel_v[4][MAXK + 1];
  __shared__ int sel_j[4][MAXK + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t slot = (int64_t)blockIdx.x * 4 + wave;
  int64_t i;
  if (a.row_list) {
    if (slot >= *a.row_count) return;
    i = a.row_list[slot];
  } else {
    if (slot >= a.rows) return;
    i = a.row_begin + slot;
  }
  const int64_t loc = i - a.row_begin;
  const int M = a.S * a.nsub * a.C;
  const int64_t cbase = slot * M;
  // candidate q: list entries first, then the symmetric form's extra ones
  int64_t xb = 0;
  int MX = M;
  if (a.xoff) {
    xb = a.xoff[i];
    MX = M + (int)(a.xoff[i + 1] - xb);
  }
  auto cand_j = [&](int q) { return q < M ? a.cidx[cbase + q] : a.xidx[xb + (q - M)]; };
  auto cand_v = [&](int q) { return q < M ? a.cval[cbase + q] : a.xval[xb + (q - M)]; };

  for (int q = lane; q < a.r; q += 64) wrow[wave][q] = (double)a.V[i * a.r + q] * a.psi[q];

  const double vmax = (double)__uint_as_float(*a.vmax_bits);
  const double beta = a.cprec * a.wnorm[i - a.w_lo] * vmax;
  // the largest value a sweep list may have dropped: its C-th entry when full,
  // and its k-th entry - 2 beta (the sweep's threshold never exceeds either)
  double mout = -1.0;
  for (int q = lane; q < a.S * a.nsub; q += 64) {
    const int64_t e = cbase + (int64_t)q * a.C;
    if (a.cidx[e + a.C - 1] != INVALID_J) mout = fmax(mout, (double)a.cval[e + a.C - 1]);
    if (a.cidx[e + a.k - 1] != INVALID_J)
      mout = fmax(mout, (double)(a.cval[e + a.k - 1] - (float)(2.0 * beta)));
  }
  mout = wave_max_f64(mout);

  // k-th largest approximate key among the candidates
  int nvalid = 0;
  for (int q = lane; q < MX; q += 64) nvalid += cand_j(q) != INVALID_J;
  nvalid = wave_sum_i32(nvalid);
  unsigned long long prev = ~0ull;
  int found = 0;
  for (int t = 0; t < a.k; ++t) {
    unsigned long long best = 0;
    for (int q = lane; q < MX; q += 64) {
      const int j = cand_j(q);
      if (j == INVALID_J) continue;
      const unsigned long long key = approx_key(cand_v(q), j);
      if (key < prev && key > best) best = key;
    }
    best = wave_max_u64(best);
    if (best == 0) break;
    prev = best;
    found++;
  }
  const float ak = found == a.k ? __uint_as_float((unsigned)(prev >> 32)) : -1.0f;
  const double thr = (double)ak - 2.0 * beta;

  // rescoring set R, compacted into LDS
  int rc = 0;
  __builtin_amdgcn_wave_barrier();
  for (int base = 0; base < MX; base += 64) {
    const int q = base + lane;
    bool take = false;
    int j = INVALID_J;
    if (q < MX) {
      j = cand_j(q);
      take = j != INVALID_J && (double)cand_v(q) >= thr;
    }
    const unsigned long long mask = __ballot(take);
    const int pos = rc + __popcll(mask & ((1ull << lane) - 1ull));
    if (take && pos < RCAP) rj[wave][pos] = j;
    rc += __popcll(mask);
  }
  __builtin_amdgcn_wave_barrier();
  const bool overflow = rc > RCAP;
  const int nr = rc < RCAP ? rc : RCAP;
  // exact values, eight candidates at a time: lane group g (8 lanes) takes
  // candidate c + g, its lane t the elements t, t + 8, ... (r <= 128), so that
  // all of a group's loads are in flight together; fixed-order sum per group
  {
    const int g = lane >> 3, t = lane & 7;
    for (int c = 0; c < nr; c += 8) {
      const int q = c + g;
      double s = 0.0;
      if (q < nr) {
        const float* vj = a.V + (int64_t)rj[wave][q] * a.r;
        float x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = t + 8 * u < a.r ? vj[t + 8 * u] : 0.0f;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (t + 8 * u < a.r) s = fma(wrow[wave][t + 8 * u], (double)x[u], s);
      }
#pragma unroll
      for (int o = 4; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (t == 0 && q < nr) rv[wave][q] = s;
    }
  }
  __builtin_amdgcn_wave_barrier();

  // exact top-(k + 1) of R by (|value| desc, j asc)
  double pv = __builtin_inf();
  int pj = -1;
  int nsel = 0;
  for (int t = 0; t <= a.k; ++t) {
    double bv = -1.0, bs = 0.0;
    int bj = INVALID_J;
    for (int q = lane; q < nr; q += 64) {
      const double av = fabs(rv[wave][q]);
      const int j = rj[wave][q];
      if (key_greater(pv, pj, av, j) && key_greater(av, j, bv, bj)) {
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
      if (key_greater(ov, oj, bv, bj)) {
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
    // symmetric form: values at or below the starting bound were dropped on
    // both sides; none of them can reach the k-th exact value
    if (a.tau) ok = ok && (double)a.tau[i] + beta < tk;
  }
  if (lane == 0) {
    if (a.counters) {   // statistics requested
      atomicAdd(&a.counters[0], (unsigned long long)nvalid);
      if (ok && nsel > a.k && tk - fabs(sel_v[wave][a.k]) <= 1e-6 * tk) atomicAdd(&a.counters[1], 1ull);
    }
    if (!ok) {
      const int pos = atomicAdd(a.fail_count, 1);
      a.fail_list[pos] = (int)i;
    }
  }
  if (!ok) return;
  if (lane < a.k) {
    const int jt = sel_j[wave][lane];
    int rank = 0;
    for (int u = 0; u < a.k; ++u) rank += sel_j[wave][u] < jt;
    a.col_out[loc * a.k + rank] = jt;
    a.val_out[loc * a.k + rank] = (float)sel_v[wave][lane];
  }
}

// ------------------------------------------------------------------ exact scan
// Exact FP64 top-k of whole rows (global rows in `list`); one workgroup per row.
__global__ void __launch_bounds__(256) exact_scan_kernel(const float* __restrict__ V,
                                                         const double* __restrict__ psi, int64_t n,
                                                         int r, int k, int64_t row_begin,
                                                         const int* __restrict__ list,
                                                         const int* __restrict__ count,
                                                         int32_t* __restrict__ col_out,
                                                         float* __restrict__ val_out) {
  __shared__ double wrow[128];
  __shared__ double red_v[256];
  __shared__ int red_j[256];
  __shared__ int red_t[256];
  __shared__ double sel_v[MAXK];
  __shared__ int sel_j[MAXK];
  const int tid = threadIdx.x;
  const int cnt = *count;
  for (int f = blockIdx.x; f < cnt; f += gridDim.x) {
    const int64_t i = list[f];
    const int64_t loc = i - row_begin;
    __syncthreads();
    for (int q = tid; q < r; q += 256) wrow[q] = (double)V[i * r + q] * psi[q];
    __syncthreads();
    double lv[MAXK];
    int li[MAXK];
#pragma unroll
    for (int s = 0; s < MAXK; ++s) {
      lv[s] = -1.0;
      li[s] = INVALID_J;
    }
    for (int64_t j = tid; j < n; j += 256) {
      if (j == i) continue;
      const float* vj = V + j * r;
      double s = 0.0;
      for (int kk = 0; kk < r; ++kk) s = fma(wrow[kk], (double)vj[kk], s);
      const double x = fabs(s);
      if (x > lv[MAXK - 1]) {
        bool gt[MAXK];
#pragma unroll
        for (int q = 0; q < MAXK; ++q) gt[q] = x > lv[q];
#pragma unroll
        for (int q = MAXK - 1; q > 0; --q) {
          const double nv = gt[q - 1] ? lv[q - 1] : (gt[q] ? x : lv[q]);
          const int nj = gt[q - 1] ? li[q - 1] : (gt[q] ? (int)j : li[q]);
          lv[q] = nv;
          li[q] = nj;
        }
        lv[0] = gt[0] ? x : lv[0];
        li[0] = gt[0] ? (int)j : li[0];
      }
    }
    // k rounds of block argmax over the heads of the per-thread lists
    int head = 0;
    for (int t = 0; t < k; ++t) {
      double hv = -1.0;
      int hj = INVALID_J;
#pragma unroll
      for (int q = 0; q < MAXK; ++q)
        if (q == head) {
          hv = lv[q];
          hj = li[q];
        }
      red_v[tid] = hv;
      red_j[tid] = hj;
      red_t[tid] = tid;
      __syncthreads();
      for (int o = 128; o > 0; o >>= 1) {
        if (tid < o && key_greater(red_v[tid + o], red_j[tid + o], red_v[tid], red_j[tid])) {
          red_v[tid] = red_v[tid + o];
          red_j[tid] = red_j[tid + o];
          red_t[tid] = red_t[tid + o];
        }
        __syncthreads();
      }
      if (tid == 0) sel_j[t] = red_j[0];
      if (tid == red_t[0]) head++;
      __syncthreads();
    }
    // Signed values and CSR order.  A selection is INVALID_J only when the row
    // has fewer than k comparable (non-NaN) values, i.e. with non-finite inputs,
    // which prep has flagged; such slots are never dereferenced.
    if (tid < k) {
      const int jt = sel_j[tid];
      double s = __builtin_nan("");
      if (jt != INVALID_J) {
        const float* vj = V + (int64_t)jt * r;
        s = 0.0;
        for (int kk = 0; kk < r; ++kk) s = fma(wrow[kk], (double)vj[kk], s);
      }
      sel_v[tid] = s;
    }
    __syncthreads();
    if (tid < k) {
      const int jt = sel_j[tid];
      if (jt == INVALID_J) {            // invalid selections come last: slot tid is free
        col_out[loc * k + tid] = -1;
        val_out[loc * k + tid] = __builtin_nanf("");
      } else {
        int rank = 0;
        for (int u = 0; u < k; ++u) rank += sel_j[u] < jt;
        col_out[loc * k + rank] = jt;
        val_out[loc * k + rank] = (float)sel_v[tid];
      }
    }
  }
}

__global__ void zero_words_kernel(unsigned* __restrict__ p, int words) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < words) p[t] = 0u;
}

__global__ void row_ptr_kernel(int64_t* __restrict__ rp, int64_t rows, int k) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= rows) rp[t] = t * k;
}

// ------------------------------------------------------------------ dispatch
int kpad_for(int prec, int r) {
  static const int f32[] = {32, 64, 104, 128};
  static const int bf16[] = {32, 64, 112, 128};
  static const int fp8[] = {64, 128};
  const int* t = prec == P_F32 ? f32 : prec == P_FP8 ? fp8 : bf16;
  int cnt = prec == P_FP8 ? 2 : 4;
  for (int q = 0; q < cnt; ++q)
    if (t[q] >= r) return t[q];
  return -1;
}

SweepFn pick_sweep(int prec, int kpad, int C) {
  if (prec == P_F32) return C == 16 ? pick_sweep_f32_c16(kpad) : pick_sweep_f32_c32(kpad);
  if (prec == P_BF16) return C == 16 ? pick_sweep_bf16_c16(kpad) : pick_sweep_bf16_c32(kpad);
  return C == 16 ? pick_sweep_fp8_c16(kpad) : pick_sweep_fp8_c32(kpad);
}


// Split BF16 (x = hi + lo + e, hi = bf16(x), lo = bf16(x - hi)):
// |lo| <= d (1 + d) |x|, |e| <= d^2 |x|, |hi| <= (1 + d) |x| with d = 2^-8.
// x y - (hi_x hi_y + hi_x lo_y + lo_x hi_y) = hi_x e_y + lo_x lo_y + lo_x e_y + e_x y,
// at most d^2 ((1 + d) + (1 + d)^2 + d (1 + d) + 1) |x||y|; the three products
// are exact in FP32 and sum (in 3 K + 1 accumulation steps) to at most
// (1 + d)^2 (1 + 2 d (1 + d)) |x||y| in magnitude.
static double cprec_split_bf16(int kpad) {
  const double u32 = std::ldexp(1.0, -24);
  const double uacc = std::ldexp(1.0, -23);
  const double d = std::ldexp(1.0, -8);
  const double K = 3.0 * kpad + 1;
  const double gam = K * uacc / (1.0 - K * uacc);
  const double drop = d * d * ((1 + d) + (1 + d) * (1 + d) + d * (1 + d) + 1);
  const double mag = (1 + d) * (1 + d) * (1 + 2 * d * (1 + d));
  const double c = (1 + u32) * (1 + drop + mag * gam) - 1;
  return c * (1 + 1e-6) + 1e-12;
}

// Rounding bound c with |Psi~_ij - Psi_ij| <= c ||W_i||_2 max_j ||V_j||_2 (see header).
// Operands: a format keeping p significant bits rounds to nearest with relative
// error at most 2^-p (FP32 p = 24, BF16 p = 8, FP8 e4m3 p = 4, plus e4m3's
// subnormal floor); W = V diag(psi) is first rounded to FP32, then to the
// operand format.  Products of BF16 or FP8 operands are exact in FP32.  The
// MFMA's internal summation order and rounding are not documented, so each of
// the K additions is charged a full unit in the last place of FP32 (2^-23),
// which also covers truncating adders.  Cauchy-Schwarz turns the elementwise
// bound sum_k |W_ik||V_jk| into ||W_i|| ||V_j||.
double cprec_for(int prec, int kpad) {
  if (prec == P_BF16X3) return cprec_split_bf16(kpad);
  const double u32 = std::ldexp(1.0, -24);     // FP32 rounding of W = V psi
  const double uacc = std::ldexp(1.0, -23);    // one FP32 ulp per accumulation step
  const double K = kpad + 1;
  const double gam = K * uacc / (1.0 - K * uacc);
  double c;
  if (prec == P_F32) {
    c = (1 + u32) * (1 + gam) - 1 + gam;          // W rounding; products and sums rounded
  } else if (prec == P_BF16) {
    const double d = std::ldexp(1.0, -8);         // BF16: 8 significant bits
    const double dw = (1 + u32) * (1 + d) - 1;
    c = (1 + dw) * (1 + d) * (1 + gam) - 1;
  } else {
    const double d = std::ldexp(1.0, -4);         // e4m3: 4 significant bits
    const double dw = (1 + u32) * (1 + d) - 1;
    // subnormal floor: half of e4m3's smallest spacing 2^-9 in scaled units,
    // per unit of the row / tile maximum, which is scaled above 224
    const double fl = std::ldexp(1.0, -10) / 224.0;
    c = (1 + dw) * (1 + d) * (1 + gam) - 1 + 2 * (1 + d) * std::sqrt((double)kpad) * fl * (1 + gam) +
        kpad * fl * fl;
  }
  return c * (1 + 1e-6) + 1e-12;
}


// Split the columns so that the grid has about `target` workgroups, keeping
// at least two LDS stages per split.
static int pick_splits(int64_t gx, int n_vtiles, int smax, int64_t target) {
  int S = 1;
  while (S < smax && gx * S < target && (int64_t)n_vtiles >= (int64_t)(2 * S) * 8) S *= 2;
  return S;
}

struct StageBufs {
  const u32x4* vp;
  const u32x4* wp;
  float* cval;
  int* cidx;
};

static gmgm_status stage_buffers(gmgm_ctx* c, int slot_wp, int slot_cand, int64_t wtiles, int units,
                                 int64_t slots, int S, int nsub, int C, StageBufs* b) {
  void *wp, *cand;
  const size_t ncand = (size_t)slots * S * nsub * C;
  GMGM_TRY(ws_get(c, slot_wp, (size_t)wtiles * units * 64 * 16, &wp));
  GMGM_TRY(ws_get(c, slot_cand, ncand * 8, &cand));
  b->wp = (const u32x4*)wp;
  b->cval = (float*)cand;
  b->cidx = (int*)((char*)cand + ncand * 4);
  return GMGM_OK;
}

template <class F>
static void launch_repack(int prec, F&& f) {
  if (prec == P_F32) f(repack_kernel<P_F32>);
  else if (prec == P_BF16) f(repack_kernel<P_BF16>);
  else f(repack_kernel<P_FP8>);
}


// ---------------------------------------------------------------------------
// Threshold mode: every j != i with |Psi_ij| >= thr (the significance
// threshold of Theorem 3, or any fixed threshold), as CSR.

constexpr int THR_CAPT = 1024;   // sweep candidates per row (more: exact scan)

struct ThrArgs {
  const float* V;
  const double* psi;
  int64_t n;
  int r;
  double thr;
  int64_t row_begin, rows;
  const int* cidx;          // candidates, ascending j per row: [slot][THR_CAPT], or at toff[q]
  const int* tcount;        // per verified row; above its room: overflowed
  const int* list;          // verified rows (slots), or null: every slot in order
  const long long* toff;    // with list: candidate offsets per listed row (room: the next offset)
  int* fail_rows;           // overflowed rows as global row ids (for a listed re-sweep)
  int* pool_j;              // kept entries, one contiguous run per row
  float* pool_v;
  long long pool_cap;
  long long* pool_top;      // bump allocator (may pass pool_cap: then nothing is written)
  long long* pool_off;      // [slot]
  int* kept_n;              // [slot]
  int* fail_list;           // rows whose candidates overflowed (exact scan)
  int* fail_count;
};

// One wave per row: exact FP64 value of every candidate (eight-lane groups, as
// in finalize), kept when |Psi_ij| >= thr; the candidates arrive in ascending
// j, and the kept ones are written in that order to a run reserved in the pool.
__global__ void __launch_bounds__(256) thr_verify_kernel(ThrArgs a) {
  __shared__ double wrow[4][128];
  __shared__ double sv[4][THR_CAPT];    // exact values of the candidates, chunk by chunk
  __shared__ long long soff[4];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t qv = (int64_t)blockIdx.x * 4 + wave;      // index among the verified rows
  if (qv >= a.rows) return;
  const int64_t slot = a.list ? a.list[qv] : qv;
  const int64_t i = a.row_begin + slot;
  const int m = a.tcount[qv];
  const int room = a.list ? (int)(a.toff[qv + 1] - a.toff[qv]) : THR_CAPT;
  if (m > room) {
    if (lane == 0) {
      const int f = atomicAdd(a.fail_count, 1);
      a.fail_list[f] = (int)slot;
      if (a.fail_rows) a.fail_rows[f] = (int)i;
    }
    return;
  }
  for (int q = lane; q < a.r; q += 64) wrow[wave][q] = (double)a.V[i * a.r + q] * a.psi[q];
  __builtin_amdgcn_wave_barrier();
  const int* cj = a.cidx + (a.list ? a.toff[qv] : slot * THR_CAPT);
  const int g = lane >> 3, t = lane & 7;
  // the exact value of candidate q (lanes of group g = q % 8 take part; the sum
  // lands on every lane of the group)
  auto exact = [&](int q) {
    double s = 0.0;
    if (q < m) {
      const float* vj = a.V + (int64_t)cj[q] * a.r;
      float x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = t + 8 * u < a.r ? vj[t + 8 * u] : 0.0f;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (t + 8 * u < a.r) s = fma(wrow[wave][t + 8 * u], (double)x[u], s);
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
  };
  // pass 1: count the kept candidates (caching their values when they fit)
  const bool cached = m <= THR_CAPT;
  int kept = 0;
  for (int c = 0; c < m; c += 8) {
    const int q = c + g;
    const double s = exact(q);
    const bool keep = t == 0 && q < m && cj[q] != (int)i && fabs(s) >= a.thr;
    if (cached && t == 0 && q < m) sv[wave][q] = keep ? s : __builtin_nan("");
    kept += __popcll(__ballot(keep));
  }
  if (lane == 0) {
    soff[wave] = atomicAdd((unsigned long long*)a.pool_top, (unsigned long long)kept);
    a.pool_off[slot] = soff[wave];
    a.kept_n[slot] = kept;
  }
  __builtin_amdgcn_wave_barrier();
  const long long off = soff[wave];
  if (off + kept > a.pool_cap) return;       // the pool is too small: sizes only
  // pass 2: the kept candidates, in order, into the row's run
  int pos = 0;
  if (cached) {
    for (int c = 0; c < m; c += 64) {
      const int q = c + lane;
      const bool keep = q < m && !(sv[wave][q] != sv[wave][q]);
      const unsigned long long mask = __ballot(keep);
      if (keep) {
        const long long o = off + pos + __popcll(mask & ((1ull << lane) - 1ull));
        a.pool_j[o] = cj[q];
        a.pool_v[o] = (float)sv[wave][q];
      }
      pos += __popcll(mask);
    }
  } else {
    for (int c = 0; c < m; c += 8) {
      const int q = c + g;
      const double s = exact(q);
      const bool keep = t == 0 && q < m && cj[q] != (int)i && fabs(s) >= a.thr;
      const unsigned long long mask = __ballot(keep);
      if (keep) {
        const long long o = off + pos + __popcll(mask & ((1ull << lane) - 1ull));
        a.pool_j[o] = cj[q];
        a.pool_v[o] = (float)s;
      }
      pos += __popcll(mask);
    }
  }
}

// Rows whose candidates overflowed: one workgroup per row scans every column
// exactly in FP64 twice, to count and then to write its run in column order.
__global__ void __launch_bounds__(256) thr_exact_kernel(ThrArgs a) {
  __shared__ double wrow[128];
  __shared__ int wcnt[4];
  __shared__ long long soff;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cnt = *a.fail_count;
  for (int f = blockIdx.x; f < cnt; f += gridDim.x) {
    const int64_t slot = a.fail_list[f];
    const int64_t i = a.row_begin + slot;
    __syncthreads();
    for (int q = tid; q < a.r; q += 256) wrow[q] = (double)a.V[i * a.r + q] * a.psi[q];
    __syncthreads();
    long long off = 0;
    for (int pass = 0; pass < 2; ++pass) {
      long long kept = 0;   // uniform across the workgroup
      for (int64_t j0 = 0; j0 < a.n; j0 += 256) {
        const int64_t j = j0 + tid;
        bool keep = false;
        double s = 0.0;
        if (j < a.n && j != i) {
          const float* vj = a.V + j * a.r;
          for (int kk = 0; kk < a.r; ++kk) s = fma(wrow[kk], (double)vj[kk], s);
          keep = fabs(s) >= a.thr;
        }
        const unsigned long long mask = __ballot(keep);
        if (lane == 0) wcnt[wave] = __popcll(mask);
        __syncthreads();
        long long before = kept;
        for (int w = 0; w < wave; ++w) before += wcnt[w];
        const long long o = off + before + __popcll(mask & ((1ull << lane) - 1ull));
        if (pass == 1 && keep && o < a.pool_cap) {
          a.pool_j[o] = (int)j;
          a.pool_v[o] = (float)s;
        }
        kept += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
      }
      if (pass == 0) {
        if (tid == 0) {
          soff = atomicAdd((unsigned long long*)a.pool_top, (unsigned long long)kept);
          a.pool_off[slot] = soff;
          a.kept_n[slot] = (int)kept;
        }
        __syncthreads();
        off = soff;
        if (off + kept > a.pool_cap) break;   // sizes only
      }
    }
  }
}

// Candidate counts of the listed rows (out[q] = count[list[q]]).
__global__ void thr_counts_kernel(const int* __restrict__ list, int nl, const int* __restrict__ count,
                                  int* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nl) out[q] = count[list[q]];
}

// One workgroup: row_ptr = exclusive prefix sum of the kept counts (int64),
// plus the total and the largest count (info[0], info[1]).
__global__ void __launch_bounds__(1024) thr_scan_kernel(const int* __restrict__ kept_n, int64_t rows,
                                                        int64_t* __restrict__ row_ptr,
                                                        long long* __restrict__ info) {
  __shared__ long long part[1024];
  __shared__ int pmax[1024];
  const int tid = threadIdx.x;
  const int64_t per = (rows + 1023) / 1024;
  const int64_t b = tid * per, e = min(rows, b + per);
  long long sum = 0;
  int mx = 0;
  for (int64_t q = b; q < e; ++q) {
    sum += kept_n[q];
    mx = max(mx, kept_n[q]);
  }
  part[tid] = sum;
  pmax[tid] = mx;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan (Hillis-Steele)
    const long long v = tid >= off ? part[tid - off] : 0;
    const int m2 = tid >= off ? pmax[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    pmax[tid] = max(pmax[tid], m2);
    __syncthreads();
  }
  long long run = tid > 0 ? part[tid - 1] : 0;
  for (int64_t q = b; q < e; ++q) {
    row_ptr[q] = run;
    run += kept_n[q];
  }
  if (tid == 1023) {
    row_ptr[rows] = part[1023];
    info[0] = part[1023];
    info[1] = pmax[1023];
  }
}

// One wave per row: its run of the pool into the CSR arrays.
__global__ void __launch_bounds__(256) thr_gather_kernel(const int* __restrict__ pool_j, const float* __restrict__ pool_v,
                                                         const long long* __restrict__ pool_off,
                                                         const int* __restrict__ kept_n, const int64_t* __restrict__ row_ptr,
                                                         int64_t rows, int32_t* __restrict__ col_out,
                                                         float* __restrict__ val_out) {
  const int lane = threadIdx.x & 63;
  const int64_t slot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (slot >= rows) return;
  const int64_t o = row_ptr[slot];
  const long long src = pool_off[slot];
  const int cnt = kept_n[slot];
  for (int q = lane; q < cnt; q += 64) {
    col_out[o + q] = pool_j[src + q];
    val_out[o + q] = pool_v[src + q];
  }
}

// ------------------------------------------------------------ symmetric form
// Bound of every row from a sweep over a sample of the columns: the exact FP64
// values of the sample's k largest approximate |Psi_ij| (list entries 0 .. k-1,
// k distinct columns), their minimum e_k, minus beta_i, rounded down to a
// float.  The row's final k-th exact value T is at least e_k (k of its values
// are at least e_k).  A value whose approximation is at most the bound is at
// most bound + beta_i exactly; the finalize certifies a row only when
// bound + beta_i < T, so no such value can be among its top k.  Rows without
// a positive bound (fewer than k sample columns, a rounding margin as large as
// the values) get +inf: the column side keeps nothing for them and their
// certificate fails (they are re-swept in full).  Rows n .. 32 n_vtiles - 1
// (padding) get +inf.  One wave per row, four rows per workgroup.
__global__ void __launch_bounds__(256) tau_kernel(const float* __restrict__ cval, const int* __restrict__ cidx,
                                                  int C, int k, const float* __restrict__ V,
                                                  const double* __restrict__ psi, int r,
                                                  const double* __restrict__ wnorm,
                                                  const unsigned* __restrict__ vmax_bits, double cprec, int64_t n,
                                                  float* __restrict__ tau) {
  __shared__ double wrow[4][128];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  float out = INFINITY;
  bool have = i < n;
  if (have) have = cidx[i * C + k - 1] != INVALID_J;
  if (have) {
    for (int q = lane; q < r; q += 64) wrow[wave][q] = (double)V[i * r + q] * psi[q];
    __builtin_amdgcn_wave_barrier();
    // eight lanes per candidate: lane t of group g takes elements t, t + 8, ...
    const int g = lane >> 3, t = lane & 7;
    double ek = INFINITY;
    for (int c0 = 0; c0 < k; c0 += 8) {
      const int q = c0 + g;
      double sum = 0.0;
      if (q < k) {
        const float* vj = V + (int64_t)cidx[i * C + q] * r;
        for (int u = t; u < r; u += 8) sum = fma(wrow[wave][u], (double)vj[u], sum);
      }
#pragma unroll
      for (int o = 4; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
      double m = q < k ? fabs(sum) : INFINITY;
#pragma unroll
      for (int o = 8; o < 64; o <<= 1) m = fmin(m, __shfl_xor(m, o, 64));
      ek = fmin(ek, m);
    }
    const double beta = cprec * wnorm[i] * (double)__uint_as_float(*vmax_bits);
    const double b = ek - beta;
    if (b > 0.0 && b < 3.0e38) {
      float f = (float)b;
      if ((double)f > b) f = float_below(f);
      out = f;
    }
  }
  if (lane == 0) tau[i] = out;
}

// Exclusive prefix sum of per-row counts into int64 offsets (off[n] = total),
// in three steps: sums of 1024-row blocks, their scan (one workgroup), then
// each block's own scan plus its base.
__device__ inline long long block_scan_1024(long long v, long long* sh, long long* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {   // inclusive scan (Hillis-Steele)
    const long long w = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += w;
    __syncthreads();
  }
  *total = sh[1023];
  const long long ex = t > 0 ? sh[t - 1] : 0;
  __syncthreads();
  return ex;
}

__global__ void __launch_bounds__(1024) rows_block_sum_kernel(const int* __restrict__ cnt, int64_t n,
                                                              long long* __restrict__ bsum) {
  __shared__ long long sh[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  long long tot;
  block_scan_1024(i < n ? cnt[i] : 0, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) rows_base_scan_kernel(long long* __restrict__ bsum, int nb,
                                                              int64_t* __restrict__ off_end, long long* __restrict__ info) {
  __shared__ long long sh[1024];
  long long run = 0;
  for (int b0 = 0; b0 < nb; b0 += 1024) {
    const int b = b0 + threadIdx.x;
    long long tot;
    const long long ex = block_scan_1024(b < nb ? bsum[b] : 0, sh, &tot);
    if (b < nb) bsum[b] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) {
    *off_end = run;
    info[0] = run;
  }
}

__global__ void __launch_bounds__(1024) rows_offsets_kernel(const int* __restrict__ cnt, int64_t n,
                                                            const long long* __restrict__ bbase,
                                                            int64_t* __restrict__ off) {
  __shared__ long long sh[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  long long tot;
  const long long ex = block_scan_1024(i < n ? cnt[i] : 0, sh, &tot);
  if (i < n) off[i] = bbase[blockIdx.x] + ex;
}

// Column-side entries per row: count (one workgroup per pool chunk; chunks
// never handed out have fill 0).
__global__ void __launch_bounds__(256) cs_count_kernel(const int* __restrict__ cs_j, const int* __restrict__ fill,
                                                       int chunk, int64_t n, int* __restrict__ per_row) {
  const int m = min(fill[blockIdx.x], chunk);
  const int64_t b = (int64_t)blockIdx.x * chunk;
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    const int j = cs_j[b + e];
    if (j >= 0 && j < n) atomicAdd(&per_row[j], 1);
  }
}

// ... and scatter into per-row runs at off[j] (per_row counts down to zero;
// the order inside a run is arbitrary, the finalize orders by value and index).
__global__ void __launch_bounds__(256) cs_scatter_kernel(const int* __restrict__ cs_j, const int* __restrict__ cs_i,
                                                         const float* __restrict__ cs_v, const int* __restrict__ fill,
                                                         int chunk, int64_t n, const int64_t* __restrict__ off,
                                                         int* __restrict__ per_row, int* __restrict__ xidx,
                                                         float* __restrict__ xval) {
  const int m = min(fill[blockIdx.x], chunk);
  const int64_t b = (int64_t)blockIdx.x * chunk;
  for (int e = threadIdx.x; e < m; e += blockDim.x) {
    const int j = cs_j[b + e];
    if (j < 0 || j >= n) continue;
    const int64_t pos = off[j] + atomicSub(&per_row[j], 1) - 1;
    xidx[pos] = cs_i[b + e];
    xval[pos] = cs_v[b + e];
  }
}

}  // namespace gmgm_rc

using namespace gmgm_rc;

constexpr int TOPK_MAX_R = 32768;
constexpr int TOPK_MAX_K = 64;

// The register-resident sweep (W held in registers, lists of 16 or 32) serves
// r <= 128 and k <= 24; everything else takes the K-loop sweep.
static bool topk_fast_path(int64_t r, int k, int cand_cap) {
  return r <= 128 && k <= 24 && (cand_cap == 0 || cand_cap == 16 || cand_cap == 32);
}

// K-loop path: the contraction padded to a multiple of 32 (one chunk), FP8
// requests served by the BF16 sweep.  Above KL_BF16_MAX_R the BF16 bound
// (which grows with ||W_i|| max_j ||V_j|| while the entries near the k-th do
// not) certifies no row in practice (n = r = 20000: every row re-swept), so
// the first sweep runs in FP32 whatever the request.
constexpr int64_t KL_BF16_MAX_R = 4096;
static int kl_prec(int prec, int64_t r) {
  return (prec == P_F32 || r > KL_BF16_MAX_R) ? P_F32 : P_BF16;
}
static int kl_kpad(int64_t r) { return (int)ceil_div(r, 32) * 32; }

// Arguments of gmgm_recompose_topk, checked before anything is launched.
static gmgm_status topk_check(gmgm_ctx* c, int64_t n, int64_t r, const float* V, const double* psi,
                              int64_t row_begin, int64_t row_end, int32_t k, int prec, int32_t cand_cap,
                              const int64_t* row_ptr_out, const int32_t* col_out, const float* val_out,
                              int* C_out) {
  if (prec < 0 || prec > 2) return set_err(c, GMGM_E_ARG, "unknown precision %d", prec);
  if (n < 2 || n > 0x7fffffc0LL) return set_err(c, GMGM_E_SHAPE, "n = %lld out of range [2, 2^31 - 64]", (long long)n);
  if (r < 1 || r > TOPK_MAX_R)
    return set_err(c, GMGM_E_SHAPE, "r = %lld must be in [1, %d]", (long long)r, TOPK_MAX_R);
  if (row_begin < 0 || row_end > n || row_begin >= row_end)
    return set_err(c, GMGM_E_SHAPE, "row range [%lld, %lld) invalid for n = %lld",
                   (long long)row_begin, (long long)row_end, (long long)n);
  if (!V || !psi || !row_ptr_out || !col_out || !val_out)
    return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (k < 1 || k > TOPK_MAX_K || k > n - 1)
    return set_err(c, GMGM_E_ARG, "k = %d must be in [1, min(%d, n-1)]", k, TOPK_MAX_K);
  if (topk_fast_path(r, k, cand_cap)) {
    // Default list length: 32 per full row (BF16 / FP8 sweeps) or 16 per half row
    // (FP32 sweep): both leave 32 candidates per row.
    const int C = cand_cap != 0 ? cand_cap : (prec != P_F32 || k > 12) ? 32 : 16;
    if (C <= k) return set_err(c, GMGM_E_ARG, "cand_cap %d must exceed k = %d", C, k);
    *C_out = C;
    return GMGM_OK;
  }
  // K-loop sweep: lists of 32, 64 or 128 per row, at least twice k by default
  const int C = cand_cap != 0 ? cand_cap : (2 * k <= 32 ? 32 : 2 * k <= 64 ? 64 : 128);
  if (C != 32 && C != 64 && C != 128)
    return set_err(c, GMGM_E_ARG, "cand_cap must be 0, 16 or 32 (r <= 128, k <= 24), else 0, 32, 64 or 128");
  if (C <= k) return set_err(c, GMGM_E_ARG, "cand_cap %d must exceed k = %d", C, k);
  *C_out = C;
  return GMGM_OK;
}

// Workspace of the first sweep of one gmgm_recompose_topk call (every slot it
// asks for, each rounded up to 256 bytes as the fixed arena places them), with
// the column splits capped at smax.
static size_t topk_workspace_bound(int prec, int64_t n, int64_t r, int64_t row_begin, int64_t row_end, int C,
                                   int smax, int k) {
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  if (!topk_fast_path(r, k, C)) {
    const int pk = kl_prec(prec, r);
    const int units = kl_kpad(r) / chunk_elems(pk) / 2;
    const int64_t rows = row_end - row_begin;
    const int n_vtiles = (int)ceil_div(n, 32);
    const int n_wtiles = (int)ceil_div(row_end, 32) - (int)(row_begin / 32);
    const int64_t w_rows = (int64_t)n_wtiles * 32;
    const int S = pick_splits(ceil_div(n_wtiles, (int64_t)KL_WAVES * 2), n_vtiles, smax, 1024);
    size_t t = 0;
    t += up((size_t)n_vtiles * units * 64 * 16);                    // WS_VP
    t += up((size_t)n * 4 + (size_t)w_rows * 12 + 256);               // WS_NORMS
    t += up(256);                                                     // WS_MISC
    t += up((size_t)rows * 8 + 64);                                   // WS_FALLBACK
    t += up((size_t)n_wtiles * units * 64 * 16);                      // WS_WP
    t += up((size_t)rows * S * C * 8);                                // WS_CAND
    t += up((size_t)n * 8);                                           // one exact panel row
    return t;
  }
  const int kpad = kpad_for(prec, (int)r);
  const int TI = ti_for(prec, C);
  const int units = kpad / chunk_elems(prec) / 2;
  const int64_t rows = row_end - row_begin;
  const int n_vtiles = (int)ceil_div(n, 32);
  const int n_wtiles = (int)ceil_div(row_end, 32) - (int)(row_begin / 32);
  const int64_t w_rows = (int64_t)n_wtiles * 32;
  const int64_t gx = ceil_div(n_wtiles, (int64_t)SW_WAVES * TI);
  const int S = pick_splits(gx, n_vtiles, smax, 1024);
  const int nsub = sweep_nsub(TI);
  size_t t = 0;
  t += up((size_t)n_vtiles * units * 64 * 16);                      // WS_VP
  t += up((size_t)n * 4 + (size_t)w_rows * 12 + 256);                 // WS_NORMS
  t += up(256);                                                       // WS_MISC
  t += up((size_t)rows * 8 + 64);                                     // WS_FALLBACK
  t += up(((size_t)n_vtiles + (size_t)w_rows) * 4 + 64);              // WS_SCALES
  t += up((size_t)n_wtiles * units * 64 * 16);                        // WS_WP
  t += up((size_t)rows * S * nsub * C * 8);                           // WS_CAND
  return t;
}

static gmgm_status topk_impl(gmgm_ctx* c, int64_t n, int64_t r, const float* V, const double* psi,
                             int64_t row_begin, int64_t row_end, int32_t k, int prec, int C, int smax,
                             int64_t* row_ptr_out, int32_t* col_out, float* val_out, gmgm_topk_stats* stats,
                             bool allow_sym = true);
static gmgm_status topk_general(gmgm_ctx* c, int64_t n, int64_t r, const float* V, const double* psi,
                                int64_t row_begin, int64_t row_end, int32_t k, int prec, int C, int smax,
                                int64_t* row_ptr_out, int32_t* col_out, float* val_out, gmgm_topk_stats* stats);

extern "C" gmgm_status gmgm_recompose_topk(gmgm_ctx_t c, int64_t n, int64_t r, const float* V,
                                           const double* psi, int64_t row_begin, int64_t row_end,
                                           int32_t k, gmgm_prec prec_e, int32_t cand_cap,
                                           int64_t* row_ptr_out, int32_t* col_out, float* val_out,
                                           gmgm_topk_stats* stats) {
  GMGM_CHECK_CTX(c);
  int C = 0;
  GMGM_TRY(topk_check(c, n, r, V, psi, row_begin, row_end, k, (int)prec_e, cand_cap, row_ptr_out, col_out,
                      val_out, &C));
  return topk_impl(c, n, r, V, psi, row_begin, row_end, k, (int)prec_e, C, 16, row_ptr_out, col_out, val_out,
                   stats);
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the same call with every workspace slot carved
// from a fixed device array.  Each device holds its own copy of the array
// from the library's load until the process ends; its device address is
// looked up once per device (gmgm_create) and only that address is used.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch_address(int device, void** ptr, size_t* bytes) {
  static std::mutex mu;
  static std::vector<void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *ptr = nullptr;
      *bytes = 0;
      return e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    addr[device] = p;
  }
  *ptr = addr[device];
  *bytes = NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

extern "C" gmgm_status gmgm_recompose_topk_noalloc(gmgm_ctx_t c, int64_t n, int64_t r, const float* V,
                                                   const double* psi, int64_t row_begin, int64_t row_end,
                                                   int32_t k, gmgm_prec prec_e, int32_t cand_cap,
                                                   int64_t* row_ptr_out, int32_t* col_out, float* val_out,
                                                   gmgm_topk_stats* stats) {
  GMGM_CHECK_CTX(c);
  int C = 0;
  GMGM_TRY(topk_check(c, n, r, V, psi, row_begin, row_end, k, (int)prec_e, cand_cap, row_ptr_out, col_out,
                      val_out, &C));
  if (c->scratch_status != hipSuccess || !c->scratch)
    return hip_err(c, c->scratch_status != hipSuccess ? c->scratch_status : hipErrorInvalidSymbol,
                   "hipGetSymbolAddress(scratch) at context creation");
  // fewer column splits (less parallelism for small n, shorter candidate
  // buffers) until the first sweep's workspace fits
  int smax = 16;
  while (smax > 1 && topk_workspace_bound((int)prec_e, n, r, row_begin, row_end, C, smax, k) > c->scratch_bytes)
    smax /= 2;
  const size_t need = topk_workspace_bound((int)prec_e, n, r, row_begin, row_end, C, smax, k);
  if (need > c->scratch_bytes)
    return set_err(c, GMGM_E_SHAPE,
                   "workspace of %zu bytes needed for n = %lld, r = %lld, %lld rows exceeds the fixed %zu bytes",
                   need, (long long)n, (long long)r, (long long)(row_end - row_begin), c->scratch_bytes);
  // no event is created while the arena is set (timing is off for this call)
  const bool timing = c->timing;
  c->timing = false;
  arena_begin(c, c->scratch, c->scratch_bytes);
  const gmgm_status s = topk_impl(c, n, r, V, psi, row_begin, row_end, k, (int)prec_e, C, smax, row_ptr_out,
                                  col_out, val_out, stats);
  arena_end(c);
  c->timing = timing;
  return s;
}

// The symmetric form serves BF16 calls for every row of Psi (outside
// allocation-free calls) from SYM_MIN_N rows on; GMGM_RECOMPOSE_PATH=full or
// =symmetric (n >= 1024) overrides the size rule.  Measured with r = 100,
// k = 10 on clustered factors: 0.92x the full sweep's step time at n = 10^6,
// 1.08x at n = 2^19 (its bound pass and grouping cost a fixed share that the
// halved sweep outgrows only at large n).
constexpr int64_t SYM_MIN_N = 800000;
constexpr int SYM_STRIDE = 8;         // the bound pass visits every 8th column tile
// Column-side pool: SYM_MARGIN times the entries expected (a value beats its
// row's bound with probability about k SYM_STRIDE / n, the bound being near
// the k-th largest of a 1/SYM_STRIDE sample), plus a chunk per wave.  A chunk
// holds at least 2048 entries and twice SYM_MARGIN times what a wave expects
// in one stage (a stage starts with half a chunk free).
constexpr double SYM_MARGIN = 4.0;

static bool sym_wanted(gmgm_ctx* c, int prec, int64_t n, int64_t row_begin, int64_t row_end) {
  if (prec != P_BF16 || row_begin != 0 || row_end != n || c->arena || n < 1024) return false;
  const char* e = getenv("GMGM_RECOMPOSE_PATH");
  if (e && !strcmp(e, "full")) return false;
  if (e && !strcmp(e, "symmetric")) return true;
  return n >= SYM_MIN_N;
}

struct SymBufs {
  const float* tau;
  const int64_t* off;
  const int* xidx;
  const float* xval;
};

// The symmetric form of the sweep for every row (contiguous from 0), in three
// steps:
//  1. bound pass: the sweep over every SYM_STRIDE-th column tile with lists of
//     16 (k <= 16) or 32, then the per-row bound tau (tau_kernel);
//  2. symmetric sweep: workgroup b visits column tiles from its own first row
//     tile on; its rows' lists start from tau, and values beyond its own block
//     above tau[j] go to the column-side pool;
//  3. the column-side entries grouped by row (count, prefix sum, scatter), for
//     the finalize to take with the lists.
// Sets *overflow (and does nothing else after step 2) when the pool ran out
// or one wave's stage produced more entries than the half chunk it started
// with; before step 1 when the pool would need 2^31 entries or more.
static gmgm_status sym_sweep(gmgm_ctx* c, const SweepArgs& sa, const float* V, const double* psi, int r, int kpad,
                             int C, int64_t gx, SymBufs* out, double* flops, bool* overflow) {
  hipStream_t st = c->stream;
  const int64_t n = sa.n;
  const int n_vtiles = sa.n_vtiles;
  const int64_t npad = (int64_t)n_vtiles * 32;
  const int64_t w_rows = (int64_t)sa.n_wtiles * 32;
  const int k = sa.k;
  const int CA = k <= 16 ? 16 : 32;
  SweepFn sweepA = pick_sweep_bf16_sample(kpad, CA);
  SweepFn sweepS = pick_sweep_bf16_sym(kpad, C);
  if (!sweepA || !sweepS) return set_err(c, GMGM_E_SHAPE, "no symmetric sweep variant for kpad = %d", kpad);
  // pool size: workgroup b's 64-row waves see 32 T_b columns each
  const double p_hit = std::min(1.0, (double)k * SYM_STRIDE / (double)n);
  double expect = 0.0;
  for (int64_t b = 0; b < gx; ++b) {
    const int64_t tb = std::max<int64_t>(0, n_vtiles - (b + 1) * SW_WAVES * 2);
    expect += SW_WAVES * 64.0 * 32.0 * (double)tb * p_hit;
  }
  const int tps = sweep_tps(kpad / 16);   // column tiles per stage (BF16 units of 16)
  const double per_stage = 64.0 * 32.0 * tps * p_hit;
  const int chunk = (int)std::max<double>(2048.0, std::ceil(2.0 * SYM_MARGIN * per_stage / 256.0) * 256.0);
  const int64_t chunks = (int64_t)std::ceil(SYM_MARGIN * expect / chunk) + gx * SW_WAVES;
  const int64_t cap = chunks * chunk;
  if (cap >= ((int64_t)1 << 31) - chunk) {   // 32-bit pool indices: the full sweep instead
    *overflow = true;
    return GMGM_OK;
  }
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  // WS_SYM0: tau | bound-pass lists (values, indices) | per-row counts | row
  // offsets | info | pool counter + flag | chunk fills
  const size_t o_tau = 0;
  const size_t o_av = o_tau + up((size_t)npad * 4);
  const size_t o_ai = o_av + up((size_t)w_rows * CA * 4);
  const size_t o_cnt = o_ai + up((size_t)w_rows * CA * 4);
  const size_t o_off = o_cnt + up((size_t)n * 4);
  const size_t o_bs = o_off + up((size_t)(n + 1) * 8);
  const size_t o_info = o_bs + up((size_t)ceil_div(n, 1024) * 8);
  const size_t o_flag = o_info + 256;
  const size_t o_fill = o_flag + 256;
  const size_t bytes0 = o_fill + up((size_t)chunks * 4);
  void *w0, *w1;
  GMGM_TRY(ws_get(c, WS_SYM0, bytes0, &w0));
  GMGM_TRY(ws_get(c, WS_SYM1, (size_t)cap * 12, &w1));
  char* b0 = (char*)w0;
  float* tau = (float*)(b0 + o_tau);
  float* av = (float*)(b0 + o_av);
  int* ai = (int*)(b0 + o_ai);
  int* per_row = (int*)(b0 + o_cnt);
  int64_t* off = (int64_t*)(b0 + o_off);
  long long* bsum = (long long*)(b0 + o_bs);
  long long* info = (long long*)(b0 + o_info);
  unsigned* next = (unsigned*)(b0 + o_flag);
  int* flag = (int*)(b0 + o_flag + 8);
  int* fill = (int*)(b0 + o_fill);
  int* cs_j = (int*)w1;
  int* cs_i = cs_j + cap;
  float* cs_v = (float*)(cs_i + cap);

  // 1. bound pass
  SweepArgs pa = sa;
  pa.cval = av;
  pa.cidx = ai;
  pa.S = 1;
  pa.tiles_per_split = n_vtiles;
  pa.jt_stride = SYM_STRIDE;
  sweepA<<<dim3((unsigned)gx, 1), dim3(SW_THREADS), 0, st>>>(pa);
  hipLaunchKernelGGL(tau_kernel, dim3((unsigned)(npad / 4)), dim3(256), 0, st, (const float*)av, (const int*)ai,
                     CA, k, V, psi, r, sa.wnorm, sa.vmax_bits, sa.cprec, n, tau);
  // 2. symmetric sweep (pool counter, flag and chunk fills cleared first)
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)ceil_div(chunks + 64, 256)), dim3(256), 0, st,
                     (unsigned*)next, (int)(256 / 4 + chunks));
  SweepArgs sy = sa;
  sy.S = 1;
  sy.tiles_per_split = n_vtiles;
  sy.tau = tau;
  sy.cs_j = cs_j;
  sy.cs_i = cs_i;
  sy.cs_v = cs_v;
  sy.cs_next = next;
  sy.cs_cap = (int)cap;
  sy.cs_chunk = chunk;
  sy.cs_fill = fill;
  sy.cs_overflow = flag;
  hipEvent_t t0 = timing_start(c);
  sweepS<<<dim3((unsigned)gx, 1), dim3(SW_THREADS), 0, st>>>(sy);
  timing_stop(c, t0);
  // 3. group the column side by row
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, (unsigned*)per_row,
                     (int)n);
  hipLaunchKernelGGL(cs_count_kernel, dim3((unsigned)chunks), dim3(256), 0, st, (const int*)cs_j,
                     (const int*)fill, chunk, n, per_row);
  const int nb = (int)ceil_div(n, 1024);
  hipLaunchKernelGGL(rows_block_sum_kernel, dim3((unsigned)nb), dim3(1024), 0, st, (const int*)per_row, n, bsum);
  hipLaunchKernelGGL(rows_base_scan_kernel, dim3(1), dim3(1024), 0, st, bsum, nb, off + n, info);
  hipLaunchKernelGGL(rows_offsets_kernel, dim3((unsigned)nb), dim3(1024), 0, st, (const int*)per_row, n,
                     (const long long*)bsum, off);
  GMGM_HIP(c, hipGetLastError());
  long long h[1];
  int hf = 0;
  GMGM_HIP(c, hipMemcpyAsync(h, info, 8, hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipMemcpyAsync(&hf, flag, 4, hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipStreamSynchronize(st));
  // executed MFMA work: the bound pass over its tiles, the symmetric sweep
  // over the column tiles from each workgroup's first row tile on
  const double per_tile = 2.0 * 32.0 * 32.0 * kpad;
  double tiles = (double)sa.n_wtiles * (double)ceil_div(n_vtiles, SYM_STRIDE);
  for (int64_t b = 0; b < gx; ++b) {
    const int64_t t_lo = b * SW_WAVES * 2;
    const int64_t wt = std::min<int64_t>(SW_WAVES * 2, sa.n_wtiles - t_lo);
    tiles += (double)wt * (double)(n_vtiles - t_lo);
  }
  *flops = per_tile * tiles;
  if (hf) {
    *overflow = true;
    return GMGM_OK;
  }
  void* w2;
  const long long tot = std::max<long long>(h[0], 1);
  GMGM_TRY(ws_get(c, WS_SYM2, (size_t)tot * 8, &w2));
  int* xidx = (int*)w2;
  float* xval = (float*)(xidx + tot);
  hipLaunchKernelGGL(cs_scatter_kernel, dim3((unsigned)chunks), dim3(256), 0, st, (const int*)cs_j,
                     (const int*)cs_i, (const float*)cs_v, (const int*)fill, chunk, n, (const int64_t*)off, per_row,
                     xidx, xval);
  GMGM_HIP(c, hipGetLastError());
  out->tau = tau;
  out->off = off;
  out->xidx = xidx;
  out->xval = xval;
  *overflow = false;
  return GMGM_OK;
}

static gmgm_status topk_impl(gmgm_ctx* c, int64_t n, int64_t r, const float* V, const double* psi,
                             int64_t row_begin, int64_t row_end, int32_t k, int prec, int C, int smax,
                             int64_t* row_ptr_out, int32_t* col_out, float* val_out, gmgm_topk_stats* stats,
                             bool allow_sym) {
  GMGM_HIP(c, hipSetDevice(c->device));
  if (!topk_fast_path(r, k, C))
    return topk_general(c, n, r, V, psi, row_begin, row_end, k, prec, C, smax, row_ptr_out, col_out, val_out,
                        stats);
  hipStream_t st = c->stream;
  const bool sym = allow_sym && sym_wanted(c, prec, n, row_begin, row_end);

  const int kpad = kpad_for(prec, (int)r);
  SweepFn sweep = pick_sweep(prec, kpad, C);
  if (!sweep) return set_err(c, GMGM_E_SHAPE, "no sweep variant for r = %lld", (long long)r);
  const int TI = ti_for(prec, C);
  const int units = kpad / chunk_elems(prec) / 2;
  const int64_t rows = row_end - row_begin;
  const int n_vtiles = (int)ceil_div(n, 32);
  const int rt_begin = (int)(row_begin / 32);
  const int rt_end = (int)ceil_div(row_end, 32);
  const int n_wtiles = rt_end - rt_begin;
  const int64_t w_lo = (int64_t)rt_begin * 32;
  const int64_t w_rows = (int64_t)n_wtiles * 32;
  const int64_t gx = ceil_div(n_wtiles, (int64_t)SW_WAVES * TI);
  const int S = sym ? 1 : pick_splits(gx, n_vtiles, smax, 1024);
  const int tps = (int)ceil_div(n_vtiles, S);

  // ---- workspace
  void *vp, *norms, *misc, *lists, *scl;
  GMGM_TRY(ws_get(c, WS_VP, (size_t)n_vtiles * units * 64 * 16, &vp));
  GMGM_TRY(ws_get(c, WS_NORMS, (size_t)n * 4 + (size_t)w_rows * 12 + 256, &norms));
  GMGM_TRY(ws_get(c, WS_MISC, 256, &misc));
  GMGM_TRY(ws_get(c, WS_FALLBACK, (size_t)rows * 8 + 64, &lists));
  GMGM_TRY(ws_get(c, WS_SCALES, ((size_t)n_vtiles + (size_t)w_rows) * 4 + 64, &scl));
  StageBufs A;
  const int nsub = sweep_nsub(TI);
  GMGM_TRY(stage_buffers(c, WS_WP, WS_CAND, n_wtiles, units, rows, S, nsub, C, &A));
  A.vp = (const u32x4*)vp;
  float* vrowmax = (float*)norms;
  double* wnorm = (double*)((char*)norms + (((size_t)n * 4 + 15) & ~(size_t)15));
  float* wrowmax = (float*)(wnorm + w_rows);
  unsigned* vmax_bits = (unsigned*)misc;
  int* cnt1 = (int*)((char*)misc + 16);
  int* cnt2 = (int*)((char*)misc + 20);
  unsigned long long* counters = (unsigned long long*)((char*)misc + 32);
  int* list1 = (int*)lists;
  int* list2 = list1 + rows;
  int* ev = (int*)scl;
  int* ew = ev + n_vtiles;

  // ---- stage A: prep, repack, sweep in `prec`, certify
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, (unsigned*)misc, 16);
  const int prep_blocks = (int)std::min<int64_t>(ceil_div(n, 4), 4096);
  hipLaunchKernelGGL(prep_kernel, dim3(prep_blocks), dim3(256), 0, st, V, psi, n, (int)r, w_lo,
                     std::min<int64_t>(n, w_lo + w_rows), vrowmax, wnorm, wrowmax, vmax_bits,
                     c->dev_status);
  if (prec == P_FP8) {
    const int64_t m = std::max<int64_t>(n_vtiles, w_rows);
    hipLaunchKernelGGL(fp8_exps_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, vrowmax,
                       n, n_vtiles, wrowmax, w_rows, ev, ew);
  }
  const int nch = kpad / chunk_elems(prec);
  launch_repack(prec, [&](auto kern) {
    const int64_t tv = (int64_t)n_vtiles * 32 * nch, tw = w_rows * nch;
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(tv, 256)), dim3(256), 0, st, V, psi, (int64_t)0,
                       n, (int64_t)n_vtiles * 32, (int)r, kpad, false, ev, true, (const int*)nullptr,
                       (const int*)nullptr, (u32x4*)vp);
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(tw, 256)), dim3(256), 0, st, V, psi, w_lo, n,
                       w_rows, (int)r, kpad, true, ew, false, (const int*)nullptr,
                       (const int*)nullptr, (u32x4*)A.wp);
  });
  SweepArgs sa{};
  sa.Vp = A.vp;
  sa.Wp = A.wp;
  sa.ev = ev;
  sa.ew = ew;
  sa.cval = A.cval;
  sa.cidx = A.cidx;
  sa.row_list = nullptr;
  sa.row_count = nullptr;
  sa.n = n;
  sa.n_vtiles = n_vtiles;
  sa.n_wtiles = n_wtiles;
  sa.row0 = w_lo;
  sa.row_begin = row_begin;
  sa.row_end = row_end;
  sa.S = S;
  sa.tiles_per_split = tps;
  sa.wnorm = wnorm;
  sa.vmax_bits = vmax_bits;
  sa.w_lo = w_lo;
  sa.cprec = cprec_for(prec, kpad);
  sa.k = k;
  double flops = 0.0;
  SymBufs symb{};
  if (sym) {
    bool overflow = false;
    GMGM_TRY(sym_sweep(c, sa, V, psi, (int)r, kpad, C, gx, &symb, &flops, &overflow));
    if (overflow)   // the column side outgrew its buffers: the full sweep instead
      return topk_impl(c, n, r, V, psi, row_begin, row_end, k, prec, C, smax, row_ptr_out, col_out, val_out,
                       stats, false);
  } else {
    hipEvent_t t0 = timing_start(c);
    sweep<<<dim3((unsigned)gx, (unsigned)S), dim3(SW_THREADS), 0, st>>>(sa);
    timing_stop(c, t0);
    flops = 2.0 * (double)w_rows * 32.0 * n_vtiles * kpad;
  }

  FinalArgs fa{};
  fa.cval = A.cval;
  fa.cidx = A.cidx;
  fa.V = V;
  fa.psi = psi;
  fa.wnorm = wnorm;
  fa.vmax_bits = vmax_bits;
  fa.n = n;
  fa.r = (int)r;
  fa.k = k;
  fa.C = C;
  fa.S = S;
  fa.nsub = nsub;
  fa.row_begin = row_begin;
  fa.rows = rows;
  fa.w_lo = w_lo;
  fa.row_list = nullptr;
  fa.row_count = nullptr;
  fa.cprec = cprec_for(prec, kpad);
  fa.col_out = col_out;
  fa.val_out = val_out;
  fa.fail_list = list1;
  fa.fail_count = cnt1;
  fa.counters = stats ? counters : nullptr;   // counted only when asked for
  if (sym) {
    fa.xoff = (const long long*)symb.off;
    fa.xidx = symb.xidx;
    fa.xval = symb.xval;
    fa.tau = symb.tau;
  }
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)ceil_div(rows, 4)), dim3(256), 0, st, fa);
  hipLaunchKernelGGL(row_ptr_kernel, dim3((unsigned)ceil_div(rows + 1, 256)), dim3(256), 0, st,
                     row_ptr_out, rows, k);
  GMGM_HIP(c, hipGetLastError());

  // ---- stage B: rows stage A could not certify are re-swept with finer operands
  int h1 = 0, h2 = 0;
  GMGM_HIP(c, hipMemcpyAsync(&h1, cnt1, 4, hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipStreamSynchronize(st));
  if (h1 > 0) {
    // FP32 operands after an FP32 sweep; after a BF16 / FP8 sweep split BF16
    // (three BF16 MFMAs per K step, about 4x FP32's rounding bound)
    const int CB = k <= 12 ? 16 : 32;
    const int precB = prec == P_F32 ? P_F32 : P_BF16X3;
    const int kpadB = kpad_for(precB, (int)r);
    const int unitsB = units_for(precB, kpadB);
    SweepFn sweepB = precB == P_F32 ? pick_sweep(P_F32, kpadB, CB) : pick_sweep_bf16x3(kpadB, CB);
    const int TIB = ti_for(precB, CB);
    const int64_t wtB = ceil_div(h1, 32);
    const int64_t gxB = ceil_div(wtB, (int64_t)SW_WAVES * TIB);
    const int SB = pick_splits(gxB, n_vtiles, 64, 1024);
    const int tpsB = (int)ceil_div(n_vtiles, SB);
    StageBufs B;
    const int nsubB = sweep_nsub(TIB);
    void* vpb = nullptr;
    gmgm_status sB = stage_buffers(c, WS_WP2, WS_CAND2, wtB, unitsB, h1, SB, nsubB, CB, &B);
    if (sB == GMGM_OK && !sweepB) sB = set_err(c, GMGM_E_SHAPE, "no re-sweep variant for r = %lld", (long long)r);
    if (sB == GMGM_OK && !(prec == P_F32 && kpadB == kpad))
      sB = ws_get(c, WS_VP2, (size_t)n_vtiles * unitsB * 64 * 16, &vpb);
    if (sB != GMGM_OK) {
      // only a fixed arena can run out here: the uncertified rows then go
      // straight to the exact scan (same result, no re-sweep buffers)
      if (!c->arena) return sB;
      c->err.clear();
      hipLaunchKernelGGL(exact_scan_kernel, dim3((unsigned)std::min(h1, 4096)), dim3(256), 0, st, V, psi, n,
                         (int)r, k, row_begin, list1, cnt1, col_out, val_out);
      GMGM_HIP(c, hipGetLastError());
      if (stats) {
        unsigned long long hc[2];
        GMGM_HIP(c, hipMemcpyAsync(hc, counters, 16, hipMemcpyDeviceToHost, st));
        GMGM_HIP(c, hipStreamSynchronize(st));
        stats->cand_total = (int64_t)hc[0];
        stats->rows_near_tie = (int64_t)hc[1];
        stats->rows_fallback = h1;
        stats->rows_exact = h1;
        stats->mfma_flops = flops;
        stats->symmetric = 0;
      }
      return GMGM_OK;
    }
    if (prec == P_F32 && kpadB == kpad) {
      B.vp = A.vp;
    } else {
      B.vp = (const u32x4*)vpb;
      const int64_t tv = (int64_t)n_vtiles * 32 * (kpadB / chunk_elems(precB));
      hipLaunchKernelGGL(precB == P_F32 ? repack_kernel<P_F32> : repack_kernel<P_BF16X3>,
                         dim3((unsigned)ceil_div(tv, 256)), dim3(256), 0, st, V, psi, (int64_t)0, n,
                         (int64_t)n_vtiles * 32, (int)r, kpadB, false, ev, true, (const int*)nullptr,
                         (const int*)nullptr, (u32x4*)vpb);
    }
    const int64_t twB = wtB * 32 * (kpadB / chunk_elems(precB));
    hipLaunchKernelGGL(precB == P_F32 ? repack_kernel<P_F32> : repack_kernel<P_BF16X3>,
                       dim3((unsigned)ceil_div(twB, 256)), dim3(256), 0, st, V, psi, (int64_t)0, n, wtB * 32,
                       (int)r, kpadB, true, ew, false, (const int*)list1, (const int*)cnt1, (u32x4*)B.wp);
    SweepArgs sb = sa;
    sb.Vp = B.vp;
    sb.Wp = B.wp;
    sb.cval = B.cval;
    sb.cidx = B.cidx;
    sb.row_list = list1;
    sb.row_count = cnt1;
    sb.n_wtiles = (int)wtB;
    sb.S = SB;
    sb.tiles_per_split = tpsB;
    sb.cprec = cprec_for(precB, kpadB);
    sweepB<<<dim3((unsigned)gxB, (unsigned)SB), dim3(SW_THREADS), 0, st>>>(sb);
    FinalArgs fb = fa;
    fb.xoff = nullptr;   // whole rows: no symmetric-form extras
    fb.xidx = nullptr;
    fb.xval = nullptr;
    fb.tau = nullptr;
    fb.cval = B.cval;
    fb.cidx = B.cidx;
    fb.C = CB;
    fb.S = SB;
    fb.nsub = nsubB;
    fb.row_list = list1;
    fb.row_count = cnt1;
    fb.cprec = cprec_for(precB, kpadB);
    fb.fail_list = list2;
    fb.fail_count = cnt2;
    fb.counters = stats ? counters + 2 : nullptr;   // stage-B candidates are not counted with stage A's
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)ceil_div(h1, 4)), dim3(256), 0, st, fb);
    GMGM_HIP(c, hipGetLastError());
    flops += (precB == P_F32 ? 2.0 : 6.0) * (double)wtB * 32.0 * n_vtiles * 32.0 * kpadB;
    GMGM_HIP(c, hipMemcpyAsync(&h2, cnt2, 4, hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    // ---- stage C: rows still uncertified (exact ties at the boundary, non-finite inputs)
    if (h2 > 0) {
      hipLaunchKernelGGL(exact_scan_kernel, dim3((unsigned)std::min(h2, 4096)), dim3(256), 0, st, V,
                         psi, n, (int)r, k, row_begin, list2, cnt2, col_out, val_out);
      GMGM_HIP(c, hipGetLastError());
    }
  }
  if (stats) {
    unsigned long long hc[2];
    GMGM_HIP(c, hipMemcpyAsync(hc, counters, 16, hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    stats->cand_total = (int64_t)hc[0];
    stats->rows_near_tie = (int64_t)hc[1];
    stats->rows_fallback = h1;
    stats->rows_exact = h2;
    stats->mfma_flops = flops;
    stats->symmetric = sym ? 1 : 0;
  }
  return GMGM_OK;
}

// The K-loop path: prep, repack (contraction padded to a multiple of 32), the
// K-loop sweep, exact rescoring and certificate; uncertified rows of a BF16
// sweep are re-swept in FP32; rows that still fail get exact FP64 panels.
static gmgm_status topk_general(gmgm_ctx* c, int64_t n, int64_t r, const float* V, const double* psi,
                                int64_t row_begin, int64_t row_end, int32_t k, int prec_in, int C, int smax,
                                int64_t* row_ptr_out, int32_t* col_out, float* val_out, gmgm_topk_stats* stats) {
  hipStream_t st = c->stream;
  const int prec = kl_prec(prec_in, r);
  const int kpad = kl_kpad(r);
  const int units = kpad / chunk_elems(prec) / 2;
  const int64_t rows = row_end - row_begin;
  const int n_vtiles = (int)ceil_div(n, 32);
  const int rt_begin = (int)(row_begin / 32);
  const int n_wtiles = (int)ceil_div(row_end, 32) - rt_begin;
  const int64_t w_lo = (int64_t)rt_begin * 32;
  const int64_t w_rows = (int64_t)n_wtiles * 32;
  const int64_t gx = ceil_div(n_wtiles, (int64_t)KL_WAVES * 2);
  const int S = pick_splits(gx, n_vtiles, smax, 1024);
  const int tps = (int)ceil_div(n_vtiles, S);

  void *vp, *norms, *misc, *lists, *wp, *cand;
  GMGM_TRY(ws_get(c, WS_VP, (size_t)n_vtiles * units * 64 * 16, &vp));
  GMGM_TRY(ws_get(c, WS_NORMS, (size_t)n * 4 + (size_t)w_rows * 12 + 256, &norms));
  GMGM_TRY(ws_get(c, WS_MISC, 256, &misc));
  GMGM_TRY(ws_get(c, WS_FALLBACK, (size_t)rows * 8 + 64, &lists));
  GMGM_TRY(ws_get(c, WS_WP, (size_t)n_wtiles * units * 64 * 16, &wp));
  const size_t ncand = (size_t)rows * S * C;
  GMGM_TRY(ws_get(c, WS_CAND, ncand * 8, &cand));
  float* vrowmax = (float*)norms;
  double* wnorm = (double*)((char*)norms + (((size_t)n * 4 + 15) & ~(size_t)15));
  float* wrowmax = (float*)(wnorm + w_rows);
  unsigned* vmax_bits = (unsigned*)misc;
  int* cnt1 = (int*)((char*)misc + 16);
  int* cnt2 = (int*)((char*)misc + 20);
  unsigned long long* counters = (unsigned long long*)((char*)misc + 32);
  int* list1 = (int*)lists;
  int* list2 = list1 + rows;

  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, (unsigned*)misc, 16);
  const int prep_blocks = (int)std::min<int64_t>(ceil_div(n, 4), 4096);
  hipLaunchKernelGGL(prep_kernel, dim3(prep_blocks), dim3(256), 0, st, V, psi, n, (int)r, w_lo,
                     std::min<int64_t>(n, w_lo + w_rows), vrowmax, wnorm, wrowmax, vmax_bits, c->dev_status);
  const int nch = kpad / chunk_elems(prec);
  launch_repack(prec, [&](auto kern) {
    const int64_t tv = (int64_t)n_vtiles * 32 * nch, tw = w_rows * nch;
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(tv, 256)), dim3(256), 0, st, V, psi, (int64_t)0, n,
                       (int64_t)n_vtiles * 32, (int)r, kpad, false, (const int*)nullptr, true, (const int*)nullptr,
                       (const int*)nullptr, (u32x4*)vp);
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(tw, 256)), dim3(256), 0, st, V, psi, w_lo, n, w_rows,
                       (int)r, kpad, true, (const int*)nullptr, false, (const int*)nullptr, (const int*)nullptr,
                       (u32x4*)wp);
  });
  KloopArgs ka{};
  ka.Vp = (const u32x4*)vp;
  ka.Wp = (const u32x4*)wp;
  ka.cval = (float*)cand;
  ka.cidx = (int*)((char*)cand + ncand * 4);
  ka.n = n;
  ka.n_vtiles = n_vtiles;
  ka.n_wtiles = n_wtiles;
  ka.units = units;
  ka.row0 = w_lo;
  ka.row_begin = row_begin;
  ka.row_end = row_end;
  ka.S = S;
  ka.tiles_per_split = tps;
  ka.wnorm = wnorm;
  ka.vmax_bits = vmax_bits;
  ka.w_lo = w_lo;
  ka.cprec = cprec_for(prec, kpad);
  ka.k = k;
  hipEvent_t t0 = timing_start(c);
  launch_sweep_kloop(prec, C, gx, S, st, ka);
  timing_stop(c, t0);
  FinalGenArgs fa{};
  fa.cval = ka.cval;
  fa.cidx = ka.cidx;
  fa.V = V;
  fa.psi = psi;
  fa.wnorm = wnorm;
  fa.vmax_bits = vmax_bits;
  fa.n = n;
  fa.r = (int)r;
  fa.k = k;
  fa.C = C;
  fa.S = S;
  fa.row_begin = row_begin;
  fa.rows = rows;
  fa.w_lo = w_lo;
  fa.cprec = ka.cprec;
  fa.col_out = col_out;
  fa.val_out = val_out;
  fa.fail_list = list1;
  fa.fail_count = cnt1;
  fa.counters = stats ? counters : nullptr;
  launch_finalize_gen(rows, st, fa);
  hipLaunchKernelGGL(row_ptr_kernel, dim3((unsigned)ceil_div(rows + 1, 256)), dim3(256), 0, st, row_ptr_out, rows,
                     k);
  GMGM_HIP(c, hipGetLastError());
  double flops = 2.0 * (double)w_rows * 32.0 * n_vtiles * kpad;

  int h1 = 0, h2 = 0;
  GMGM_HIP(c, hipMemcpyAsync(&h1, cnt1, 4, hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipStreamSynchronize(st));
  const int* exact_list = list1;
  int h_exact = h1;
  if (h1 > 0 && prec != P_F32 && !c->arena) {
    // FP32 re-sweep of the rows the BF16 sweep could not certify (with a fixed
    // arena the rows go straight to the exact panels, which need less room)
    const int unitsB = kpad / chunk_elems(P_F32) / 2;
    const int64_t wtB = ceil_div(h1, 32);
    const int64_t gxB = ceil_div(wtB, (int64_t)KL_WAVES * 2);
    const int SB = pick_splits(gxB, n_vtiles, 64, 1024);
    const size_t ncandB = (size_t)h1 * SB * C;
    void *vpb, *wpb, *candb;
    GMGM_TRY(ws_get(c, WS_VP2, (size_t)n_vtiles * unitsB * 64 * 16, &vpb));
    GMGM_TRY(ws_get(c, WS_WP2, (size_t)wtB * unitsB * 64 * 16, &wpb));
    GMGM_TRY(ws_get(c, WS_CAND2, ncandB * 8, &candb));
    {
      const int64_t tv = (int64_t)n_vtiles * 32 * (kpad / 4), twB = wtB * 32 * (kpad / 4);
      hipLaunchKernelGGL(repack_kernel<P_F32>, dim3((unsigned)ceil_div(tv, 256)), dim3(256), 0, st, V, psi,
                         (int64_t)0, n, (int64_t)n_vtiles * 32, (int)r, kpad, false, (const int*)nullptr, true,
                         (const int*)nullptr, (const int*)nullptr, (u32x4*)vpb);
      hipLaunchKernelGGL(repack_kernel<P_F32>, dim3((unsigned)ceil_div(twB, 256)), dim3(256), 0, st, V, psi,
                         (int64_t)0, n, wtB * 32, (int)r, kpad, true, (const int*)nullptr, false,
                         (const int*)list1, (const int*)cnt1, (u32x4*)wpb);
      KloopArgs kb = ka;
      kb.Vp = (const u32x4*)vpb;
      kb.Wp = (const u32x4*)wpb;
      kb.cval = (float*)candb;
      kb.cidx = (int*)((char*)candb + ncandB * 4);
      kb.row_list = list1;
      kb.row_count = cnt1;
      kb.n_wtiles = (int)wtB;
      kb.units = unitsB;
      kb.S = SB;
      kb.tiles_per_split = (int)ceil_div(n_vtiles, SB);
      kb.cprec = cprec_for(P_F32, kpad);
      launch_sweep_kloop(P_F32, C, gxB, SB, st, kb);
      FinalGenArgs fb = fa;
      fb.cval = kb.cval;
      fb.cidx = kb.cidx;
      fb.S = SB;
      fb.row_list = list1;
      fb.row_count = cnt1;
      fb.cprec = kb.cprec;
      fb.fail_list = list2;
      fb.fail_count = cnt2;
      fb.counters = stats ? counters + 2 : nullptr;
      launch_finalize_gen(h1, st, fb);
      GMGM_HIP(c, hipGetLastError());
      flops += 2.0 * (double)wtB * 32.0 * n_vtiles * 32.0 * kpad;
      GMGM_HIP(c, hipMemcpyAsync(&h2, cnt2, 4, hipMemcpyDeviceToHost, st));
      GMGM_HIP(c, hipStreamSynchronize(st));
      exact_list = list2;
      h_exact = h2;
    }
  }
  if (h_exact > 0) {
    // exact FP64 values of whole rows, a panel of rows at a time
    const size_t row_bytes = (size_t)n * 8;
    size_t room = (size_t)256 << 20;
    if (c->arena) room = c->arena_bytes - std::min(c->arena_bytes, ((c->arena_top + 255) & ~(size_t)255));
    const int64_t prow = std::max<int64_t>(1, std::min<int64_t>(h_exact, (int64_t)(room / row_bytes)));
    void* panel;
    GMGM_TRY(ws_get(c, WS_THR0, (size_t)prow * row_bytes, &panel));
    for (int64_t q0 = 0; q0 < h_exact; q0 += prow) {
      const int pr = (int)std::min<int64_t>(prow, h_exact - q0);
      launch_exact_panel(V, psi, n, (int)r, exact_list, (int)q0, pr, (double*)panel, st);
      launch_panel_topk((const double*)panel, n, exact_list, (int)q0, pr, k, row_begin, col_out, val_out, st);
    }
    GMGM_HIP(c, hipGetLastError());
  }
  if (stats) {
    unsigned long long hc[2];
    GMGM_HIP(c, hipMemcpyAsync(hc, counters, 16, hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    stats->cand_total = (int64_t)hc[0];
    stats->rows_near_tie = (int64_t)hc[1];
    stats->rows_fallback = h1;
    stats->rows_exact = h_exact;
    stats->mfma_flops = flops;
    stats->symmetric = 0;
  }
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_recompose_threshold(gmgm_ctx_t c, int64_t n, int64_t r, const float* V,
                                                const double* psi, int64_t row_begin, int64_t row_end,
                                                double thr, gmgm_prec prec_e, int32_t max_per_row,
                                                int64_t* row_ptr_out, int32_t* col_out, float* val_out,
                                                int64_t capacity, int64_t* nnz_out) {
  GMGM_CHECK_CTX(c);
  const int prec = (int)prec_e;
  if (prec < 0 || prec > 2) return set_err(c, GMGM_E_ARG, "unknown precision %d", prec);
  if (n < 2 || n > 0x7fffffc0LL) return set_err(c, GMGM_E_SHAPE, "n = %lld out of range [2, 2^31 - 64]", (long long)n);
  if (r < 1 || r > 128) return set_err(c, GMGM_E_SHAPE, "r = %lld must be in [1, 128]", (long long)r);
  if (row_begin < 0 || row_end > n || row_begin >= row_end)
    return set_err(c, GMGM_E_SHAPE, "row range [%lld, %lld) invalid for n = %lld",
                   (long long)row_begin, (long long)row_end, (long long)n);
  if (!(thr > 0.0) || !std::isfinite(thr)) return set_err(c, GMGM_E_DOMAIN, "thr must be positive and finite");
  if (capacity < 0 || !V || !psi || !row_ptr_out || !nnz_out || (capacity > 0 && (!col_out || !val_out)))
    return set_err(c, GMGM_E_ARG, "null pointer or negative capacity");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;

  const int kpad = kpad_for(prec, (int)r);
  SweepFn sweep = pick_sweep_thr(prec, kpad);
  if (!sweep) return set_err(c, GMGM_E_SHAPE, "no sweep variant for r = %lld", (long long)r);
  const int TI = 2;                       // pair mode: one whole row per lane
  const int units = kpad / chunk_elems(prec) / 2;
  const int64_t rows = row_end - row_begin;
  const int n_vtiles = (int)ceil_div(n, 32);
  const int rt_begin = (int)(row_begin / 32);
  const int n_wtiles = (int)ceil_div(row_end, 32) - rt_begin;
  const int64_t w_lo = (int64_t)rt_begin * 32;
  const int64_t w_rows = (int64_t)n_wtiles * 32;
  const int64_t gx = ceil_div(n_wtiles, (int64_t)SW_WAVES * TI);
  // one column split, so that each row's candidates come out in column order
  const int S = 1;
  const long long pool_cap = std::max<long long>(capacity, 1);

  void *vp, *norms, *misc, *scl, *pool, *aux;
  GMGM_TRY(ws_get(c, WS_VP, (size_t)n_vtiles * units * 64 * 16, &vp));
  GMGM_TRY(ws_get(c, WS_NORMS, (size_t)n * 4 + (size_t)w_rows * 12 + 256, &norms));
  GMGM_TRY(ws_get(c, WS_MISC, 256, &misc));
  GMGM_TRY(ws_get(c, WS_SCALES, ((size_t)n_vtiles + (size_t)w_rows) * 4 + 64, &scl));
  GMGM_TRY(ws_get(c, WS_THR0, (size_t)pool_cap * 8, &pool));
  GMGM_TRY(ws_get(c, WS_THR1, (size_t)rows * 24 + 64, &aux));
  StageBufs A;
  GMGM_TRY(stage_buffers(c, WS_WP, WS_CAND, n_wtiles, units, rows, S, 1, THR_CAPT, &A));
  A.vp = (const u32x4*)vp;
  float* vrowmax = (float*)norms;
  double* wnorm = (double*)((char*)norms + (((size_t)n * 4 + 15) & ~(size_t)15));
  float* wrowmax = (float*)(wnorm + w_rows);
  unsigned* vmax_bits = (unsigned*)misc;
  int* fail_count = (int*)((char*)misc + 16);
  long long* pool_top = (long long*)((char*)misc + 32);
  long long* info = (long long*)((char*)misc + 64);
  int* ev = (int*)scl;
  int* ew = ev + n_vtiles;
  long long* pool_off = (long long*)aux;
  int* tcount = (int*)(pool_off + rows);
  int* kept_n = tcount + rows;
  int* fail_list = kept_n + rows;
  int* fail_rows = fail_list + rows;
  int* fail_count2 = (int*)((char*)misc + 20);
  int* pool_j = (int*)pool;
  float* pool_v = (float*)((char*)pool + (size_t)pool_cap * 4);

  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, st, (unsigned*)misc, 32);
  const int prep_blocks = (int)std::min<int64_t>(ceil_div(n, 4), 4096);
  hipLaunchKernelGGL(prep_kernel, dim3(prep_blocks), dim3(256), 0, st, V, psi, n, (int)r, w_lo,
                     std::min<int64_t>(n, w_lo + w_rows), vrowmax, wnorm, wrowmax, vmax_bits,
                     c->dev_status);
  if (prec == P_FP8) {
    const int64_t m = std::max<int64_t>(n_vtiles, w_rows);
    hipLaunchKernelGGL(fp8_exps_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, vrowmax,
                       n, n_vtiles, wrowmax, w_rows, ev, ew);
  }
  const int nch = kpad / chunk_elems(prec);
  launch_repack(prec, [&](auto kern) {
    const int64_t tv = (int64_t)n_vtiles * 32 * nch, tw = w_rows * nch;
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(tv, 256)), dim3(256), 0, st, V, psi, (int64_t)0,
                       n, (int64_t)n_vtiles * 32, (int)r, kpad, false, ev, true, (const int*)nullptr,
                       (const int*)nullptr, (u32x4*)vp);
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(tw, 256)), dim3(256), 0, st, V, psi, w_lo, n,
                       w_rows, (int)r, kpad, true, ew, false, (const int*)nullptr,
                       (const int*)nullptr, (u32x4*)A.wp);
  });
  SweepArgs sa{};
  sa.Vp = A.vp;
  sa.Wp = A.wp;
  sa.ev = ev;
  sa.ew = ew;
  sa.cval = A.cval;
  sa.cidx = A.cidx;
  sa.n = n;
  sa.n_vtiles = n_vtiles;
  sa.n_wtiles = n_wtiles;
  sa.row0 = w_lo;
  sa.row_begin = row_begin;
  sa.row_end = row_end;
  sa.S = S;
  sa.tiles_per_split = n_vtiles;
  sa.wnorm = wnorm;
  sa.vmax_bits = vmax_bits;
  sa.w_lo = w_lo;
  sa.cprec = cprec_for(prec, kpad);
  sa.k = 1;
  sa.thr = thr;
  sa.capt = THR_CAPT;
  sa.tcount = tcount;
  hipEvent_t t0 = timing_start(c);
  sweep<<<dim3((unsigned)gx, 1), dim3(SW_THREADS), 0, st>>>(sa);
  timing_stop(c, t0);
  GMGM_HIP(c, hipGetLastError());

  ThrArgs ta{};
  ta.V = V;
  ta.psi = psi;
  ta.n = n;
  ta.r = (int)r;
  ta.thr = thr;
  ta.row_begin = row_begin;
  ta.rows = rows;
  ta.cidx = A.cidx;
  ta.tcount = tcount;
  ta.list = nullptr;
  ta.toff = nullptr;
  ta.fail_rows = fail_rows;
  ta.pool_j = pool_j;
  ta.pool_v = pool_v;
  ta.pool_cap = capacity;
  ta.pool_top = pool_top;
  ta.pool_off = pool_off;
  ta.kept_n = kept_n;
  ta.fail_list = fail_list;
  ta.fail_count = fail_count;
  hipLaunchKernelGGL(thr_verify_kernel, dim3((unsigned)ceil_div(rows, 4)), dim3(256), 0, st, ta);
  int h_fail = 0;
  GMGM_HIP(c, hipMemcpyAsync(&h_fail, fail_count, 4, hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipStreamSynchronize(st));
  if (h_fail > 0) {
    // ---- rows with more candidates than the sweep's room: re-swept as a
    // list, with room for exactly the candidates the first sweep counted
    // (BF16 operands when the first sweep used FP8, whose per-row scales are
    // not kept for listed rows)
    void* auxB;
    GMGM_TRY(ws_get(c, WS_THR2, (size_t)h_fail * 12 + (size_t)(h_fail + 1) * 8 + 64, &auxB));
    long long* toffB = (long long*)auxB;
    int* cntB = (int*)(toffB + h_fail + 1);
    int* tcountB = cntB + h_fail;
    int* fail2 = tcountB + h_fail;
    long long* infoB = info + 2;
    hipLaunchKernelGGL(thr_counts_kernel, dim3((unsigned)ceil_div(h_fail, 256)), dim3(256), 0, st, fail_list,
                       h_fail, tcount, cntB);
    hipLaunchKernelGGL(thr_scan_kernel, dim3(1), dim3(1024), 0, st, cntB, (int64_t)h_fail, (int64_t*)toffB, infoB);
    long long totB = 0;
    GMGM_HIP(c, hipMemcpyAsync(&totB, infoB, 8, hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    const int precB = prec == P_F32 ? P_F32 : P_BF16;
    const int kpadB = kpad_for(precB, (int)r);
    const int unitsB = kpadB / chunk_elems(precB) / 2;
    SweepFn sweepB = pick_sweep_thr(precB, kpadB);
    if (!sweepB) return set_err(c, GMGM_E_SHAPE, "no sweep variant for r = %lld", (long long)r);
    void *candB, *wpB;
    GMGM_TRY(ws_get(c, WS_CAND2, (size_t)std::max<long long>(totB, 1) * 8, &candB));
    const int64_t wtB = ceil_div(h_fail, 32);
    GMGM_TRY(ws_get(c, WS_WP2, (size_t)wtB * unitsB * 64 * 16, &wpB));
    const u32x4* vpB = A.vp;
    if (precB != prec) {
      void* v2;
      GMGM_TRY(ws_get(c, WS_VP2, (size_t)n_vtiles * unitsB * 64 * 16, &v2));
      const int64_t tv = (int64_t)n_vtiles * 32 * (kpadB / chunk_elems(precB));
      hipLaunchKernelGGL(repack_kernel<P_BF16>, dim3((unsigned)ceil_div(tv, 256)), dim3(256), 0, st, V, psi,
                         (int64_t)0, n, (int64_t)n_vtiles * 32, (int)r, kpadB, false, ev, true, (const int*)nullptr,
                         (const int*)nullptr, (u32x4*)v2);
      vpB = (const u32x4*)v2;
    }
    const int64_t twB = wtB * 32 * (kpadB / chunk_elems(precB));
    if (precB == P_F32)
      hipLaunchKernelGGL(repack_kernel<P_F32>, dim3((unsigned)ceil_div(twB, 256)), dim3(256), 0, st, V, psi,
                         (int64_t)0, n, wtB * 32, (int)r, kpadB, true, ew, false, (const int*)fail_rows,
                         (const int*)fail_count, (u32x4*)wpB);
    else
      hipLaunchKernelGGL(repack_kernel<P_BF16>, dim3((unsigned)ceil_div(twB, 256)), dim3(256), 0, st, V, psi,
                         (int64_t)0, n, wtB * 32, (int)r, kpadB, true, ew, false, (const int*)fail_rows,
                         (const int*)fail_count, (u32x4*)wpB);
    SweepArgs sb = sa;
    sb.Vp = vpB;
    sb.Wp = (const u32x4*)wpB;
    sb.cval = (float*)candB;
    sb.cidx = (int*)((char*)candB + (size_t)std::max<long long>(totB, 1) * 4);
    sb.row_list = fail_rows;
    sb.row_count = fail_count;
    sb.n_wtiles = (int)wtB;
    sb.cprec = cprec_for(precB, kpadB);
    sb.toff = toffB;
    sb.tcount = tcountB;
    const int64_t gxB = ceil_div(wtB, (int64_t)SW_WAVES * 2);
    hipEvent_t t1 = timing_start(c);
    sweepB<<<dim3((unsigned)gxB, 1), dim3(SW_THREADS), 0, st>>>(sb);
    timing_stop(c, t1);
    GMGM_HIP(c, hipGetLastError());
    ThrArgs tb = ta;
    tb.cidx = sb.cidx;
    tb.tcount = tcountB;
    tb.list = fail_list;
    tb.toff = toffB;
    tb.rows = h_fail;
    tb.fail_list = fail2;
    tb.fail_rows = nullptr;
    tb.fail_count = fail_count2;
    hipLaunchKernelGGL(thr_verify_kernel, dim3((unsigned)ceil_div(h_fail, 4)), dim3(256), 0, st, tb);
    // ---- rows whose listed re-sweep still overflowed: exact scan
    int h_fail2 = 0;
    GMGM_HIP(c, hipMemcpyAsync(&h_fail2, fail_count2, 4, hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    if (h_fail2 > 0)
      hipLaunchKernelGGL(thr_exact_kernel, dim3((unsigned)std::min(h_fail2, 4096)), dim3(256), 0, st, tb);
  }
  hipLaunchKernelGGL(thr_scan_kernel, dim3(1), dim3(1024), 0, st, kept_n, rows, row_ptr_out, info);
  long long h_info[2];
  GMGM_HIP(c, hipMemcpyAsync(h_info, info, 16, hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipStreamSynchronize(st));
  GMGM_TRY(gmgm_sync(c));   // non-finite inputs found by prep
  *nnz_out = (int64_t)h_info[0];
  if (max_per_row > 0 && h_info[1] > max_per_row)
    return set_err(c, GMGM_E_OVERFLOW, "a row keeps %lld entries, more than max_per_row = %d", h_info[1], max_per_row);
  if (h_info[0] > capacity)
    return set_err(c, GMGM_E_OVERFLOW, "%lld entries exceed the capacity %lld", h_info[0], (long long)capacity);
  hipLaunchKernelGGL(thr_gather_kernel, dim3((unsigned)ceil_div(rows, 4)), dim3(256), 0, st, pool_j, pool_v, pool_off,
                     kept_n, row_ptr_out, rows, col_out, val_out);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

// Upper normal quantile z with 0.5 erfc(z / sqrt 2) = p, 0 < p <= 0.5: the
// rational starting value of Abramowitz and Stegun 26.2.23, then Newton steps
// on the tail itself (quadratic convergence to double precision).
static double upper_normal_quantile(double p) {
  const double t = std::sqrt(-2.0 * std::log(p));
  double z = t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                     (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t);
  for (int it = 0; it < 8; ++it) {
    const double tail = 0.5 * std::erfc(z / std::sqrt(2.0));
    const double dens = std::exp(-0.5 * z * z) / std::sqrt(2.0 * M_PI);
    const double step = (tail - p) / dens;
    z += step;
    if (std::fabs(step) <= 1e-15 * std::fabs(z)) break;
  }
  return z;
}

extern "C" gmgm_status gmgm_significance_threshold(gmgm_ctx_t c, int64_t d_l, int32_t n_mod, const double* d_all,
                                                   const double* trace_s, double alpha, double n_tests,
                                                   double* thr_out) {
  // host arithmetic only: a null context is allowed (errors are then returned
  // without a message)
#define SIG_ERR(code, ...) (c ? set_err(c, code, __VA_ARGS__) : code)
  if (d_l < 2 || n_mod < 1 || !d_all || !trace_s || !thr_out)
    return SIG_ERR(GMGM_E_ARG, "need d_l >= 2, n_mod >= 1 and non-null arrays");
  if (!(alpha > 0.0 && alpha < 1.0)) return SIG_ERR(GMGM_E_DOMAIN, "alpha must be in (0, 1)");
  const double m = n_tests > 0.0 ? n_tests : 0.5 * (double)d_l * (double)(d_l - 1);
  double denom = 0.0;
  for (int g = 0; g < n_mod; ++g) {
    if (!(d_all[g] > 0.0) || !(trace_s[g] > 0.0) || !std::isfinite(d_all[g]) || !std::isfinite(trace_s[g]))
      return SIG_ERR(GMGM_E_DOMAIN, "modality %d: d_all and trace_s must be positive and finite", g);
    const double s2 = trace_s[g] / d_all[g];     // the null model's variance
    denom += d_all[g] * s2 * s2;
  }
  const double p = alpha / (2.0 * m);
  if (!(p > 0.0)) return SIG_ERR(GMGM_E_DOMAIN, "alpha / (2 n_tests) underflows");
  *thr_out = 2.0 * upper_normal_quantile(p) * std::sqrt((double)d_l / denom);
  return GMGM_OK;
#undef SIG_ERR
}

extern "C" gmgm_status gmgm_rounding_bound(int32_t prec, int64_t r, double* c_out, int32_t* kpad_out) {
  if (prec < 0 || prec > 2 || !c_out) return GMGM_E_ARG;
  if (r < 1 || r > TOPK_MAX_R) return GMGM_E_SHAPE;
  // r > 128 takes the K-loop sweep (FP8 requests run in BF16 there, every
  // request in FP32 above 4096)
  if (r > 128) prec = kl_prec(prec, r);
  const int kpad = r <= 128 ? kpad_for(prec, (int)r) : kl_kpad(r);
  *c_out = cprec_for(prec, kpad);
  if (kpad_out) *kpad_out = kpad;
  return GMGM_OK;
}
