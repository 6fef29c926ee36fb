// Eigenvalue maximum-likelihood estimate on the GPU (FP64).
//
// With Theorem 1's eigenvectors fixed, the model equation's negative
// log-likelihood in the eigenvalues is, for modalities gamma = (a, b),
//   NLL = 1/2 [ sum_l sum_i E_l,i lam_l,i - sum_gamma sum_{i,j} log(lam_a,i + lam_b,j) ],
// with gradient (eigenvalue-gradient Proposition)
//   dNLL/dlam_l,i = 1/2 ( E_l,i - sum_{partners m} sum_j 1/(lam_l,i + lam_m,j) ),
// and for modalities of K axes the log term sums over all index tuples of the
// tuple's eigenvalue sum; minimised over the Existence lemma's box
// lam_l,i >= eps_l.
//
// Method: projected Newton for bound constraints with a vanishing
// Levenberg-Marquardt damping rho = min(1e-2, KKT residual) and an Armijo
// search along the projection arc.  Both solvers switch after 30
// iterations to an escape mode (Bertsekas' active set with the diagonal
// h + |g|/x, as in Levenberg-Marquardt, and no limit on how far a coordinate
// may shrink per step) for directions of almost zero slope whose minimiser
// sits on the box.  The host drives the iteration; every
// arithmetic step runs in the kernels below (and rocBLAS/rocSOLVER for dense
// factorisations).  Two solvers share the driver:
//  - pairs (gmgm_solve_eigs): a Schur complement on "hub" axes (a minimum-rank
//    vertex cover of the modality graph; the other axes have diagonal Hessian
//    blocks and are eliminated), the hub system factored by a one-workgroup
//    Cholesky (rocSOLVER's above 2048 unknowns);
//  - any number of axes (gmgm_solve_eigs_tensor): batched tuple sums, the
//    Newton system held dense and solved by block elimination of each
//    modality's private axes.
// Along axis shifts with zero NLL slope the NLL is constant; the result is
// moved to the gauge of the start 1/E as far as the box allows.  A warm start
// is used when its NLL is not above that of 1/E.  Reductions are deterministic
// (fixed order, compensated).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "gmgm_internal.h"
#include "solve_host.h"

namespace gmgm_sv {

constexpr int RED_THREADS = 1024;
constexpr int MAX_AXES = 8;        // pair solver; axes of one modality (tensor solver)
constexpr int MAX_HUB = 32768;     // pair solver: unknowns of the Schur system
constexpr int CHOL_ONE_WG = 2048;  // up to this size the Schur system is factorised by one workgroup
constexpr int MAX_TAXES = 64;      // tensor solver: axes
constexpr int MAX_DENSE = 8192;    // tensor solver: unknowns of the dense Newton system

__device__ inline void neumaier(double& s, double& c, double x) {
  const double t = s + x;
  c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over a block of RED_THREADS threads (result valid in thread 0).
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < RED_THREADS / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// For every i < nx: s1[i] (+)= sum_j 1/(x_i + y_j), s2[i] (+)= sum_j (x_i + y_j)^-2 and,
// when lg is given, lg[i] (+)= sum_j log(x_i + y_j).  One wave per i.
__global__ void __launch_bounds__(256) pair_sums_kernel(const double* __restrict__ x, int nx,
                                                        const double* __restrict__ y, int ny,
                                                        double* __restrict__ s1,
                                                        double* __restrict__ s2,
                                                        double* __restrict__ lg, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nx) return;
  const double xi = x[i];
  double a1 = 0, c1 = 0, a2 = 0, c2 = 0, a3 = 0, c3 = 0;
  for (int j = lane; j < ny; j += 64) {
    const double s = xi + y[j];
    const double r = 1.0 / s;
    neumaier(a1, c1, r);
    neumaier(a2, c2, r * r);
    if (lg) neumaier(a3, c3, log(s));
  }
  a1 = wave_sum(a1) + wave_sum(c1);
  a2 = wave_sum(a2) + wave_sum(c2);
  if (lg) a3 = wave_sum(a3) + wave_sum(c3);
  if (lane == 0) {
    if (s1) s1[i] = accumulate ? s1[i] + a1 : a1;
    if (s2) s2[i] = accumulate ? s2[i] + a2 : a2;
    if (lg) lg[i] = accumulate ? lg[i] + a3 : a3;
  }
}

// ---- batched forms for the tensor solver: one launch per pass over all
// modalities, job tables in device memory, partial sums reduced in a fixed order.

// Tuple sums of one modality seen from one of its axes (own): the other axes
// (the largest rank last) and where its r_own partial sums go.
struct TupleJob {
  int own;
  int n;                      // other axes, 1 .. MAX_AXES - 1
  int other[MAX_AXES - 1];
  int first_wave;             // prefix over jobs of r_own
  int part;                   // offset of its partial sums
};

// Cross block of axes a < b: the sum over the modalities holding both (terms
// [term0, term0 + nterm) of the term table, each the modality's other axes).
struct CrossJob {
  int a, b;
  int first_tile, tiles_x;    // 16 x 16 tiles, prefix over jobs
  int term0, nterm;
};
struct CrossTerm {
  int n;
  int other[MAX_AXES - 2];
};

__device__ inline int find_job_wave(const TupleJob* __restrict__ jobs, int njobs, int w) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first_wave <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Every job's tuple sums at x (axis l at x + ax_off[l]): with logs = 0 the
// partials p1 = sum 1/s and p2 = sum s^-2, with logs = 1 the partial plg =
// sum log s.  One wave per (job, index of the own axis); the tuples of all
// but the last other axis in a fixed order, the last one over the lanes, then
// a fixed-order wave reduction of compensated sums.
__global__ void __launch_bounds__(256) tuple_jobs_kernel(const double* __restrict__ x,
                                                         const int* __restrict__ ax_off,
                                                         const int* __restrict__ ax_r,
                                                         const TupleJob* __restrict__ jobs, int njobs,
                                                         int total_waves, int logs, double* __restrict__ p1,
                                                         double* __restrict__ p2, double* __restrict__ plg) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= total_waves) return;
  const TupleJob& jb = jobs[find_job_wave(jobs, njobs, w)];
  const int i = w - jb.first_wave;
  const int nl = jb.n - 1;
  unsigned long long P = 1;
  for (int u = 0; u < nl; ++u) P *= (unsigned long long)ax_r[jb.other[u]];
  const double* __restrict__ last = x + ax_off[jb.other[nl]];
  const int rl = ax_r[jb.other[nl]];
  const double xi = x[ax_off[jb.own] + i];
  double a1 = 0, c1 = 0, a2 = 0, c2 = 0;
  for (unsigned long long p = 0; p < P; ++p) {
    double base = xi;
    unsigned long long q = p;
    for (int u = 0; u < nl; ++u) {
      const unsigned long long r = (unsigned long long)ax_r[jb.other[u]];
      base += x[ax_off[jb.other[u]] + (int)(q % r)];
      q /= r;
    }
    for (int j = lane; j < rl; j += 64) {
      const double s = base + last[j];
      if (logs) {
        neumaier(a1, c1, log(s));
      } else {
        const double rs = 1.0 / s;
        neumaier(a1, c1, rs);
        neumaier(a2, c2, rs * rs);
      }
    }
  }
  a1 = wave_sum(a1) + wave_sum(c1);
  if (!logs) a2 = wave_sum(a2) + wave_sum(c2);
  if (lane == 0) {
    if (logs) {
      plg[jb.part + i] = a1;
    } else {
      p1[jb.part + i] = a1;
      p2[jb.part + i] = a2;
    }
  }
}

// assemble_kernel over all coordinates: s1, s2 are the sums of the partials of
// the coordinate's axis' jobs (axis_jobs[axis_ptr[l] ..], modality order).
__global__ void tensor_assemble_kernel(const double* __restrict__ E, const double* __restrict__ lam,
                                       const double* __restrict__ p1, const double* __restrict__ p2,
                                       const int* __restrict__ axis_of, const int* __restrict__ ax_off,
                                       const int* __restrict__ axis_ptr, const int* __restrict__ axis_jobs,
                                       const TupleJob* __restrict__ jobs, const double* __restrict__ eps_ax,
                                       int n, int lm, double* __restrict__ g, double* __restrict__ h,
                                       int* __restrict__ active, double* __restrict__ kkt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int l = axis_of[c], i = c - ax_off[l];
  double s1 = 0.0, s2 = 0.0;
  for (int k = axis_ptr[l]; k < axis_ptr[l + 1]; ++k) {
    const int part = jobs[axis_jobs[k]].part + i;
    s1 += p1[part];
    s2 += p2[part];
  }
  const double gi = 0.5 * (E[c] - s1);
  const double hi = 0.5 * s2;
  const double eps = eps_ax[l];
  g[c] = gi;
  h[c] = hi;
  // lm: Bertsekas' rule with the Levenberg-Marquardt diagonal h + |g|/x, the
  // whole diagonal step reaching the bound
  const double reach = lm ? gi / (hi + fabs(gi) / lam[c]) : fmin(1e-3 * lam[c], gi / hi);
  active[c] = (lam[c] - eps <= reach) && (gi > 0.0);
  const bool at = lam[c] <= eps * (1.0 + 1e-12);
  kkt[c] = (at ? fmax(0.0, -gi) : fabs(gi)) / (0.5 * E[c]);
}

// Every cross block at x: S[a][b] = S[b][a]^T = sum over the job's terms of the
// tuple sums of 1/2 s^-2 (one compensated sum over the terms and their tuples
// in a fixed order).  One 16 x 16 tile per workgroup, one thread per entry.
__global__ void __launch_bounds__(256) cross_jobs_kernel(const double* __restrict__ x,
                                                         const int* __restrict__ ax_off,
                                                         const int* __restrict__ ax_r,
                                                         const CrossJob* __restrict__ jobs, int njobs,
                                                         const CrossTerm* __restrict__ terms,
                                                         double* __restrict__ S, int ldS) {
  const int tile = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first_tile <= tile) lo = mid;
    else hi = mid - 1;
  }
  const CrossJob& jb = jobs[lo];
  const int t = tile - jb.first_tile;
  const int i = (t / jb.tiles_x) * 16 + (threadIdx.x >> 4), j = (t % jb.tiles_x) * 16 + (threadIdx.x & 15);
  if (i >= ax_r[jb.a] || j >= ax_r[jb.b]) return;
  const double base0 = x[ax_off[jb.a] + i] + x[ax_off[jb.b] + j];
  double acc = 0.0, cc = 0.0;
  for (int k = 0; k < jb.nterm; ++k) {
    const CrossTerm& tm = terms[jb.term0 + k];
    if (tm.n == 0) {
      neumaier(acc, cc, 0.5 / (base0 * base0));
      continue;
    }
    const int nl = tm.n - 1;
    unsigned long long P = 1;
    for (int u = 0; u < nl; ++u) P *= (unsigned long long)ax_r[tm.other[u]];
    const double* __restrict__ last = x + ax_off[tm.other[nl]];
    const int rl = ax_r[tm.other[nl]];
    for (unsigned long long p = 0; p < P; ++p) {
      double base = base0;
      unsigned long long q = p;
      for (int u = 0; u < nl; ++u) {
        const unsigned long long r = (unsigned long long)ax_r[tm.other[u]];
        base += x[ax_off[tm.other[u]] + (int)(q % r)];
        q /= r;
      }
      for (int kk = 0; kk < rl; ++kk) {
        const double s = base + last[kk];
        neumaier(acc, cc, 0.5 / (s * s));
      }
    }
  }
  acc += cc;
  S[(size_t)(ax_off[jb.a] + i) * ldS + ax_off[jb.b] + j] = acc;
  S[(size_t)(ax_off[jb.b] + j) * ldS + ax_off[jb.a] + i] = acc;
}

// Schur complement of the shared block after the private blocks' forward
// elimination (S seen column-major, leading dimension ld: the shared block
// C(i, j) at S[(K + j) ld + K + i], the private rows of the shared columns
// B(k, i) = S[(K + i) ld + k], k < K):  C(i, j) -= sum_{k<K} B(k, i) B(k, j) for
// i >= j.  One 16 x 16 tile and one of `slices` equal ranges of k per
// workgroup (blockIdx.z; tiles above the diagonal exit), k staged in LDS 64 at
// a time; each range's sums go to part[z][i][j] and hub_schur_reduce_kernel
// subtracts them in range order (fixed summation order throughout).
__global__ void __launch_bounds__(256) hub_schur_kernel(const double* __restrict__ S, int ld, int K, int nh,
                                                        int slices, double* __restrict__ part) {
  const int bi = blockIdx.y, bj = blockIdx.x, z = blockIdx.z;
  if (bj > bi) return;
  __shared__ double bI[16][65], bJ[16][65];
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  const int i = bi * 16 + ti, j = bj * 16 + tj;
  const int per = (K + slices - 1) / slices;
  const int kb = z * per, ke = min(K, kb + per);
  double acc = 0.0;
  for (int k0 = kb; k0 < ke; k0 += 64) {
    for (int q = threadIdx.x; q < 16 * 64; q += 256) {
      const int rr = q >> 6, kk = q & 63, k = k0 + kk;
      const int ir = bi * 16 + rr, jr = bj * 16 + rr;
      bI[rr][kk] = (k < ke && ir < nh) ? S[(size_t)(K + ir) * ld + k] : 0.0;
      bJ[rr][kk] = (k < ke && jr < nh) ? S[(size_t)(K + jr) * ld + k] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 64; ++kk) acc += bI[ti][kk] * bJ[tj][kk];
    __syncthreads();
  }
  if (i < nh && j < nh && i >= j) part[((size_t)z * nh + i) * nh + j] = acc;
}

__global__ void hub_schur_reduce_kernel(double* __restrict__ S, int ld, int K, int nh, int slices,
                                        const double* __restrict__ part) {
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > i || i >= nh) return;
  double a = 0.0;
  for (int z = 0; z < slices; ++z) a += part[((size_t)z * nh + i) * nh + j];
  S[(size_t)(K + j) * ld + K + i] -= a;
}

// rhs[K + i] -= sum_{k<K} B(k, i) rhs[k] (B as in hub_schur_kernel); one wave per i.
__global__ void __launch_bounds__(256) hub_rhs_kernel(const double* __restrict__ S, int ld, int K, int nh,
                                                      double* __restrict__ rhs) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nh) return;
  const double* __restrict__ col = S + (size_t)(K + i) * ld;
  double a = 0.0;
  for (int k = lane; k < K; k += 64) a += col[k] * rhs[k];
  a = wave_sum(a);
  if (lane == 0) rhs[K + i] -= a;
}

// Diagonal (1+rho) h (lm: h + |g|/x), right-hand side -g and activity flags
// of every coordinate (S's diagonal holds zeros before).
__global__ void tensor_diag_kernel(const double* __restrict__ h, const double* __restrict__ g,
                                   const int* __restrict__ act, int n, double damp, const double* __restrict__ x,
                                   int lm, double* __restrict__ S, double* __restrict__ rhs,
                                   int* __restrict__ act_hub) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  S[(size_t)c * n + c] = lm ? h[c] + fabs(g[c]) / x[c] : damp * h[c];
  rhs[c] = -g[c];
  act_hub[c] = act[c];
}

// pair_sums_kernel's s1, s2 for a short x against a long y: nsplit waves per i,
// each over one of nsplit equal ranges of j, partial sums to p1, p2 [s][i];
// pair_merge_kernel adds them in range order.
__global__ void __launch_bounds__(256) pair_sums_split_kernel(const double* __restrict__ x, int nx,
                                                              const double* __restrict__ y, int ny, int nsplit,
                                                              double* __restrict__ p1, double* __restrict__ p2) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nx * nsplit) return;
  const int i = w / nsplit, sp = w % nsplit;
  const int per = (ny + nsplit - 1) / nsplit;
  const int jb = sp * per, je = min(ny, jb + per);
  const double xi = x[i];
  double a1 = 0, c1 = 0, a2 = 0, c2 = 0;
  for (int j = jb + lane; j < je; j += 64) {
    const double r = 1.0 / (xi + y[j]);
    neumaier(a1, c1, r);
    neumaier(a2, c2, r * r);
  }
  a1 = wave_sum(a1) + wave_sum(c1);
  a2 = wave_sum(a2) + wave_sum(c2);
  if (lane == 0) {
    p1[(size_t)sp * nx + i] = a1;
    p2[(size_t)sp * nx + i] = a2;
  }
}

__global__ void pair_merge_kernel(int nx, int nsplit, const double* __restrict__ p1, const double* __restrict__ p2,
                                  double* __restrict__ s1, double* __restrict__ s2, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx) return;
  double a1 = 0.0, a2 = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) {
    a1 += p1[(size_t)sp * nx + i];
    a2 += p2[(size_t)sp * nx + i];
  }
  s1[i] = accumulate ? s1[i] + a1 : a1;
  s2[i] = accumulate ? s2[i] + a2 : a2;
}

// g = (E - s1)/2, h = s2/2, the active set and each coordinate's KKT term:
// |g| / (E/2) when free, max(0, -g) / (E/2) at the bound.
__global__ void assemble_kernel(const double* __restrict__ E, const double* __restrict__ lam,
                                const double* __restrict__ s1, const double* __restrict__ s2,
                                double eps, int n, int lm, double* __restrict__ g, double* __restrict__ h,
                                int* __restrict__ active, double* __restrict__ kkt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double gi = 0.5 * (E[i] - s1[i]);
  const double hi = 0.5 * s2[i];
  g[i] = gi;
  h[i] = hi;
  // coordinates within a diagonal-Newton step of their bound that want to go down
  const double reach = lm ? gi / (hi + fabs(gi) / lam[i]) : fmin(1e-3 * lam[i], gi / hi);
  active[i] = (lam[i] - eps <= reach) && (gi > 0.0);
  const bool at = lam[i] <= eps * (1.0 + 1e-12);
  kkt[i] = (at ? fmax(0.0, -gi) : fabs(gi)) / (0.5 * E[i]);
}

// Schur complement of a leaf axis m against hub axes K1 (rows) and K2 (columns):
//   S[K1_i][K2_k] -= sum_{free j} B1[i][j] B2[k][j] / ((1+rho) h_m[j])   (lm: h_m + |g_m|/y),
//   B[i][j] = 1/2 (x_i + y_j)^-2,
// and, when with_rhs, rhs[K1_i] += sum_{free j} B1[i][j] g_m[j] / ((1+rho) h_m[j]).
// A 16 x 16 tile of S per workgroup.
// The leaf's j range is split into gridDim.z equal parts: part z writes its
// sums to part[z][i][k] (and rpart[z][i]); schur_leaf_merge_kernel applies
// them to S and rhs in part order.
__global__ void __launch_bounds__(256) schur_leaf_kernel(
    const double* __restrict__ x1, int n1, const double* __restrict__ x2, int n2,
    const double* __restrict__ ym, int nm, const int* __restrict__ act_m,
    const double* __restrict__ hm, const double* __restrict__ gm, double damp, int lm,
    double* __restrict__ part, double* __restrict__ rpart, int with_rhs) {
  __shared__ double b1[16][65], b2[16][65], w[64], wg[64];
  const int ti = threadIdx.x >> 4, tk = threadIdx.x & 15;
  const int i = blockIdx.y * 16 + ti, k = blockIdx.x * 16 + tk;
  const int z = blockIdx.z, nz = gridDim.z;
  const int per = ((nm + nz - 1) / nz + 63) / 64 * 64;
  const int jb = z * per, je = min(nm, jb + per);
  double acc = 0.0, racc = 0.0;
  for (int j0 = jb; j0 < je; j0 += 64) {
    for (int q = threadIdx.x; q < 16 * 64; q += 256) {
      const int rr = q >> 6, jj = q & 63, j = j0 + jj;
      const int ir = blockIdx.y * 16 + rr, kr = blockIdx.x * 16 + rr;
      double v1 = 0.0, v2 = 0.0;
      if (j < je && !act_m[j]) {
        if (ir < n1) {
          const double s = x1[ir] + ym[j];
          v1 = 0.5 / (s * s);
        }
        if (kr < n2) {
          const double s = x2[kr] + ym[j];
          v2 = 0.5 / (s * s);
        }
      }
      b1[rr][jj] = v1;
      b2[rr][jj] = v2;
    }
    if (threadIdx.x < 64) {
      const int j = j0 + threadIdx.x;
      const bool fr = j < je && !act_m[j];
      const double dj = fr ? (lm ? hm[j] + fabs(gm[j]) / ym[j] : damp * hm[j]) : 1.0;
      w[threadIdx.x] = fr ? 1.0 / dj : 0.0;
      wg[threadIdx.x] = fr ? gm[j] / dj : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int jj = 0; jj < 64; ++jj) acc += b1[ti][jj] * b2[tk][jj] * w[jj];
    if (with_rhs && blockIdx.x == 0 && tk == 0)
      for (int jj = 0; jj < 64; ++jj) racc += b1[ti][jj] * wg[jj];
    __syncthreads();
  }
  if (i < n1 && k < n2) part[((size_t)z * n1 + i) * n2 + k] = acc;
  if (with_rhs && blockIdx.x == 0 && tk == 0 && i < n1) rpart[(size_t)z * n1 + i] = racc;
}

__global__ void schur_leaf_merge_kernel(int n1, int off1, int n2, int off2, int nz,
                                        const double* __restrict__ part, const double* __restrict__ rpart,
                                        double* __restrict__ S, int ldS, double* __restrict__ rhs, int with_rhs) {
  const int i = blockIdx.y, k = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1 || k >= n2) return;
  double a = 0.0;
  for (int z = 0; z < nz; ++z) a += part[((size_t)z * n1 + i) * n2 + k];
  S[(size_t)(off1 + i) * ldS + off2 + k] -= a;
  if (with_rhs && k == 0) {
    double r = 0.0;
    for (int z = 0; z < nz; ++z) r += rpart[(size_t)z * n1 + i];
    rhs[off1 + i] += r;
  }
}

// Cross block between hub axes K1 (rows) and K2 (columns): S[K1][K2] += B, S[K2][K1] += B^T.
__global__ void schur_cross_kernel(const double* __restrict__ x1, int n1, int off1,
                                   const double* __restrict__ x2, int n2, int off2,
                                   double* __restrict__ S, int ldS) {
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4), k = blockIdx.x * 16 + (threadIdx.x & 15);
  if (i >= n1 || k >= n2) return;
  const double s = x1[i] + x2[k];
  const double b = 0.5 / (s * s);
  S[(size_t)(off1 + i) * ldS + off2 + k] += b;
  S[(size_t)(off2 + k) * ldS + off1 + i] += b;
}

// Diagonal (1+rho) h (lm: h + |g|/x) and right-hand side -g of a hub axis;
// copies its activity flags into hub order.
__global__ void schur_diag_kernel(const double* __restrict__ h, const double* __restrict__ g,
                                  const int* __restrict__ act, int n, int off, double damp,
                                  const double* __restrict__ x, int lm,
                                  double* __restrict__ S, int ldS, double* __restrict__ rhs,
                                  int* __restrict__ act_hub) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  S[(size_t)(off + i) * ldS + off + i] += lm ? h[i] + fabs(g[i]) / x[i] : damp * h[i];
  rhs[off + i] = -g[i];
  act_hub[off + i] = act[i];
}

// Active hub coordinates: identity row and column, zero right-hand side.
__global__ void schur_pin_kernel(const int* __restrict__ act_hub, int nS, double* __restrict__ S,
                                 double* __restrict__ rhs) {
  const int i = blockIdx.y, k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nS) return;
  if (act_hub[i] || act_hub[k]) S[(size_t)i * nS + k] = (i == k) ? 1.0 : 0.0;
  if (k == 0 && act_hub[i]) rhs[i] = 0.0;
}

// Cholesky factorisation (lower, in place) and solve of the SPD system S x = b,
// row-major n x n, one workgroup.  *bad = 1 if a pivot is not positive.
__global__ void __launch_bounds__(1024) cholesky_solve_kernel(double* __restrict__ S, int n,
                                                              double* __restrict__ b,
                                                              int* __restrict__ bad) {
  __shared__ double piv;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int c = 0; c < n; ++c) {
    if (tid == 0) {
      const double d = S[(size_t)c * n + c];
      if (!(d > 0.0)) *bad = 1;
      piv = sqrt(fmax(d, 1e-300));
      S[(size_t)c * n + c] = piv;
    }
    __syncthreads();
    for (int r = c + 1 + tid; r < n; r += nt) S[(size_t)r * n + c] /= piv;
    __syncthreads();
    // trailing update of the lower triangle, 32 threads per row
    for (int r = c + 1 + tid / 32; r < n; r += nt / 32) {
      const double lr = S[(size_t)r * n + c];
      for (int k = c + 1 + (tid & 31); k <= r; k += 32) S[(size_t)r * n + k] -= lr * S[(size_t)k * n + c];
    }
    __syncthreads();
  }
  for (int c = 0; c < n; ++c) {          // L y = b
    if (tid == 0) b[c] /= S[(size_t)c * n + c];
    __syncthreads();
    for (int r = c + 1 + tid; r < n; r += nt) b[r] -= S[(size_t)r * n + c] * b[c];
    __syncthreads();
  }
  for (int c = n - 1; c >= 0; --c) {     // L^T x = y
    if (tid == 0) b[c] /= S[(size_t)c * n + c];
    __syncthreads();
    for (int r = tid; r < c; r += nt) b[r] -= S[(size_t)c * n + r] * b[c];
    __syncthreads();
  }
}

// Newton step of a hub axis: the Schur solution on free coordinates, -g/h on
// active ones (lm: -g/(h + |g|/lam)).
__global__ void hub_step_kernel(const double* __restrict__ x, const double* __restrict__ g,
                                const double* __restrict__ h, const int* __restrict__ act, int n,
                                const double* __restrict__ lam, int lm, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  d[i] = act[i] ? -g[i] / (lm ? h[i] + fabs(g[i]) / lam[i] : h[i]) : x[i];
}

// acc[j] += sum_{free hub i} B[i][j] d_K[i] for a leaf axis (one wave per j).
__global__ void __launch_bounds__(256) leaf_partner_kernel(const double* __restrict__ ym, int nm,
                                                           const double* __restrict__ xK, int nK,
                                                           const int* __restrict__ actK,
                                                           const double* __restrict__ dK,
                                                           double* __restrict__ acc) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nm) return;
  double s = 0.0;
  for (int i = lane; i < nK; i += 64) {
    if (actK[i]) continue;
    const double t = xK[i] + ym[j];
    s += 0.5 / (t * t) * dK[i];
  }
  s = wave_sum(s);
  if (lane == 0) acc[j] += s;
}

__global__ void leaf_step_kernel(const double* __restrict__ g, const double* __restrict__ h,
                                 const int* __restrict__ act, const double* __restrict__ acc,
                                 int n, double damp, const double* __restrict__ x, int lm,
                                 double* __restrict__ d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double dj = lm ? h[j] + fabs(g[j]) / x[j] : h[j];
  d[j] = act[j] ? -g[j] / dj : (-g[j] - acc[j]) / (lm ? dj : damp * h[j]);
}

// *out = sum_i a[i] * (b ? b[i] : 1)  (one workgroup, fixed order)
__global__ void __launch_bounds__(RED_THREADS) dot_kernel(const double* __restrict__ a,
                                                          const double* __restrict__ b, int n,
                                                          double* __restrict__ out) {
  __shared__ double red[RED_THREADS / 64];
  double s = 0, c = 0;
  for (int i = threadIdx.x; i < n; i += RED_THREADS) neumaier(s, c, b ? a[i] * b[i] : a[i]);
  const double t = block_sum(s + c, red);
  if (threadIdx.x == 0) *out = t;
}

// *out = max_i a[i]  (one workgroup)
__global__ void __launch_bounds__(RED_THREADS) max_kernel(const double* __restrict__ a, int n,
                                                          double* __restrict__ out) {
  __shared__ double red[RED_THREADS / 64];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += RED_THREADS) m = fmax(m, a[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < RED_THREADS / 64; ++w) r = fmax(r, red[w]);
    *out = r;
  }
}

// Per axis l (one workgroup each): sums[l] = sum of v over the axis (the order
// and compensation of dot_kernel) and mins[l] = its minimum.
__global__ void __launch_bounds__(RED_THREADS) axis_stats_kernel(const double* __restrict__ v,
                                                                 const int* __restrict__ ax_off,
                                                                 const int* __restrict__ ax_r,
                                                                 double* __restrict__ sums,
                                                                 double* __restrict__ mins) {
  __shared__ double red[RED_THREADS / 64];
  const int l = blockIdx.x;
  const double* __restrict__ a = v + ax_off[l];
  const int n = ax_r[l];
  double s = 0, c = 0, m = INFINITY;
  for (int i = threadIdx.x; i < n; i += RED_THREADS) {
    neumaier(s, c, a[i]);
    m = fmin(m, a[i]);
  }
  const double t = block_sum(s + c, red);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < RED_THREADS / 64; ++w) r = fmin(r, red[w]);
    sums[l] = t;
    mins[l] = r;
  }
}

// Trial point t = max(x + alpha d, floor) over all coordinates (axis of
// coordinate i: axis_of[i]): an active coordinate may reach its bound, a free
// one may shrink by at most STEP_SHRINK per iteration (a coupled Newton step can
// overshoot far below the optimum, and recovery from the bound doubles the
// value per iteration at best).
constexpr double STEP_SHRINK = 64.0;
__global__ void trial_all_kernel(const double* __restrict__ x, const double* __restrict__ d,
                                 const int* __restrict__ act, const int* __restrict__ axis_of,
                                 const double* __restrict__ eps_ax, int n, double alpha, int limit,
                                 double* __restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double eps = eps_ax[axis_of[i]];
  const double fl = (act[i] || !limit) ? eps : fmax(eps, x[i] / STEP_SHRINK);
  t[i] = fmax(x[i] + alpha * d[i], fl);
}

__global__ void clip_all_kernel(double* __restrict__ lam, const int* __restrict__ axis_of,
                                const double* __restrict__ eps_ax, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) lam[i] = fmax(lam[i], eps_ax[axis_of[i]]);
}

// Armijo prediction: alpha sum_free g d + sum_active g (t - x)   (one workgroup)
__global__ void __launch_bounds__(RED_THREADS) pred_kernel(
    const double* __restrict__ g, const double* __restrict__ d, const double* __restrict__ x,
    const double* __restrict__ t, const int* __restrict__ act, int n, double alpha,
    double* __restrict__ out) {
  __shared__ double red[RED_THREADS / 64];
  double s = 0, c = 0;
  for (int i = threadIdx.x; i < n; i += RED_THREADS)
    neumaier(s, c, act[i] ? g[i] * (t[i] - x[i]) : alpha * g[i] * d[i]);
  const double v = block_sum(s + c, red);
  if (threadIdx.x == 0) *out = v;
}

__global__ void add_const_kernel(double* __restrict__ x, int n, double a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += a;
}

// Start point: the warm start, or Algorithm 1's 1/E; flags non-positive or non-finite
// E (1) and a non-finite warm start (2).
__global__ void init_kernel(const double* __restrict__ E, const double* __restrict__ warm, int n,
                            double* __restrict__ lam, int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double e = E[i];
  if (!(e > 0.0) || !isfinite(e)) atomicMax(bad, 1);
  const double v = warm ? warm[i] : 1.0 / e;
  if (warm && !isfinite(v)) atomicMax(bad, 2);
  lam[i] = v;
}

__global__ void __launch_bounds__(RED_THREADS) count_pinned_kernel(const double* __restrict__ lam,
                                                                   double eps, int n,
                                                                   double* __restrict__ out) {
  __shared__ double red[RED_THREADS / 64];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += RED_THREADS) s += lam[i] <= eps * (1.0 + 1e-12) ? 1.0 : 0.0;
  const double v = block_sum(s, red);
  if (threadIdx.x == 0) *out = v;
}

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------ host side

// Minimum total-rank vertex cover of the modality graph (exhaustive; at most 8 axes).
std::vector<int> hub_axes(const std::vector<Axis>& ax, const std::vector<std::pair<int, int>>& mods) {
  const int L = (int)ax.size();
  std::vector<int> best;
  long bestw = -1;
  for (int mask = 0; mask < (1 << L); ++mask) {
    bool cover = true;
    for (auto& m : mods) cover = cover && (((mask >> m.first) & 1) || ((mask >> m.second) & 1));
    if (!cover) continue;
    long w = 0;
    for (int l = 0; l < L; ++l)
      if ((mask >> l) & 1) w += ax[l].r;
    if (bestw < 0 || w < bestw) {
      bestw = w;
      best.clear();
      for (int l = 0; l < L; ++l)
        if ((mask >> l) & 1) best.push_back(l);
    }
  }
  return best;
}

// State shared by the pair and tensor solvers: per-axis vectors concatenated
// (axis l at ax[l].off), the Newton system of nS unknowns, device scalars.
struct Core {
  gmgm_ctx* c = nullptr;
  hipStream_t st = nullptr;
  int L = 0;
  std::vector<Axis> ax;
  std::vector<std::vector<int>> sets;   // each modality's axes
  size_t T = 0, nS = 0;
  // escape mode (after lm_after iterations): Levenberg-Marquardt diagonal
  // |g|/x in the Newton system and the active-set reach, no shrink limit
  int lm_after = 1 << 30;
  bool lm = false;
  double *lam, *trial, *Ec, *s1, *s2, *lg, *g, *h, *d, *acc, *kkt, *S, *rhs, *scal, *eps_ax;
  int *act, *act_hub, *flag, *axis_of, *ax_off, *ax_r;
  std::vector<int> h_axis_of, h_off, h_r;   // host copies (alive while copies are in flight)
  std::vector<double> h_eps;

  gmgm_status fetch(double* host, const double* dev, int count) {
    GMGM_HIP(c, hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    return GMGM_OK;
  }

  // every axis' sum and minimum of v (one launch, one read-back)
  gmgm_status axis_stats(const double* v, std::vector<double>& sums, std::vector<double>& mins) {
    hipLaunchKernelGGL(axis_stats_kernel, dim3(L), dim3(RED_THREADS), 0, st, v, ax_off, ax_r, scal, scal + L);
    std::vector<double> both(2 * L);
    GMGM_TRY(fetch(both.data(), scal, 2 * L));
    sums.assign(both.begin(), both.begin() + L);
    mins.assign(both.begin() + L, both.end());
    return GMGM_OK;
  }

  // sum_l cdir_l sums_l (axes with cdir_l = 0 skipped)
  static double gauge_value(const std::vector<double>& sums, const std::vector<double>& cdir) {
    double out = 0;
    for (size_t l = 0; l < sums.size(); ++l)
      if (cdir[l] != 0.0) out += cdir[l] * sums[l];
    return out;
  }

  gmgm_status bind_workspace() {
    void *w0, *w1;
    const size_t nd = T * 11 + 3 * (size_t)L + 64, ni = T + 2 * (size_t)L;
    GMGM_TRY(ws_get(c, WS_SOLVE0, nd * sizeof(double) + ni * sizeof(int), &w0));
    GMGM_TRY(ws_get(c, WS_SOLVE1, nS * nS * 8 + nS * 8 + (T + nS + 64) * 4, &w1));
    double* base = (double*)w0;
    lam = base;
    trial = base + T;
    Ec = base + 2 * T;
    s1 = base + 3 * T;
    s2 = base + 4 * T;
    lg = base + 5 * T;
    g = base + 6 * T;
    h = base + 7 * T;
    d = base + 8 * T;
    acc = base + 9 * T;
    kkt = base + 10 * T;
    scal = base + 11 * T;                 // 2 L + 64 scalars
    eps_ax = scal + 2 * L + 64;
    axis_of = (int*)(base + nd);
    ax_off = axis_of + T;
    ax_r = ax_off + L;
    h_axis_of.resize(T);
    h_off.resize(L);
    h_r.resize(L);
    for (int l = 0; l < L; ++l) {
      h_off[l] = (int)ax[l].off;
      h_r[l] = ax[l].r;
      for (int i = 0; i < ax[l].r; ++i) h_axis_of[ax[l].off + i] = l;
    }
    GMGM_HIP(c, hipMemcpyAsync(axis_of, h_axis_of.data(), T * sizeof(int), hipMemcpyHostToDevice, st));
    GMGM_HIP(c, hipMemcpyAsync(ax_off, h_off.data(), L * sizeof(int), hipMemcpyHostToDevice, st));
    GMGM_HIP(c, hipMemcpyAsync(ax_r, h_r.data(), L * sizeof(int), hipMemcpyHostToDevice, st));
    S = (double*)w1;
    rhs = S + nS * nS;
    act = (int*)(rhs + nS);
    act_hub = act + T;
    flag = act_hub + nS;
    return GMGM_OK;
  }

  // the bounds eps_l, once known, to the device
  gmgm_status upload_eps() {
    h_eps.resize(L);
    for (int l = 0; l < L; ++l) h_eps[l] = ax[l].eps;
    GMGM_HIP(c, hipMemcpyAsync(eps_ax, h_eps.data(), L * sizeof(double), hipMemcpyHostToDevice, st));
    return GMGM_OK;
  }

  void clip(double* v) {
    hipLaunchKernelGGL(clip_all_kernel, dim3(nblk(T)), dim3(256), 0, st, v, axis_of, eps_ax, (int)T);
  }

  // trial = max(lam + alpha d, floor) over all coordinates
  void trial_point(double alpha) {
    hipLaunchKernelGGL(trial_all_kernel, dim3(nblk(T)), dim3(256), 0, st, lam, d, act, axis_of, eps_ax, (int)T,
                       alpha, lm ? 0 : 1, trial);
  }
};

// Modalities of two axes: Newton system by the Schur complement on the hub axes.
struct Solver : Core {
  std::vector<std::pair<int, int>> mods;
  std::vector<int> hub, is_hub;
  std::vector<size_t> hoff;
  double* split_buf = nullptr;   // partial sums of the split pair-sum and Schur-leaf passes

  // Ranges of the long axis for one short axis' pair sums (enough waves to fill
  // the chip, at least 256 partners each); 1 = no split.
  static int pair_splits(int nx, int ny) {
    if (nx >= 2048) return 1;
    return std::max(1, std::min({64, (4096 + nx - 1) / nx, (ny + 255) / 256}));
  }
  // Ranges of a leaf axis for one Schur block (about 1024 workgroups, at least
  // 256 leaf coordinates each, partial sums at most 64 MiB).
  static int leaf_splits(int n1, int n2, int nm) {
    const long tiles = (long)nblk(n1, 16) * nblk(n2, 16);
    const long by_mem = std::max<long>(1, (64L << 20) / (8L * n1 * n2 + 8L * n1));
    return (int)std::max<long>(
        1, std::min<long>({64L, std::max<long>(1, 1024 / tiles), (long)(nm + 255) / 256, by_mem}));
  }

  // workspace for the largest split pass (WS_SOLVE2)
  gmgm_status plan_splits() {
    size_t need = 16;
    for (int l = 0; l < L; ++l)
      for (auto& m : mods) {
        const int other = m.first == l ? m.second : m.second == l ? m.first : -1;
        if (other < 0) continue;
        need = std::max(need, 2 * (size_t)pair_splits(ax[l].r, ax[other].r) * ax[l].r);
      }
    for (int m = 0; m < L; ++m) {
      if (is_hub[m]) continue;
      for (auto& md : mods) {
        const int K1 = md.first == m ? md.second : md.second == m ? md.first : -1;
        if (K1 < 0) continue;
        for (auto& md2 : mods) {
          const int K2 = md2.first == m ? md2.second : md2.second == m ? md2.first : -1;
          if (K2 < 0) continue;
          const size_t nz = leaf_splits(ax[K1].r, ax[K2].r, ax[m].r);
          need = std::max(need, nz * ax[K1].r * ax[K2].r + nz * ax[K1].r);
        }
      }
    }
    void* w;
    GMGM_TRY(ws_get(c, WS_SOLVE2, need * sizeof(double), &w));
    split_buf = (double*)w;
    return GMGM_OK;
  }

  // NLL(x) = 1/2 (sum E x - sum log); each modality's log terms counted once.
  gmgm_status nll(const double* x, double* out) {
    GMGM_TRY(nll_launch(x));
    double v[2];
    GMGM_TRY(fetch(v, scal, 2));
    *out = 0.5 * (v[0] - v[1]);
    return GMGM_OK;
  }

  // sum E x into out[0] and the log sum into out[1] (out: scal when null)
  gmgm_status nll_launch(const double* x, double* out = nullptr) {
    if (!out) out = scal;
    // each modality's log terms from its larger axis (one wave per entry)
    std::vector<int> written(L, 0);
    for (auto& m : mods) {
      const int l = ax[m.second].r > ax[m.first].r ? m.second : m.first;
      const int o = l == m.first ? m.second : m.first;
      hipLaunchKernelGGL(pair_sums_kernel, dim3(nblk(ax[l].r, 4)), dim3(256), 0, st, x + ax[l].off, ax[l].r,
                         x + ax[o].off, ax[o].r, (double*)nullptr, (double*)nullptr, lg + ax[l].off, written[l]);
      written[l] = 1;
    }
    for (int l = 0; l < L; ++l)
      if (!written[l]) GMGM_HIP(c, hipMemsetAsync(lg + ax[l].off, 0, ax[l].r * sizeof(double), st));
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(RED_THREADS), 0, st, Ec, x, (int)T, out);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(RED_THREADS), 0, st, lg, (const double*)nullptr,
                       (int)T, out + 1);
    return GMGM_OK;
  }

  // g, h, the active set and the KKT residual at x.
  gmgm_status gradient(const double* x, double* kres) {
    for (int l = 0; l < L; ++l) {
      int first = 1;
      for (auto& m : mods) {
        const int other = m.first == l ? m.second : m.second == l ? m.first : -1;
        if (other < 0) continue;
        const int ns = pair_splits(ax[l].r, ax[other].r);
        if (ns > 1) {
          double* p1 = split_buf;
          double* p2 = split_buf + (size_t)ns * ax[l].r;
          hipLaunchKernelGGL(pair_sums_split_kernel, dim3(nblk((int64_t)ax[l].r * ns, 4)), dim3(256), 0, st,
                             x + ax[l].off, ax[l].r, x + ax[other].off, ax[other].r, ns, p1, p2);
          hipLaunchKernelGGL(pair_merge_kernel, dim3(nblk(ax[l].r)), dim3(256), 0, st, ax[l].r, ns, p1, p2,
                             s1 + ax[l].off, s2 + ax[l].off, first ? 0 : 1);
        } else {
          hipLaunchKernelGGL(pair_sums_kernel, dim3(nblk(ax[l].r, 4)), dim3(256), 0, st, x + ax[l].off,
                             ax[l].r, x + ax[other].off, ax[other].r, s1 + ax[l].off, s2 + ax[l].off,
                             (double*)nullptr, first ? 0 : 1);
        }
        first = 0;
      }
      hipLaunchKernelGGL(assemble_kernel, dim3(nblk(ax[l].r)), dim3(256), 0, st, Ec + ax[l].off,
                         x + ax[l].off, s1 + ax[l].off, s2 + ax[l].off, ax[l].eps, ax[l].r, lm ? 1 : 0,
                         g + ax[l].off, h + ax[l].off, act + ax[l].off, kkt + ax[l].off);
    }
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(RED_THREADS), 0, st, kkt, (int)T, scal);
    return fetch(kres, scal, 1);
  }

  // Damped projected-Newton direction d at lam (g, h and act current).
  gmgm_status direction(double rho) {
    const double damp = 1.0 + rho;
    GMGM_HIP(c, hipMemsetAsync(S, 0, nS * nS * sizeof(double), st));
    for (int l : hub)
      hipLaunchKernelGGL(schur_diag_kernel, dim3(nblk(ax[l].r)), dim3(256), 0, st, h + ax[l].off,
                         g + ax[l].off, act + ax[l].off, ax[l].r, (int)hoff[l], damp, lam + ax[l].off, lm ? 1 : 0,
                         S, (int)nS, rhs, act_hub);
    for (auto& m : mods)
      if (is_hub[m.first] && is_hub[m.second]) {
        const int a = m.first, b = m.second;
        hipLaunchKernelGGL(schur_cross_kernel, dim3(nblk(ax[b].r, 16), nblk(ax[a].r, 16)), dim3(256), 0,
                           st, lam + ax[a].off, ax[a].r, (int)hoff[a], lam + ax[b].off, ax[b].r,
                           (int)hoff[b], S, (int)nS);
      }
    for (int m = 0; m < L; ++m) {
      if (is_hub[m]) continue;
      std::vector<int> partners;   // all hubs: the leaves form an independent set
      for (auto& md : mods) {
        if (md.first == m) partners.push_back(md.second);
        if (md.second == m) partners.push_back(md.first);
      }
      for (int K1 : partners)
        for (int K2 : partners) {
          const int nz = leaf_splits(ax[K1].r, ax[K2].r, ax[m].r);
          double* part = split_buf;
          double* rpart = split_buf + (size_t)nz * ax[K1].r * ax[K2].r;
          const int wr = K1 == K2 ? 1 : 0;
          hipLaunchKernelGGL(schur_leaf_kernel, dim3(nblk(ax[K2].r, 16), nblk(ax[K1].r, 16), (unsigned)nz),
                             dim3(256), 0, st, lam + ax[K1].off, ax[K1].r, lam + ax[K2].off, ax[K2].r,
                             lam + ax[m].off, ax[m].r, act + ax[m].off, h + ax[m].off, g + ax[m].off, damp,
                             lm ? 1 : 0, part, rpart, wr);
          hipLaunchKernelGGL(schur_leaf_merge_kernel, dim3(nblk(ax[K2].r), (unsigned)ax[K1].r), dim3(256), 0, st,
                             ax[K1].r, (int)hoff[K1], ax[K2].r, (int)hoff[K2], nz, part, rpart, S, (int)nS, rhs, wr);
        }
    }
    hipLaunchKernelGGL(schur_pin_kernel, dim3(nblk(nS), (unsigned)nS), dim3(256), 0, st, act_hub,
                       (int)nS, S, rhs);
    GMGM_HIP(c, hipMemsetAsync(flag, 0, sizeof(int), st));
    if (nS <= (size_t)CHOL_ONE_WG) {
      hipLaunchKernelGGL(cholesky_solve_kernel, dim3(1), dim3(1024), 0, st, S, (int)nS, rhs, flag);
    } else {
      // larger systems: rocSOLVER's blocked Cholesky (S is symmetric and fully
      // stored, so its row-major storage is its column-major one); a failed
      // factorisation leaves a positive info in flag, as the kernel above does
      void* hv;
      GMGM_TRY(blas_handle(c, &hv));
      rocblas_handle bh = (rocblas_handle)hv;
      const rocblas_int n = (rocblas_int)nS;
      if (rocsolver_dpotrf(bh, rocblas_fill_lower, n, S, n, flag) != rocblas_status_success ||
          rocsolver_dpotrs(bh, rocblas_fill_lower, n, 1, S, n, rhs, n) != rocblas_status_success)
        return set_err(c, GMGM_E_HIP, "rocSOLVER Cholesky failed in the Newton solve");
    }
    for (int l : hub)
      hipLaunchKernelGGL(hub_step_kernel, dim3(nblk(ax[l].r)), dim3(256), 0, st, rhs + hoff[l],
                         g + ax[l].off, h + ax[l].off, act + ax[l].off, ax[l].r, lam + ax[l].off, lm ? 1 : 0,
                         d + ax[l].off);
    for (int m = 0; m < L; ++m) {
      if (is_hub[m]) continue;
      GMGM_HIP(c, hipMemsetAsync(acc + ax[m].off, 0, ax[m].r * sizeof(double), st));
      for (auto& md : mods) {
        const int K = md.first == m ? md.second : md.second == m ? md.first : -1;
        if (K < 0) continue;
        hipLaunchKernelGGL(leaf_partner_kernel, dim3(nblk(ax[m].r, 4)), dim3(256), 0, st, lam + ax[m].off,
                           ax[m].r, lam + ax[K].off, ax[K].r, act + ax[K].off, d + ax[K].off,
                           acc + ax[m].off);
      }
      hipLaunchKernelGGL(leaf_step_kernel, dim3(nblk(ax[m].r)), dim3(256), 0, st, g + ax[m].off,
                         h + ax[m].off, act + ax[m].off, acc + ax[m].off, ax[m].r, damp, lam + ax[m].off,
                         lm ? 1 : 0, d + ax[m].off);
    }
    int bad = 0;
    GMGM_HIP(c, hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    if (bad) return set_err(c, GMGM_E_NOCONV, "Newton system is not positive definite");
    return GMGM_OK;
  }
};

// Modalities of any number of axes: the Newton system over all coordinates,
// held dense and solved by block elimination of each modality's private axes.
// Each pass over the modalities (gradient, log sums, cross blocks) is one launch
// driven by job tables built once per solve.
struct TensorSolver : Core {
  // Coordinates of each modality's private axes (those in no other modality)
  // form one contiguous group per modality; the shared axes come last, from
  // hub_off.  The Hessian then has the block-arrow form: private groups couple
  // only with themselves and the shared axes.
  std::vector<std::pair<size_t, size_t>> groups;   // (offset, size)
  size_t hub_off = 0;
  int* ginfo = nullptr;                           // factorisation flags of the groups
  double* hub_part = nullptr;                     // partial Schur sums of the shared block
  int hub_slices = 1;
  std::vector<TupleJob> h_grad_jobs, h_log_jobs;
  std::vector<CrossJob> h_cross_jobs;
  std::vector<CrossTerm> h_terms;
  std::vector<int> h_axis_ptr, h_axis_jobs;
  TupleJob *grad_jobs = nullptr, *log_jobs = nullptr;
  CrossJob* cross_jobs = nullptr;
  CrossTerm* terms = nullptr;
  int *axis_ptr = nullptr, *axis_jobs = nullptr;
  double *p1 = nullptr, *p2 = nullptr, *plg = nullptr;
  int grad_waves = 0, log_waves = 0, cross_tiles = 0, log_parts = 0;

  // Axes of m other than skip_a and skip_b, the largest rank last.
  std::vector<int> others(const std::vector<int>& m, int skip_a, int skip_b) const {
    std::vector<int> o;
    for (int a : m)
      if (a != skip_a && a != skip_b) o.push_back(a);
    if (!o.empty()) {
      size_t big = 0;
      for (size_t u = 1; u < o.size(); ++u)
        if (ax[o[u]].r > ax[o[big]].r) big = u;
      std::swap(o[big], o.back());
    }
    return o;
  }

  // Job tables and partial-sum buffers (in WS_SOLVE2).
  gmgm_status prepare() {
    int part = 0;
    h_axis_ptr.assign(L + 1, 0);
    std::vector<std::vector<int>> per_axis(L);
    for (auto& m : sets)
      for (int a : m) {
        TupleJob j{};
        j.own = a;
        const std::vector<int> o = others(m, a, -1);
        j.n = (int)o.size();
        for (int u = 0; u < j.n; ++u) j.other[u] = o[u];
        j.first_wave = grad_waves;
        j.part = part;
        grad_waves += ax[a].r;
        part += ax[a].r;
        per_axis[a].push_back((int)h_grad_jobs.size());
        h_grad_jobs.push_back(j);
      }
    for (int l = 0; l < L; ++l) {
      h_axis_ptr[l + 1] = h_axis_ptr[l] + (int)per_axis[l].size();
      for (int k : per_axis[l]) h_axis_jobs.push_back(k);
    }
    for (auto& m : sets) {   // each modality's log terms once, from its largest-rank axis (most waves)
      int own = m[0];
      for (int a : m)
        if (ax[a].r > ax[own].r) own = a;
      TupleJob j{};
      j.own = own;
      const std::vector<int> o = others(m, own, -1);
      j.n = (int)o.size();
      for (int u = 0; u < j.n; ++u) j.other[u] = o[u];
      j.first_wave = log_waves;
      j.part = log_waves;
      log_waves += ax[own].r;
      h_log_jobs.push_back(j);
    }
    log_parts = log_waves;
    for (int a = 0; a < L; ++a)
      for (int b = a + 1; b < L; ++b) {
        CrossJob j{};
        j.a = a;
        j.b = b;
        j.term0 = (int)h_terms.size();
        for (auto& m : sets)
          if (std::find(m.begin(), m.end(), a) != m.end() && std::find(m.begin(), m.end(), b) != m.end()) {
            CrossTerm tm{};
            const std::vector<int> o = others(m, a, b);
            tm.n = (int)o.size();
            for (int u = 0; u < tm.n; ++u) tm.other[u] = o[u];
            h_terms.push_back(tm);
          }
        j.nterm = (int)h_terms.size() - j.term0;
        if (j.nterm == 0) continue;
        j.tiles_x = (int)nblk(ax[b].r, 16);
        j.first_tile = cross_tiles;
        cross_tiles += j.tiles_x * (int)nblk(ax[a].r, 16);
        h_cross_jobs.push_back(j);
      }
    auto al = [](size_t bytes) { return (bytes + 255) / 256 * 256; };
    const size_t b_gj = al(h_grad_jobs.size() * sizeof(TupleJob)), b_lj = al(h_log_jobs.size() * sizeof(TupleJob));
    const size_t b_cj = al(h_cross_jobs.size() * sizeof(CrossJob) + 1), b_tm = al(h_terms.size() * sizeof(CrossTerm) + 1);
    const size_t b_ap = al((L + 1) * sizeof(int)), b_aj = al(h_axis_jobs.size() * sizeof(int));
    const size_t b_p = al((size_t)part * sizeof(double)), b_lg = al((size_t)log_parts * sizeof(double));
    const size_t b_gi = al((groups.size() + 1) * sizeof(int));
    // k ranges of the shared block's Schur update: enough workgroups to fill the
    // chip when the block is small, partial sums at most 64 MiB
    const size_t nh = T - hub_off, tiles = (nblk(nh, 16) * (nblk(nh, 16) + 1)) / 2;
    hub_slices = 1;
    if (nh > 0 && hub_off > 0) {
      const size_t want = std::max<size_t>(1, 2048 / std::max<size_t>(tiles, 1));
      const size_t by_k = (hub_off + 255) / 256, by_mem = std::max<size_t>(1, ((size_t)64 << 20) / (8 * nh * nh));
      hub_slices = (int)std::max<size_t>(1, std::min(want, std::min(by_k, by_mem)));
    }
    const size_t b_hp = al((size_t)hub_slices * nh * nh * sizeof(double) + 8);
    void* w2;
    GMGM_TRY(ws_get(c, WS_SOLVE2, b_gj + b_lj + b_cj + b_tm + b_ap + b_aj + 2 * b_p + b_lg + b_gi + b_hp, &w2));
    char* q = (char*)w2;
    grad_jobs = (TupleJob*)q;
    q += b_gj;
    log_jobs = (TupleJob*)q;
    q += b_lj;
    cross_jobs = (CrossJob*)q;
    q += b_cj;
    terms = (CrossTerm*)q;
    q += b_tm;
    axis_ptr = (int*)q;
    q += b_ap;
    axis_jobs = (int*)q;
    q += b_aj;
    p1 = (double*)q;
    q += b_p;
    p2 = (double*)q;
    q += b_p;
    plg = (double*)q;
    q += b_lg;
    ginfo = (int*)q;
    q += b_gi;
    hub_part = (double*)q;
    auto up = [&](void* dst, const void* src, size_t bytes) -> gmgm_status {
      if (bytes) GMGM_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
      return GMGM_OK;
    };
    GMGM_TRY(up(grad_jobs, h_grad_jobs.data(), h_grad_jobs.size() * sizeof(TupleJob)));
    GMGM_TRY(up(log_jobs, h_log_jobs.data(), h_log_jobs.size() * sizeof(TupleJob)));
    GMGM_TRY(up(cross_jobs, h_cross_jobs.data(), h_cross_jobs.size() * sizeof(CrossJob)));
    GMGM_TRY(up(terms, h_terms.data(), h_terms.size() * sizeof(CrossTerm)));
    GMGM_TRY(up(axis_ptr, h_axis_ptr.data(), (L + 1) * sizeof(int)));
    GMGM_TRY(up(axis_jobs, h_axis_jobs.data(), h_axis_jobs.size() * sizeof(int)));
    return GMGM_OK;
  }

  // NLL(x) = 1/2 (sum E x - sum log)
  gmgm_status nll(const double* x, double* out) {
    GMGM_TRY(nll_launch(x));
    double v[2];
    GMGM_TRY(fetch(v, scal, 2));
    *out = 0.5 * (v[0] - v[1]);
    return GMGM_OK;
  }

  // sum E x into out[0] and the log sum into out[1] (out: scal when null)
  gmgm_status nll_launch(const double* x, double* out = nullptr) {
    if (!out) out = scal;
    hipLaunchKernelGGL(tuple_jobs_kernel, dim3(nblk(log_waves, 4)), dim3(256), 0, st, x, ax_off, ax_r, log_jobs,
                       (int)h_log_jobs.size(), log_waves, 1, (double*)nullptr, (double*)nullptr, plg);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(RED_THREADS), 0, st, Ec, x, (int)T, out);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(RED_THREADS), 0, st, plg, (const double*)nullptr, log_parts,
                       out + 1);
    return GMGM_OK;
  }

  // g, h, the active set and the KKT residual at x.
  gmgm_status gradient(const double* x, double* kres) {
    hipLaunchKernelGGL(tuple_jobs_kernel, dim3(nblk(grad_waves, 4)), dim3(256), 0, st, x, ax_off, ax_r, grad_jobs,
                       (int)h_grad_jobs.size(), grad_waves, 0, p1, p2, (double*)nullptr);
    hipLaunchKernelGGL(tensor_assemble_kernel, dim3(nblk(T)), dim3(256), 0, st, Ec, x, p1, p2, axis_of, ax_off,
                       axis_ptr, axis_jobs, grad_jobs, eps_ax, (int)T, lm ? 1 : 0, g, h, act, kkt);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(RED_THREADS), 0, st, kkt, (int)T, scal);
    return fetch(kres, scal, 1);
  }

  // Damped projected-Newton direction d at lam (g, h and act current): the free
  // block of the Hessian with its diagonal times 1 + rho, solved by
  // block_arrow_solve; -g/h on active coordinates.
  gmgm_status direction(double rho) {
    const double damp = 1.0 + rho;
    GMGM_HIP(c, hipMemsetAsync(S, 0, nS * nS * sizeof(double), st));
    hipLaunchKernelGGL(tensor_diag_kernel, dim3(nblk(T)), dim3(256), 0, st, h, g, act, (int)T, damp, lam,
                       lm ? 1 : 0, S, rhs, act_hub);
    if (cross_tiles > 0)
      hipLaunchKernelGGL(cross_jobs_kernel, dim3((unsigned)cross_tiles), dim3(256), 0, st, lam, ax_off, ax_r,
                         cross_jobs, (int)h_cross_jobs.size(), terms, S, (int)nS);
    hipLaunchKernelGGL(schur_pin_kernel, dim3(nblk(nS), (unsigned)nS), dim3(256), 0, st, act_hub,
                       (int)nS, S, rhs);
    GMGM_HIP(c, hipMemsetAsync(ginfo, 0, (groups.size() + 1) * sizeof(int), st));
    GMGM_TRY(block_arrow_solve());
    hipLaunchKernelGGL(hub_step_kernel, dim3(nblk(T)), dim3(256), 0, st, rhs, g, h, act, (int)T, lam, lm ? 1 : 0,
                       d);
    std::vector<int> bad(groups.size() + 1, 0);
    GMGM_HIP(c, hipMemcpyAsync(bad.data(), ginfo, bad.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
    for (int b : bad)
      if (b) return set_err(c, GMGM_E_NOCONV, "Newton system is not positive definite");
    return GMGM_OK;
  }

  // Solves S x = rhs in place (S symmetric positive definite, block-arrow).
  // S is symmetric, so its row-major storage is also the column-major matrix
  // that the library routines take (leading dimension nS); rhs directly follows
  // S, so it is that matrix's column nS.  Per group g: A_g = L_g L_g^T, then
  // one triangular solve with the group's rows of the shared columns and of
  // rhs (B_g <- L_g^-1 B_g, y_g = L_g^-1 rhs_g); then the shared block's Schur complement
  // C - sum_g B_g^T B_g (hub_schur_kernel: the groups are contiguous) and
  // right-hand side rhs_h - sum_g B_g^T y_g (hub_rhs_kernel), its Cholesky
  // solve, y <- y - B x_h
  // and x_g = L_g^-T y_g.  Groups of one common size go through strided-batched
  // calls.  Flags of the factorisations: ginfo[g], ginfo[G] for the shared block.
  gmgm_status block_arrow_solve() {
    void* hv;
    GMGM_TRY(blas_handle(c, &hv));
    rocblas_handle bh = (rocblas_handle)hv;
    const rocblas_int ld = (rocblas_int)nS, nh = (rocblas_int)(nS - hub_off), G = (rocblas_int)groups.size();
    const rocblas_int k = (rocblas_int)hub_off;
    const double one = 1.0, minus = -1.0;
    bool ok = true;
    auto chk = [&](rocblas_status r) { ok = ok && r == rocblas_status_success; };
    bool equal = G > 1;
    for (auto& gp : groups) equal = equal && gp.second == groups[0].second;
    double* Bh = S + hub_off * nS;   // column hub_off, row 0: all groups' rows of the shared columns
    if (equal) {
      const rocblas_int p = (rocblas_int)groups[0].second;
      const rocblas_stride sa = (rocblas_stride)p * (ld + 1);
      chk(rocsolver_dpotrf_strided_batched(bh, rocblas_fill_lower, p, S, ld, sa, ginfo, G));
      chk(rocblas_dtrsm_strided_batched(bh, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                                        rocblas_diagonal_non_unit, p, nh + 1, &one, S, ld, sa, Bh, ld, p, G));
    } else {
      for (rocblas_int q = 0; q < G; ++q) {
        const rocblas_int o = (rocblas_int)groups[q].first, p = (rocblas_int)groups[q].second;
        double* A = S + (size_t)o * nS + o;
        chk(rocsolver_dpotrf(bh, rocblas_fill_lower, p, A, ld, ginfo + q));
        chk(rocblas_dtrsm(bh, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                          rocblas_diagonal_non_unit, p, nh + 1, &one, A, ld, Bh + o, ld));
      }
    }
    if (nh > 0) {
      double* C = S + hub_off * nS + hub_off;
      if (k > 0) {
        const unsigned nt = nblk(nh, 16);
        hipLaunchKernelGGL(hub_schur_kernel, dim3(nt, nt, (unsigned)hub_slices), dim3(256), 0, st, S, (int)ld, (int)k,
                           (int)nh, hub_slices, hub_part);
        hipLaunchKernelGGL(hub_schur_reduce_kernel, dim3(nblk(nh), (unsigned)nh), dim3(256), 0, st, S, (int)ld, (int)k,
                           (int)nh, hub_slices, hub_part);
        hipLaunchKernelGGL(hub_rhs_kernel, dim3(nblk(nh, 4)), dim3(256), 0, st, S, (int)ld, (int)k, (int)nh, rhs);
      }
      chk(rocsolver_dpotrf(bh, rocblas_fill_lower, nh, C, ld, ginfo + G));
      chk(rocsolver_dpotrs(bh, rocblas_fill_lower, nh, 1, C, ld, rhs + hub_off, nh));
      if (k > 0)
        chk(rocblas_dgemv(bh, rocblas_operation_none, k, nh, &minus, Bh, ld, rhs + hub_off, 1, &one, rhs, 1));
    }
    if (equal) {
      const rocblas_int p = (rocblas_int)groups[0].second;
      chk(rocblas_dtrsv_strided_batched(bh, rocblas_fill_lower, rocblas_operation_transpose, rocblas_diagonal_non_unit,
                                        p, S, ld, (rocblas_stride)p * (ld + 1), rhs, 1, p, G));
    } else {
      for (rocblas_int q = 0; q < G; ++q) {
        const rocblas_int o = (rocblas_int)groups[q].first, p = (rocblas_int)groups[q].second;
        chk(rocblas_dtrsv(bh, rocblas_fill_lower, rocblas_operation_transpose, rocblas_diagonal_non_unit, p,
                          S + (size_t)o * nS + o, ld, rhs + o, 1));
      }
    }
    if (!ok) return set_err(c, GMGM_E_HIP, "rocBLAS or rocSOLVER call failed in the Newton solve");
    return GMGM_OK;
  }
};

// Start point, domain checks, bounds, the Newton iteration and the gauge rule,
// shared by both solvers (SV supplies nll, gradient and direction).
template <class SV>
gmgm_status drive(SV& sv, const double* const* E, const double* eps, const double* const* warm, double tol,
                  int32_t max_iter, double* const* lambda_out, gmgm_solve_info* info) {
  gmgm_ctx* c = sv.c;
  const int n_axes = sv.L;
  hipStream_t st = sv.st;
  const size_t T = sv.T;
  // E, the start point, domain checks, traces and largest E of each axis
  GMGM_HIP(c, hipMemsetAsync(sv.flag, 0, sizeof(int), st));
  for (int l = 0; l < n_axes; ++l) {
    const Axis& a = sv.ax[l];
    GMGM_HIP(c, hipMemcpyAsync(sv.Ec + a.off, E[l], a.r * sizeof(double), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(init_kernel, dim3(nblk(a.r)), dim3(256), 0, st, sv.Ec + a.off,
                       warm ? warm[l] : (const double*)nullptr, a.r, sv.lam + a.off, sv.flag);
    hipLaunchKernelGGL(init_kernel, dim3(nblk(a.r)), dim3(256), 0, st, sv.Ec + a.off,
                       (const double*)nullptr, a.r, sv.trial + a.off, sv.flag);
    hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(RED_THREADS), 0, st, sv.Ec + a.off,
                       (const double*)nullptr, a.r, sv.scal + 2 * l);
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(RED_THREADS), 0, st, sv.Ec + a.off, a.r,
                       sv.scal + 2 * l + 1);
  }
  int bad = 0;
  GMGM_HIP(c, hipMemcpyAsync(&bad, sv.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  std::vector<double> tr(2 * n_axes);
  GMGM_TRY(sv.fetch(tr.data(), sv.scal, 2 * n_axes));
  if (bad == 1) return set_err(c, GMGM_E_DOMAIN, "every E must be positive and finite");
  if (bad == 2) return set_err(c, GMGM_E_DOMAIN, "the warm start must be finite");
  for (int l = 0; l < n_axes; ++l) {
    sv.ax[l].trace = tr[2 * l];
    sv.ax[l].eps = eps ? eps[l] : 1e-10 / tr[2 * l + 1];
  }
  GMGM_TRY(sv.upload_eps());
  sv.clip(sv.trial);
  // the gauge of Algorithm 1's start max(1/E, eps) along each flat direction
  const auto flats = flat_directions(sv.ax, sv.sets);
  std::vector<double> target(flats.size(), 0.0), sums, mins;
  if (!flats.empty()) {
    GMGM_TRY(sv.axis_stats(sv.trial, sums, mins));
    for (size_t q = 0; q < flats.size(); ++q) target[q] = SV::gauge_value(sums, flats[q]);
  }
  // back to that gauge, as near as the box allows
  auto fix_gauge = [&](double* v) -> gmgm_status {
    if (flats.empty()) return GMGM_OK;
    GMGM_TRY(sv.axis_stats(v, sums, mins));
    std::vector<double> t_star(flats.size());
    for (size_t q = 0; q < flats.size(); ++q) t_star[q] = target[q] - SV::gauge_value(sums, flats[q]);
    const std::vector<double> t = nearest_feasible_shift(t_star, flats, sv.ax, mins.data());
    for (int l = 0; l < n_axes; ++l) {
      double u = 0;
      for (size_t q = 0; q < flats.size(); ++q) u += t[q] * flats[q][l];
      if (u != 0.0)
        hipLaunchKernelGGL(add_const_kernel, dim3(nblk(sv.ax[l].r)), dim3(256), 0, st, v + sv.ax[l].off,
                           sv.ax[l].r, u);
    }
    return GMGM_OK;
  };
  if (warm) GMGM_TRY(fix_gauge(sv.lam));
  sv.clip(sv.lam);
  bool warm_used = false;
  if (warm) {
    // a supplied start is used when its NLL is not above that of 1/E (held in trial)
    double f_warm, f_cold;
    GMGM_TRY(sv.nll(sv.lam, &f_warm));
    GMGM_TRY(sv.nll(sv.trial, &f_cold));
    warm_used = f_warm <= f_cold;
    if (!warm_used)
      GMGM_HIP(c, hipMemcpyAsync(sv.lam, sv.trial, T * sizeof(double), hipMemcpyDeviceToDevice, st));
  }

  double kres = 0;
  GMGM_TRY(sv.gradient(sv.lam, &kres));
  int it = 0;
  bool stalled = false;
  for (int round = 0; round < 3; ++round) {
    stalled = false;
    while (kres > tol && it < max_iter) {
      it++;
      double f0;
      GMGM_TRY(sv.nll(sv.lam, &f0));
      // steps may drift along flat directions (the NLL is constant there)
      GMGM_TRY(sv.direction(std::min(1e-2, kres)));
      // Backtracking over alpha = 2^-s, s = 0 .. 59: the first length that
      // satisfies Armijo is taken.  alpha = 1 is tried alone, later lengths
      // eight at a time with one read-back; the choice and the trial point are
      // those of trying the lengths one by one.
      double alpha = 1.0;
      bool accepted = false;
      for (int tried = 0; !accepted && tried < 60;) {
        const int nb = tried == 0 ? 1 : std::min(8, 60 - tried);
        for (int b = 0; b < nb; ++b) {
          const double a = std::ldexp(1.0, -(tried + b));
          sv.trial_point(a);
          hipLaunchKernelGGL(pred_kernel, dim3(1), dim3(RED_THREADS), 0, st, sv.g, sv.d, sv.lam, sv.trial,
                             sv.act, (int)T, a, sv.scal + 3 * b + 2);
          GMGM_TRY(sv.nll_launch(sv.trial, sv.scal + 3 * b));
        }
        double v[24];
        GMGM_TRY(sv.fetch(v, sv.scal, 3 * nb));
        for (int b = 0; b < nb && !accepted; ++b) {
          const double f1 = 0.5 * (v[3 * b] - v[3 * b + 1]), pred = v[3 * b + 2];
          if (f1 <= f0 + 1e-4 * pred || std::fabs(pred) <= 1e-13 * (std::fabs(f0) + 1.0)) {
            accepted = true;
            alpha = std::ldexp(1.0, -(tried + b));
            if (b != nb - 1) sv.trial_point(alpha);   // trial holds the last length tried
          }
        }
        tried += nb;
      }
      if (!accepted) {
        stalled = true;
        break;
      }
      std::swap(sv.lam, sv.trial);
      sv.lm = it >= sv.lm_after;
      GMGM_TRY(sv.gradient(sv.lam, &kres));
    }
    // back to the start's gauge along the flat directions; resume if that moved
    // the point off the tolerance (rounding of the shift, the box)
    GMGM_TRY(fix_gauge(sv.lam));
    sv.clip(sv.lam);
    GMGM_TRY(sv.gradient(sv.lam, &kres));
    if (kres <= tol || it >= max_iter || stalled || flats.empty()) break;
  }
  for (int l = 0; l < n_axes; ++l)
    GMGM_HIP(c, hipMemcpyAsync(lambda_out[l], sv.lam + sv.ax[l].off, sv.ax[l].r * sizeof(double),
                               hipMemcpyDeviceToDevice, st));
  if (info) {
    // the record's per-axis arrays hold the first MAX_AXES axes
    const int nrec = std::min(n_axes, MAX_AXES);
    for (int l = 0; l < nrec; ++l)
      hipLaunchKernelGGL(count_pinned_kernel, dim3(1), dim3(RED_THREADS), 0, st, sv.lam + sv.ax[l].off,
                         sv.ax[l].eps, sv.ax[l].r, sv.scal + 4 + l);
    double np[MAX_AXES];
    GMGM_TRY(sv.fetch(np, sv.scal + 4, nrec));
    *info = gmgm_solve_info{};
    info->iterations = it;
    info->converged = kres <= tol;
    info->n_flat = (int32_t)flats.size();
    info->warm_used = warm_used ? 1 : 0;
    info->kkt = kres;
    for (int l = 0; l < nrec; ++l) {
      info->n_pinned[l] = (int64_t)np[l];
      info->eps[l] = sv.ax[l].eps;
    }
  }
  GMGM_HIP(c, hipStreamSynchronize(st));
  if (kres > tol)
    return set_err(c, GMGM_E_NOCONV, "KKT residual %.3g after %d iterations%s", kres, it,
                   stalled ? " (line search stalled)" : "");
  return GMGM_OK;
}

}  // namespace gmgm_sv

using namespace gmgm_sv;

extern "C" gmgm_status gmgm_solve_eigs(gmgm_ctx_t c, int32_t n_axes, const int64_t* ranks,
                                       const double* const* E, int32_t n_mod,
                                       const int32_t* modalities, const double* eps,
                                       const double* const* warm, double tol, int32_t max_iter,
                                       double* const* lambda_out, gmgm_solve_info* info) {
  GMGM_CHECK_CTX(c);
  if (n_axes < 2 || n_axes > MAX_AXES) return set_err(c, GMGM_E_ARG, "n_axes must be in [2, 8]");
  if (n_mod < 1 || n_mod > n_axes * (n_axes - 1) / 2)
    return set_err(c, GMGM_E_ARG, "n_mod must be in [1, n_axes (n_axes - 1) / 2]");
  if (!ranks || !E || !modalities || !lambda_out) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (!(tol > 0) || max_iter < 0) return set_err(c, GMGM_E_ARG, "need tol > 0 and max_iter >= 0");
  Solver sv;
  sv.c = c;
  sv.st = c->stream;
  sv.L = n_axes;
  sv.ax.resize(n_axes);
  for (int l = 0; l < n_axes; ++l) {
    if (ranks[l] < 1 || ranks[l] > (1 << 26))
      return set_err(c, GMGM_E_SHAPE, "axis %d: rank %lld outside [1, 2^26]", l, (long long)ranks[l]);
    if (!E[l] || !lambda_out[l] || (warm && !warm[l]))
      return set_err(c, GMGM_E_ARG, "axis %d: null pointer", l);
    if (eps && !(eps[l] > 0 && std::isfinite(eps[l])))
      return set_err(c, GMGM_E_DOMAIN, "axis %d: eps must be positive and finite", l);
    sv.ax[l].r = (int)ranks[l];
    sv.ax[l].off = sv.T;
    sv.T += sv.ax[l].r;
  }
  if (sv.T > (size_t)1 << 28) return set_err(c, GMGM_E_SHAPE, "total rank too large");
  std::vector<int> used(n_axes, 0);
  for (int t = 0; t < n_mod; ++t) {
    const int a = modalities[2 * t], b = modalities[2 * t + 1];
    if (a < 0 || b < 0 || a >= n_axes || b >= n_axes || a == b)
      return set_err(c, GMGM_E_ARG, "modality %d joins invalid axes (%d, %d)", t, a, b);
    for (auto& m : sv.mods)
      if ((m.first == a && m.second == b) || (m.first == b && m.second == a))
        return set_err(c, GMGM_E_ARG, "modality %d repeats the axis pair (%d, %d)", t, a, b);
    sv.mods.push_back({a, b});
    sv.sets.push_back({a, b});
    used[a] = used[b] = 1;
  }
  for (int l = 0; l < n_axes; ++l)
    if (!used[l]) return set_err(c, GMGM_E_ARG, "axis %d belongs to no modality", l);
  sv.lm_after = 30;   // escape mode, as in the tensor solver (near-balanced pairs)
  sv.hub = hub_axes(sv.ax, sv.mods);
  sv.is_hub.assign(n_axes, 0);
  sv.hoff.assign(n_axes, 0);
  for (int l : sv.hub) {
    sv.is_hub[l] = 1;
    sv.hoff[l] = sv.nS;
    sv.nS += sv.ax[l].r;
  }
  if (sv.nS > (size_t)MAX_HUB)
    return set_err(c, GMGM_E_SHAPE, "the Schur system has %zu unknowns (at most %d)", sv.nS, MAX_HUB);
  GMGM_HIP(c, hipSetDevice(c->device));
  GMGM_TRY(sv.bind_workspace());
  GMGM_TRY(sv.plan_splits());
  return drive(sv, E, eps, warm, tol, max_iter, lambda_out, info);
}

extern "C" gmgm_status gmgm_solve_eigs_tensor(gmgm_ctx_t c, int32_t n_axes, const int64_t* ranks,
                                              const double* const* E, int32_t n_mod, const int32_t* mod_len,
                                              const int32_t* mod_axes, const double* eps,
                                              const double* const* warm, double tol, int32_t max_iter,
                                              double* const* lambda_out, gmgm_solve_info* info) {
  GMGM_CHECK_CTX(c);
  if (n_axes < 2 || n_axes > MAX_TAXES) return set_err(c, GMGM_E_ARG, "n_axes must be in [2, %d]", MAX_TAXES);
  if (n_mod < 1 || n_mod > MAX_TAXES) return set_err(c, GMGM_E_ARG, "n_mod must be in [1, %d]", MAX_TAXES);
  if (!ranks || !E || !mod_len || !mod_axes || !lambda_out) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (!(tol > 0) || max_iter < 0) return set_err(c, GMGM_E_ARG, "need tol > 0 and max_iter >= 0");
  TensorSolver sv;
  sv.c = c;
  sv.st = c->stream;
  sv.L = n_axes;
  // nearly balanced modalities (traces equal to a few ulps of the spectra's
  // precision) leave a direction of tiny slope whose minimiser lies on the
  // box far away; the default rule crawls along it, the escape mode reaches it
  sv.lm_after = 30;
  sv.ax.resize(n_axes);
  for (int l = 0; l < n_axes; ++l) {
    if (ranks[l] < 1 || ranks[l] > MAX_DENSE)
      return set_err(c, GMGM_E_SHAPE, "axis %d: rank %lld outside [1, %d]", l, (long long)ranks[l], MAX_DENSE);
    if (!E[l] || !lambda_out[l] || (warm && !warm[l]))
      return set_err(c, GMGM_E_ARG, "axis %d: null pointer", l);
    if (eps && !(eps[l] > 0 && std::isfinite(eps[l])))
      return set_err(c, GMGM_E_DOMAIN, "axis %d: eps must be positive and finite", l);
    sv.ax[l].r = (int)ranks[l];
    sv.ax[l].off = sv.T;
    sv.T += sv.ax[l].r;
  }
  if (sv.T > (size_t)MAX_DENSE)
    return set_err(c, GMGM_E_SHAPE, "the Newton system has %zu unknowns (at most %d)", sv.T, MAX_DENSE);
  std::vector<int> used(n_axes, 0);
  int pos = 0;
  for (int t = 0; t < n_mod; ++t) {
    const int K = mod_len[t];
    if (K < 2 || K > std::min(n_axes, MAX_AXES))
      return set_err(c, GMGM_E_ARG, "modality %d has %d axes (need 2 .. min(n_axes, %d))", t, K, MAX_AXES);
    std::vector<int> m(mod_axes + pos, mod_axes + pos + K);
    pos += K;
    double tuples = 1.0;
    for (int u = 0; u < K; ++u) {
      if (m[u] < 0 || m[u] >= n_axes) return set_err(c, GMGM_E_ARG, "modality %d names axis %d", t, m[u]);
      for (int u2 = 0; u2 < u; ++u2)
        if (m[u2] == m[u]) return set_err(c, GMGM_E_ARG, "modality %d repeats axis %d", t, m[u]);
      tuples *= sv.ax[m[u]].r;
      used[m[u]] = 1;
    }
    if (tuples > 1099511627776.0)
      return set_err(c, GMGM_E_SHAPE, "modality %d has %.3g index tuples (at most 2^40)", t, tuples);
    // bounded work per wave (the tuples of one index: the other K - 1 ranks)
    // and per cross-block thread (the other K - 2 ranks)
    std::vector<double> rk;
    for (int a : m) rk.push_back((double)sv.ax[a].r);
    std::sort(rk.begin(), rk.end());
    double rest1 = 1.0, rest2 = 1.0;
    for (int u = 1; u < K; ++u) rest1 *= rk[u];
    for (int u = 2; u < K; ++u) rest2 *= rk[u];
    if (rest1 > 4294967296.0 || rest2 > 67108864.0)
      return set_err(c, GMGM_E_SHAPE,
                     "modality %d: %.3g tuples per index of its smallest axis (at most 2^32) or %.3g per entry "
                     "of a cross block (at most 2^26)",
                     t, rest1, rest2);
    std::vector<int> key = m;
    std::sort(key.begin(), key.end());
    for (auto& q : sv.sets) {
      std::vector<int> k2 = q;
      std::sort(k2.begin(), k2.end());
      if (k2 == key) return set_err(c, GMGM_E_ARG, "modality %d repeats the axes of an earlier one", t);
    }
    sv.sets.push_back(m);
  }
  for (int l = 0; l < n_axes; ++l)
    if (!used[l]) return set_err(c, GMGM_E_ARG, "axis %d belongs to no modality", l);
  // coordinate order: each modality's private axes together, then the shared axes
  std::vector<int> n_of(n_axes, 0);
  for (auto& m : sv.sets)
    for (int a : m) n_of[a]++;
  size_t off = 0;
  for (auto& m : sv.sets) {
    const size_t o = off;
    for (int a : m)
      if (n_of[a] == 1) {
        sv.ax[a].off = off;
        off += sv.ax[a].r;
      }
    if (off > o) sv.groups.push_back({o, off - o});
  }
  sv.hub_off = off;
  for (int l = 0; l < n_axes; ++l)
    if (n_of[l] > 1) {
      sv.ax[l].off = off;
      off += sv.ax[l].r;
    }
  sv.nS = sv.T;
  GMGM_HIP(c, hipSetDevice(c->device));
  GMGM_TRY(sv.bind_workspace());
  GMGM_TRY(sv.prepare());
  return drive(sv, E, eps, warm, tol, max_iter, lambda_out, info);
}
