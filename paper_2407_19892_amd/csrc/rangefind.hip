// Leading eigenpairs of an axis too large for its Gram: randomized subspace
// iteration (Halko, Martinsson and Tropp 2011) on S = D D^T with
// D = [X_1 | X_2 | ...], the concatenation of the modalities sharing the axis
// (Notation section; S's eigenvectors are D's left singular vectors,
// Algorithm 1's first loop).
//
//   Y = D Omega;  Q = orth(Y);  q times: Q' = orth(D^T Q), Q = orth(D Q');
//   Z = D^T Q;  T = Z^T Z = W diag(theta) W^T;  E = theta[:r], V = Q W[:, :r]
//
// The sparse products are this file's kernels: a CSR transpose (count, scan,
// atomic-cursor scatter) and a wave-per-row SpMM that gathers FP64 panel rows
// and accumulates in FP64.  The small dense steps are plain library linear
// algebra on the context stream: orth() is CholeskyQR2 (rocBLAS dgemm for
// Y^T Y, rocSOLVER dpotrf, rocBLAS dtrsm for Y L^-T), which gives the Q factor
// with a positive R diagonal; the k x k eigenproblem is rocSOLVER dsyevd; the
// final Q W is a dgemm.  Within a transposed row the scatter order is not
// fixed, so results are reproducible up to FP64 summation order.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <vector>

#include "gmgm_internal.h"

namespace gmgm_rf {

__global__ void count_kernel(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t n, int64_t p,
                             int64_t nnz, unsigned long long* __restrict__ cnt, int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  if (b < 0 || e < b || e > nnz) {
    if (lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
    return;
  }
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    if (c < 0 || c >= p) {
      atomicCAS(status, 0, DEV_BADINDEX);
      continue;
    }
    atomicAdd(&cnt[c], 1ull);
  }
}

// Exclusive scan of cnt (p entries) into out (p + 1 entries) and cursor; one workgroup.
__global__ void __launch_bounds__(1024) scan_kernel(const unsigned long long* __restrict__ cnt, int64_t p,
                                                    int64_t* __restrict__ out,
                                                    unsigned long long* __restrict__ cursor) {
  __shared__ unsigned long long part[1024];
  const int t = threadIdx.x;
  const int64_t per = (p + 1023) / 1024;
  const int64_t lo = std::min<int64_t>(p, t * per), hi = std::min<int64_t>(p, lo + per);
  unsigned long long s = 0;
  for (int64_t j = lo; j < hi; ++j) s += cnt[j];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    unsigned long long run = 0;
    for (int q = 0; q < 1024; ++q) {
      const unsigned long long v = part[q];
      part[q] = run;
      run += v;
    }
    out[p] = (int64_t)run;
  }
  __syncthreads();
  unsigned long long run = part[t];
  for (int64_t j = lo; j < hi; ++j) {
    out[j] = (int64_t)run;
    cursor[j] = run;
    run += cnt[j];
  }
}

__global__ void scatter_kernel(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const float* __restrict__ val, int64_t n, int64_t p, int64_t nnz,
                               unsigned long long* __restrict__ cursor, int32_t* __restrict__ row_out,
                               float* __restrict__ val_out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  if (b < 0 || e < b || e > nnz) return;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    if (c < 0 || c >= p) continue;
    const unsigned long long pos = atomicAdd(&cursor[c], 1ull);
    row_out[pos] = (int32_t)i;
    val_out[pos] = val ? val[t] : 1.0f;
  }
}

// Y[i][0:k] (+)= sum_t val[t] B[col[t]][0:k]; B FP64 (p x ldb), Y FP64 (n x ldy);
// lane l owns columns [W l, W l + W) (W = ceil(k / 64) <= 2).
template <int W>
__global__ void __launch_bounds__(256) spmm64_kernel(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const float* __restrict__ val, int64_t n, int64_t p,
                                                     int64_t nnz, const double* __restrict__ B, int64_t ldb, int k,
                                                     double* __restrict__ Y, int64_t ldy, int accumulate,
                                                     int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double acc[W];
#pragma unroll
  for (int q = 0; q < W; ++q) acc[q] = 0.0;
  const int64_t b = rp[i], e = rp[i + 1];
  bool bad = false;
  if (b < 0 || e < b || e > nnz) {
    bad = true;
  } else {
    for (int64_t t0 = b; t0 < e; t0 += 64) {
      const int64_t t = t0 + lane;
      int cc = 0;
      float vv = 0.0f;
      if (t < e) {
        cc = col[t];
        vv = val ? val[t] : 1.0f;
        if (cc < 0 || cc >= p) {
          bad = true;
          cc = 0;
          vv = 0.0f;
        }
      }
      const int m = e - t0 < 64 ? (int)(e - t0) : 64;
      for (int j = 0; j < m; ++j) {
        const int c = __builtin_amdgcn_readlane(cc, j);
        const double v = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), j));
        const double* br = B + (size_t)c * ldb;
#pragma unroll
        for (int q = 0; q < W; ++q) {
          const int jc = lane * W + q;
          if (jc < k) acc[q] += v * br[jc];
        }
      }
    }
  }
  if (__ballot(bad) && lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
  double* yr = Y + (size_t)i * ldy;
#pragma unroll
  for (int q = 0; q < W; ++q) {
    const int jc = lane * W + q;
    if (jc < k) yr[jc] = accumulate ? yr[jc] + acc[q] : acc[q];
  }
}

// Eigenpairs ascending (w, W col-major k x k) -> descending; theta[j] = w[k-1-j],
// Wd column j = W column k-1-j.
__global__ void reorder_kernel(const double* __restrict__ w, const double* __restrict__ Wm, int k,
                               double* __restrict__ theta, double* __restrict__ Wd) {
  const int j = blockIdx.x, i = threadIdx.x;
  if (i < k) Wd[(size_t)j * k + i] = Wm[(size_t)(k - 1 - j) * k + i];
  if (i == 0) theta[j] = w[k - 1 - j];
}

__global__ void to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

inline unsigned nb(int64_t n, int b = 256) {
  return (unsigned)std::min<int64_t>((n + b - 1) / b, (int64_t)1 << 30);
}

gmgm_status check_csr(gmgm_ctx* c, const gmgm_csr& m, const char* what) {
  if (m.n_rows < 1 || m.n_cols < 1 || m.nnz < 0 || m.n_rows > INT32_MAX || m.n_cols > INT32_MAX)
    return set_err(c, GMGM_E_SHAPE, "%s: need n_rows, n_cols in [1, 2^31) and nnz >= 0", what);
  if (!m.row_ptr || (m.nnz > 0 && !m.col)) return set_err(c, GMGM_E_ARG, "%s: null pointer", what);
  return GMGM_OK;
}

gmgm_status spmm(gmgm_ctx* c, const gmgm_csr& m, const double* B, int64_t ldb, int k, double* Y, int64_t ldy,
                 int accumulate) {
  const dim3 grid((unsigned)((m.n_rows + 3) / 4));
  if (k <= 64)
    hipLaunchKernelGGL(spmm64_kernel<1>, grid, dim3(256), 0, c->stream, m.row_ptr, m.col, m.val, m.n_rows, m.n_cols,
                       m.nnz, B, ldb, k, Y, ldy, accumulate, c->dev_status);
  else
    hipLaunchKernelGGL(spmm64_kernel<2>, grid, dim3(256), 0, c->stream, m.row_ptr, m.col, m.val, m.n_rows, m.n_cols,
                       m.nnz, B, ldb, k, Y, ldy, accumulate, c->dev_status);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

#define RB(expr)                                                                        \
  do {                                                                                  \
    rocblas_status s__ = (expr);                                                        \
    if (s__ != rocblas_status_success) return set_err(c, GMGM_E_HIP, "%s failed (%d)", #expr, (int)s__); \
  } while (0)

// Y (m x k, row-major = column-major k x m) <- Q factor of Y with positive R diagonal (CholeskyQR2).
gmgm_status orth(gmgm_ctx* c, rocblas_handle h, double* Y, int64_t m, int k, double* G, int* info) {
  const double one = 1.0, zero = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    // G = Y^T Y (column-major k x k): (Y^T)(Y^T)^T with Y^T stored k x m
    RB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, k, k, (rocblas_int)m, &one, Y, k, Y, k,
                     &zero, G, k));
    RB(rocsolver_dpotrf(h, rocblas_fill_lower, k, G, k, info));
    int hinfo = 0;
    GMGM_HIP(c, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    GMGM_HIP(c, hipStreamSynchronize(c->stream));
    if (hinfo != 0)
      return set_err(c, GMGM_E_NOCONV, "subspace basis is numerically rank deficient (Cholesky pivot %d)", hinfo);
    // Y^T <- L^-1 Y^T, i.e. Y <- Y L^-T
    RB(rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, k,
                     (rocblas_int)m, &one, G, k, Y, k));
  }
  return GMGM_OK;
}

}  // namespace gmgm_rf

using namespace gmgm_rf;

extern "C" gmgm_status gmgm_csr_transpose(gmgm_ctx_t c, gmgm_csr X, int64_t* row_ptr_t, int32_t* col_t,
                                          float* val_t) {
  GMGM_CHECK_CTX(c);
  GMGM_TRY(check_csr(c, X, "X"));
  if (!row_ptr_t || (X.nnz > 0 && (!col_t || !val_t))) return set_err(c, GMGM_E_ARG, "null output pointer");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  void* w;
  GMGM_TRY(ws_get(c, WS_RF0, (size_t)X.n_cols * 2 * sizeof(unsigned long long), &w));
  unsigned long long* cnt = (unsigned long long*)w;
  unsigned long long* cursor = cnt + X.n_cols;
  GMGM_HIP(c, hipMemsetAsync(cnt, 0, X.n_cols * sizeof(unsigned long long), st));
  const dim3 grid((unsigned)((X.n_rows + 3) / 4));
  hipLaunchKernelGGL(count_kernel, grid, dim3(256), 0, st, X.row_ptr, X.col, X.n_rows, X.n_cols, X.nnz, cnt,
                     c->dev_status);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, cnt, X.n_cols, row_ptr_t, cursor);
  hipLaunchKernelGGL(scatter_kernel, grid, dim3(256), 0, st, X.row_ptr, X.col, X.val, X.n_rows, X.n_cols, X.nnz,
                     cursor, col_t, val_t);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_subspace_eig(gmgm_ctx_t c, int32_t n_blocks, const gmgm_csr* blocks,
                                         const gmgm_csr* blocks_t, const double* omega, int64_t k, int32_t q,
                                         int64_t r, double* evals, float* vecs) {
  GMGM_CHECK_CTX(c);
  if (n_blocks < 1 || n_blocks > 16 || !blocks || !blocks_t || !omega || !evals || !vecs)
    return set_err(c, GMGM_E_ARG, "need 1..16 blocks and non-null pointers");
  if (k < 1 || k > 128 || r < 1 || r > k || q < 0 || q > 64)
    return set_err(c, GMGM_E_ARG, "need 1 <= r <= k <= 128 and 0 <= q <= 64");
  const int64_t n = blocks[0].n_rows;
  std::vector<int64_t> off(n_blocks + 1, 0);
  for (int m = 0; m < n_blocks; ++m) {
    GMGM_TRY(check_csr(c, blocks[m], "block"));
    GMGM_TRY(check_csr(c, blocks_t[m], "transposed block"));
    if (blocks[m].n_rows != n || blocks_t[m].n_rows != blocks[m].n_cols || blocks_t[m].n_cols != n ||
        blocks_t[m].nnz != blocks[m].nnz)
      return set_err(c, GMGM_E_SHAPE, "block %d: shapes of the block and its transpose disagree", m);
    off[m + 1] = off[m] + blocks[m].n_cols;
  }
  const int64_t P = off[n_blocks];
  if (k > std::min(n, P)) return set_err(c, GMGM_E_SHAPE, "k must not exceed min(n, total columns)");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  void* hv;
  GMGM_TRY(blas_handle(c, &hv));
  rocblas_handle h = (rocblas_handle)hv;
  void *w1, *w2;
  GMGM_TRY(ws_get(c, WS_RF1, ((size_t)(n + P) * k + (size_t)n * r) * sizeof(double), &w1));
  GMGM_TRY(ws_get(c, WS_RF2, (size_t)(3 * k * k + 2 * k + 16) * sizeof(double), &w2));
  double* Y = (double*)w1;          // n x k, row-major
  double* Z = Y + (size_t)n * k;    // P x k, row-major
  double* Vt = Z + (size_t)P * k;   // V, n x r row-major (column-major r x n)
  double* G = (double*)w2;          // k x k
  double* Wm = G + k * k;
  double* Wd = Wm + k * k;
  double* wv = Wd + k * k;
  double* theta = wv + k;
  int* info = (int*)(theta + k);
  const int K = (int)k;
  hipEvent_t ev = timing_start(c);
  auto d_times = [&](const double* B, double* out) -> gmgm_status {   // out = D B (B: P x k)
    for (int m = 0; m < n_blocks; ++m) GMGM_TRY(spmm(c, blocks[m], B + off[m] * k, k, K, out, k, m > 0));
    return GMGM_OK;
  };
  auto dt_times = [&](const double* B, double* out) -> gmgm_status {  // out = D^T B (B: n x k)
    for (int m = 0; m < n_blocks; ++m) GMGM_TRY(spmm(c, blocks_t[m], B, k, K, out + off[m] * k, k, 0));
    return GMGM_OK;
  };
  GMGM_TRY(d_times(omega, Y));
  GMGM_TRY(orth(c, h, Y, n, K, G, info));
  for (int t = 0; t < q; ++t) {
    GMGM_TRY(dt_times(Y, Z));
    GMGM_TRY(orth(c, h, Z, P, K, G, info));
    GMGM_TRY(d_times(Z, Y));
    GMGM_TRY(orth(c, h, Y, n, K, G, info));
  }
  GMGM_TRY(dt_times(Y, Z));
  const double one = 1.0, zero = 0.0;
  // T = Z^T Z (k x k), its eigenpairs ascending, then descending
  RB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, K, K, (rocblas_int)P, &one, Z, K, Z, K,
                   &zero, Wm, K));
  RB(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_lower, K, Wm, K, wv, G, info));
  hipLaunchKernelGGL(reorder_kernel, dim3((unsigned)K), dim3(128), 0, st, wv, Wm, K, theta, Wd);
  // V = Q W[:, :r]: row-major n x r = column-major V^T (r x n) = W[:, :r]^T Q^T
  RB(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)r, (rocblas_int)n, K, &one,
                   Wd, K, Y, K, &zero, Vt, (rocblas_int)r));
  hipLaunchKernelGGL(to_f32_kernel, dim3(nb(n * r)), dim3(256), 0, st, Vt, vecs, n * r);
  GMGM_HIP(c, hipMemcpyAsync(evals, theta, r * sizeof(double), hipMemcpyDeviceToDevice, st));
  timing_stop(c, ev);
  int hinfo = 0;
  GMGM_HIP(c, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipStreamSynchronize(st));
  if (hinfo != 0) return set_err(c, GMGM_E_NOCONV, "rocsolver_dsyevd reported %d", hinfo);
  return GMGM_OK;
}
