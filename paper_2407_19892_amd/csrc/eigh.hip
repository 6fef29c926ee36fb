// FP64 eigendecomposition of the small-axis Gram (Algorithm 1's first loop:
// the eigenvectors of S_l are the MLE's eigenvectors by Theorem 1).
//
// The FP32 Gram is promoted to FP64 and handed to rocSOLVER's divide-and-
// conquer symmetric eigensolver (tridiagonal reduction + divide and conquer);
// a kernel then reorders the pairs to descending eigenvalues and counts the
// numerical rank #{e_i > p 2^-52 e_1}.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>

#include "gmgm_internal.h"

namespace gmgm_eh {

// A (col-major FP64) = G (row-major FP32) read as its transpose; G symmetric.
__global__ void promote_kernel(const float* __restrict__ G, int64_t n_el, double* __restrict__ A,
                               int* __restrict__ status) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_el;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = G[i];
    bad |= !isfinite(v);
    A[i] = (double)v;
  }
  if (bad) atomicCAS(status, 0, DEV_NONFINITE);
}

// evals_desc[j] = w[p-1-j]; column j of evecs = column p-1-j of A.
__global__ void reorder_kernel(const double* __restrict__ A, const double* __restrict__ w, int64_t p,
                               double* __restrict__ evals, double* __restrict__ evecs) {
  const int64_t j = blockIdx.y;
  const double* src = A + (size_t)(p - 1 - j) * p;
  double* dst = evecs + (size_t)j * p;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) evals[j] = w[p - 1 - j];
}

// evals_desc[j] = w[p-1-j] (no eigenvectors)
__global__ void reorder_values_kernel(const double* __restrict__ w, int64_t p, double* __restrict__ evals) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < p) evals[j] = w[p - 1 - j];
}

// out[0] = #{j : evals[j] > p 2^-52 evals[0]}
__global__ void rank_kernel(const double* __restrict__ evals, int64_t p, long long* __restrict__ out) {
  const double thr = (double)p * 0x1p-52 * evals[0];
  long long cnt = 0;
  for (int64_t j = threadIdx.x; j < p; j += blockDim.x) cnt += evals[j] > thr ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  __shared__ long long part[16];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (unsigned q = 0; q < blockDim.x / 64; ++q) s += part[q];
    out[0] = s;
  }
}

}  // namespace gmgm_eh

using namespace gmgm_eh;

extern "C" gmgm_status gmgm_eigh_small(gmgm_ctx_t c, int64_t p, const float* G, double* evals,
                                       double* evecs, int64_t* rank_out) {
  GMGM_CHECK_CTX(c);
  if (p < 1 || p > 46340) return set_err(c, GMGM_E_SHAPE, "p must be in [1, 46340] (got %lld)", (long long)p);
  if (!G || !evals) return set_err(c, GMGM_E_ARG, "null pointer argument");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  void* hv;
  GMGM_TRY(blas_handle(c, &hv));
  rocblas_handle h = (rocblas_handle)hv;
  void *wA, *wS;
  GMGM_TRY(ws_get(c, WS_EIGH0, (size_t)p * p * sizeof(double), &wA));
  GMGM_TRY(ws_get(c, WS_EIGH1, (size_t)p * 2 * sizeof(double) + 256, &wS));
  double* A = (double*)wA;
  double* w = (double*)wS;
  double* e = w + p;
  int* info = (int*)(e + p);
  long long* rk = (long long*)(info + 2);
  const int64_t n_el = p * p;
  hipLaunchKernelGGL(promote_kernel, dim3((unsigned)std::min<int64_t>(65536, (n_el + 255) / 256)), dim3(256), 0,
                     st, G, n_el, A, c->dev_status);
  // non-finite input would make the eigensolver's result meaningless: stop here
  GMGM_TRY(gmgm_sync(c));
  hipEvent_t ev = timing_start(c);
  // eigenvalues only when no eigenvector output is given
  const rocblas_status rs = rocsolver_dsyevd(h, evecs ? rocblas_evect_original : rocblas_evect_none,
                                             rocblas_fill_lower, (rocblas_int)p, A, (rocblas_int)p, w, e, info);
  timing_stop(c, ev);
  if (rs != rocblas_status_success)
    return set_err(c, GMGM_E_HIP, "rocsolver_dsyevd failed with status %d", (int)rs);
  if (evecs)
    hipLaunchKernelGGL(reorder_kernel, dim3((unsigned)std::min<int64_t>(64, (p + 255) / 256), (unsigned)p),
                       dim3(256), 0, st, A, w, p, evals, evecs);
  else
    hipLaunchKernelGGL(reorder_values_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, w, p, evals);
  hipLaunchKernelGGL(rank_kernel, dim3(1), dim3(1024), 0, st, evals, p, rk);
  int hinfo = 0;
  long long hrank = 0;
  GMGM_HIP(c, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipMemcpyAsync(&hrank, rk, sizeof(long long), hipMemcpyDeviceToHost, st));
  GMGM_HIP(c, hipStreamSynchronize(st));
  if (hinfo != 0) return set_err(c, GMGM_E_NOCONV, "rocsolver_dsyevd: %d off-diagonal elements did not converge", hinfo);
  if (rank_out) *rank_out = hrank;
  return GMGM_OK;
}
