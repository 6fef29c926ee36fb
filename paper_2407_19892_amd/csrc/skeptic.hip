// Nonparanormal Skeptic (rank-based Gaussian copula transform) of a sparse
// cells x genes matrix without densifying it ("Preserving input sparsity").
//
// Each gene (column) is transformed marginally: a value x of column g becomes
// Phi^-1(rank(x) / (n + 1)), rank(x) = 1 + #{values of the column below x}
// counting the column's n - m_g implicit zeros (ties share the smallest rank).
// All zeros of a column map to the same value z_g, so the transform is
//   X~ = S + 1 z^T,
// S with X's sparsity pattern (S_ig = f(x_ig) - z_g; zero where x_ig = 0).
// The library then forms the Gram of X~ from S's Gram and column sums (a
// rank-two correction) and the cell factor X~ B from S B plus one row vector,
// so the dense matrix is never built.
//
// Kernels: column counts and a one-workgroup scan give the columns' segments;
// a scatter copies every nonzero (value, source position) into its column
// segment; rocPRIM's segmented radix sort orders each segment by value; one
// workgroup per column then ranks every sorted value by a lower-bound search
// in its segment, writes f(x) - z_g to the value's source position, and forms
// z_g and the column sum of S in FP64.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <algorithm>
#include <cmath>

#include "gmgm_internal.h"
#include "mfma_util.h"

namespace gmgm_sq {

__global__ void count_kernel(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t n, int64_t p,
                             int64_t nnz, unsigned long long* __restrict__ cnt, const float* __restrict__ val,
                             int* __restrict__ status) {
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
    if (val && !isfinite(val[t])) atomicCAS(status, 0, DEV_NONFINITE);
    atomicAdd(&cnt[c], 1ull);
  }
}

// Exclusive scan of cnt (p entries) into seg (p + 1 entries) and cursor; one workgroup.
__global__ void __launch_bounds__(1024) scan_kernel(const unsigned long long* __restrict__ cnt, int64_t p,
                                                    unsigned long long* __restrict__ seg,
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
    seg[p] = run;
  }
  __syncthreads();
  unsigned long long run = part[t];
  for (int64_t j = lo; j < hi; ++j) {
    seg[j] = run;
    cursor[j] = run;
    run += cnt[j];
  }
}

__global__ void scatter_kernel(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const float* __restrict__ val, int64_t n, int64_t p, int64_t nnz,
                               unsigned long long* __restrict__ cursor, float* __restrict__ key,
                               unsigned* __restrict__ src) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  if (b < 0 || e < b || e > nnz) return;
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c = col[t];
    if (c < 0 || c >= p) continue;
    const unsigned long long pos = atomicAdd(&cursor[c], 1ull);
    key[pos] = val ? val[t] : 1.0f;
    src[pos] = (unsigned)t;
  }
}

// Phi^-1(u), 0 < u < 1: the upper-tail quantile by the rational start of
// Abramowitz and Stegun 26.2.23 and Newton steps on 0.5 erfc(z / sqrt 2).
__device__ inline double normal_quantile(double u) {
  if (u == 0.5) return 0.0;
  const double p = u < 0.5 ? u : 1.0 - u;   // tail probability
  const double t = sqrt(-2.0 * log(p));
  double z = t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                     (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t);
  for (int it = 0; it < 6; ++it) {
    const double tail = 0.5 * erfc(z * 0.70710678118654752440);
    const double dens = exp(-0.5 * z * z) * 0.39894228040143267794;
    z += (tail - p) / dens;
  }
  return u < 0.5 ? -z : z;
}

// First position in key[b, e) whose value is not below x (key sorted ascending).
__device__ inline unsigned long long lower_bound(const float* __restrict__ key, unsigned long long b,
                                                 unsigned long long e, float x) {
  while (b < e) {
    const unsigned long long m = b + (e - b) / 2;
    if (key[m] < x) b = m + 1;
    else e = m;
  }
  return b;
}

// One workgroup per column: ranks of the sorted values, f(x) - z_g to each
// value's source position, z_g, and the FP64 column sum of S.
__global__ void __launch_bounds__(256) rank_kernel(const unsigned long long* __restrict__ seg,
                                                   const float* __restrict__ key, const unsigned* __restrict__ src,
                                                   int64_t n, int64_t p, float* __restrict__ val_out,
                                                   double* __restrict__ z_out, double* __restrict__ csum) {
  __shared__ double part[256];
  const int64_t g = blockIdx.x;
  if (g >= p) return;
  const unsigned long long b = seg[g], e = seg[g + 1];
  const long long m = (long long)(e - b);
  const double inv = 1.0 / ((double)n + 1.0);
  // zeros: 1 + the number of negative values
  const double rank0 = 1.0 + (double)(lower_bound(key, b, e, 0.0f) - b);
  const double z = normal_quantile(rank0 * inv);
  double s = 0.0;
  for (unsigned long long q = b + threadIdx.x; q < e; q += 256) {
    const float x = key[q];
    const double below = (double)(lower_bound(key, b, q, x) - b) + (x > 0.0f ? (double)(n - m) : 0.0);
    const double f = (x == 0.0f) ? z : normal_quantile((1.0 + below) * inv);
    const double d = f - z;
    val_out[src[q]] = (float)d;
    s += d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    z_out[g] = z;
    csum[g] = part[0];
  }
}

}  // namespace gmgm_sq

using namespace gmgm_sq;

extern "C" gmgm_status gmgm_skeptic(gmgm_ctx_t c, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                                    const int32_t* col, const float* val, float* val_out, double* z_out,
                                    double* csum_out) {
  GMGM_CHECK_CTX(c);
  if (n < 1 || p < 1 || p > 0x7fffffffLL || nnz < 0 || nnz > 0xffffffffLL)
    return set_err(c, GMGM_E_SHAPE, "need n >= 1, 1 <= p < 2^31, 0 <= nnz < 2^32 (got n=%lld p=%lld nnz=%lld)",
                   (long long)n, (long long)p, (long long)nnz);
  if (!row_ptr || !z_out || !csum_out || (nnz > 0 && (!col || !val_out)))
    return set_err(c, GMGM_E_ARG, "null pointer argument");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const size_t nz = (size_t)std::max<int64_t>(nnz, 1);
  void *wc, *wk;
  GMGM_TRY(ws_get(c, WS_SKEP0, (size_t)p * 16 + (size_t)(p + 1) * 8 + 64, &wc));
  GMGM_TRY(ws_get(c, WS_SKEP1, nz * 16, &wk));
  unsigned long long* cnt = (unsigned long long*)wc;
  unsigned long long* cursor = cnt + p;
  unsigned long long* seg = cursor + p;
  float* key_in = (float*)wk;
  float* key_out = key_in + nz;
  unsigned* src_in = (unsigned*)(key_out + nz);
  unsigned* src_out = src_in + nz;
  GMGM_HIP(c, hipMemsetAsync(cnt, 0, (size_t)p * 8, st));
  const dim3 grid((unsigned)((n + 3) / 4));
  hipLaunchKernelGGL(count_kernel, grid, dim3(256), 0, st, row_ptr, col, n, p, nnz, cnt, val, c->dev_status);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, cnt, p, seg, cursor);
  hipLaunchKernelGGL(scatter_kernel, grid, dim3(256), 0, st, row_ptr, col, val, n, p, nnz, cursor, key_in, src_in);
  GMGM_HIP(c, hipGetLastError());
  // the malformed-CSR and non-finite checks gate the sort (its segments come
  // from the column counts)
  GMGM_TRY(gmgm_sync(c));
  if (nnz > 0) {
    size_t tmp_bytes = 0;
    GMGM_HIP(c, rocprim::segmented_radix_sort_pairs(nullptr, tmp_bytes, key_in, key_out, src_in, src_out,
                                                    (unsigned)nnz, (unsigned)p, seg, seg + 1, 0, 32, st));
    void* tmp;
    GMGM_TRY(ws_get(c, WS_SKEP2, std::max<size_t>(tmp_bytes, 16), &tmp));
    GMGM_HIP(c, rocprim::segmented_radix_sort_pairs(tmp, tmp_bytes, key_in, key_out, src_in, src_out,
                                                    (unsigned)nnz, (unsigned)p, seg, seg + 1, 0, 32, st));
  }
  hipLaunchKernelGGL(rank_kernel, dim3((unsigned)p), dim3(256), 0, st, seg, key_out, src_out, n, p, val_out, z_out,
                     csum_out);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}
