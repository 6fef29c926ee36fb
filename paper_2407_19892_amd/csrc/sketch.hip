// Cell-axis factor from the gene-axis eigenpairs: the top-r left singular
// vectors of X (Algorithm 1, first loop) through the exact identity
//   U = X V_g[:, :r] diag(e[:r])^(-1/2)
// (X = U S V^T with S^2 = e), so the n x n cell-axis Gram is never formed.
//
// A prep kernel folds the scale into an FP32 copy of the r leading
// eigenvectors (p x rs, row-major, rs = W ceil(r / W), zero padded), then one wave per CSR row
// gathers the rows of that panel named by the row's column indices and
// accumulates in FP64: lane l < rs / W owns output columns [W l, W l + W).  The
// column/value pairs of a row are read once, 64 at a time, and broadcast
// across the wave with lane reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "gmgm_internal.h"

namespace gmgm_sk {

// Bp[g][j] = V[g + j ldv] / sqrt(e[j]) for j < r, 0 for r <= j < rpad.
__global__ void panel_kernel(const double* __restrict__ V, int64_t ldv, const double* __restrict__ e,
                             int64_t p, int r, int rpad, float* __restrict__ Bp, int* __restrict__ status) {
  const int64_t total = p * rpad;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = q / rpad;
    const int j = (int)(q % rpad);
    float out = 0.0f;
    if (j < r) {
      const double ej = e[j], v = V[g + (size_t)j * ldv];
      if (!(ej > 0.0) || !isfinite(ej) || !isfinite(v)) atomicCAS(status, 0, DEV_NONFINITE);
      out = (float)(v / sqrt(ej));
    }
    Bp[q] = out;
  }
}

template <int W>
struct Vec;
template <>
struct Vec<1> {
  using T = float;
  static __device__ void add(double* a, T b, double v) { a[0] += v * (double)b; }
};
template <>
struct Vec<2> {
  using T = float2;
  static __device__ void add(double* a, T b, double v) {
    a[0] += v * (double)b.x;
    a[1] += v * (double)b.y;
  }
};
template <>
struct Vec<4> {
  using T = float4;
  static __device__ void add(double* a, T b, double v) {
    a[0] += v * (double)b.x;
    a[1] += v * (double)b.y;
    a[2] += v * (double)b.z;
    a[3] += v * (double)b.w;
  }
};

template <int W>
__global__ void __launch_bounds__(256) spmm_kernel(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const float* __restrict__ val, int64_t nnz, int64_t n, int64_t p,
                                                   const float* __restrict__ Bp, int r, float* __restrict__ U,
                                                   const double* __restrict__ wsh, int* __restrict__ status) {
  using T = typename Vec<W>::T;
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  double acc[W];   // starts at the shift row (the rank-one part of X + 1 z^T) when given
#pragma unroll
  for (int q = 0; q < W; ++q) acc[q] = (wsh && lane * W + q < r) ? wsh[lane * W + q] : 0.0;
  bool badc = false, badv = false;
  if (b < 0 || e < b || e > nnz) {
    if (lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
  } else {
    const int vl = (r + W - 1) / W;                 // vectors per panel row
    const bool act = lane < vl;
    const T* Bl = reinterpret_cast<const T*>(Bp) + (act ? lane : 0);
    for (int64_t t0 = b; t0 < e; t0 += 64) {
      const int64_t t = t0 + lane;
      int cc = 0;
      float vv = 0.0f;
      if (t < e) {
        cc = col[t];
        vv = val ? val[t] : 1.0f;
        badv |= !isfinite(vv);
        if (cc < 0 || cc >= p) {
          badc = true;
          cc = 0;
          vv = 0.0f;
        }
      }
      const int m = e - t0 < 64 ? (int)(e - t0) : 64;
      const int m8 = (m + 7) & ~7;
      for (int j = 0; j < m8; j += 8) {
        T bv[8];
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = __builtin_amdgcn_readlane(cc, j + u);
          v[u] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vv), j + u));
          bv[u] = Bl[(size_t)c * vl];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) Vec<W>::add(acc, bv[u], (double)v[u]);
      }
    }
  }
  if (__ballot(badc) && lane == 0) atomicCAS(status, 0, DEV_BADINDEX);
  if (__ballot(badv) && lane == 0) atomicCAS(status, 0, DEV_NONFINITE);
  float* out = U + (size_t)i * r;
#pragma unroll
  for (int q = 0; q < W; ++q) {
    const int jc = lane * W + q;
    if (jc < r) out[jc] = (float)acc[q];
  }
}

// w = z^T Bp (r entries, FP64): the cell-factor row every cell gets from the
// rank-one part 1 z^T of X + 1 z^T.  One thread per output column.
__global__ void shift_row_kernel(const float* __restrict__ Bp, int64_t p, int rpad, int r,
                                 const double* __restrict__ z, double* __restrict__ w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= r) return;
  double s = 0.0;
  for (int64_t g = 0; g < p; ++g) s += z[g] * (double)Bp[g * rpad + j];
  w[j] = s;
}

}  // namespace gmgm_sk

using namespace gmgm_sk;

static gmgm_status sketch_impl(gmgm_ctx* c, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col, const float* val, const double* evecs, int64_t ldv,
                               const double* evals, int64_t r, const double* z, float* U) {
  if (n < 1 || p < 1 || nnz < 0 || r < 1 || r > 256 || r > p || ldv < p)
    return set_err(c, GMGM_E_SHAPE, "need n >= 1, p >= 1, nnz >= 0, 1 <= r <= min(p, 256), ldv >= p");
  if (!row_ptr || !evecs || !evals || !U || (nnz > 0 && !col)) return set_err(c, GMGM_E_ARG, "null pointer argument");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const int W = r <= 64 ? 1 : r <= 128 ? 2 : 4;
  const int rpad = (int)((r + W - 1) / W * W);
  void* wB;
  GMGM_TRY(ws_get(c, WS_SKETCH, (size_t)p * rpad * sizeof(float), &wB));
  float* Bp = (float*)wB;
  const int64_t tot = p * rpad;
  hipLaunchKernelGGL(panel_kernel, dim3((unsigned)std::min<int64_t>(65536, (tot + 255) / 256)), dim3(256), 0, st,
                     evecs, ldv, evals, p, (int)r, rpad, Bp, c->dev_status);
  double* wsh = nullptr;
  if (z) {
    void* ww;
    GMGM_TRY(ws_get(c, WS_SKEP0, (size_t)r * sizeof(double) + 64, &ww));
    wsh = (double*)ww;
    hipLaunchKernelGGL(shift_row_kernel, dim3((unsigned)((r + 255) / 256)), dim3(256), 0, st, Bp, p, rpad, (int)r,
                       z, wsh);
  }
  const dim3 grid((unsigned)((n + 3) / 4));
  hipEvent_t ev = timing_start(c);
  if (W == 1)
    hipLaunchKernelGGL(spmm_kernel<1>, grid, dim3(256), 0, st, row_ptr, col, val, nnz, n, p, Bp, (int)r, U,
                       wsh, c->dev_status);
  else if (W == 2)
    hipLaunchKernelGGL(spmm_kernel<2>, grid, dim3(256), 0, st, row_ptr, col, val, nnz, n, p, Bp, (int)r, U,
                       wsh, c->dev_status);
  else
    hipLaunchKernelGGL(spmm_kernel<4>, grid, dim3(256), 0, st, row_ptr, col, val, nnz, n, p, Bp, (int)r, U,
                       wsh, c->dev_status);
  timing_stop(c, ev);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_sketch(gmgm_ctx_t c, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                                   const int32_t* col, const float* val, const double* evecs, int64_t ldv,
                                   const double* evals, int64_t r, float* U) {
  GMGM_CHECK_CTX(c);
  return sketch_impl(c, n, p, nnz, row_ptr, col, val, evecs, ldv, evals, r, nullptr, U);
}

extern "C" gmgm_status gmgm_sketch_shifted(gmgm_ctx_t c, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                                           const int32_t* col, const float* val, const double* evecs, int64_t ldv,
                                           const double* evals, int64_t r, const double* z, float* U) {
  GMGM_CHECK_CTX(c);
  if (!z) return set_err(c, GMGM_E_ARG, "null shift pointer");
  return sketch_impl(c, n, p, nnz, row_ptr, col, val, evecs, ldv, evals, r, z, U);
}
