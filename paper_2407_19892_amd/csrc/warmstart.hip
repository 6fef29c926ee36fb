// Learned warm start of the eigenvalue MLE (replaces Algorithm 1's start
// lambda^0 = 1/E; the solver finishes from it).
//
// Features: both axes' log-spectra resampled to 512 bins at the 0-based
// fractional indices t_b = (b + 1/2) r / 512 - 1/2 (clamped, linear
// interpolation), shifted by max(log E_c,0, log E_g,0), then log r_c, log r_g,
// log d_c, log d_g.  Network: 1028 -> 256 -> 256 -> 1024, SiLU after the two
// hidden layers, FP32 parameters W1 b1 W2 b2 W3 b3 (row-major, flat).
// Outputs: two 512-bin curves of log(lambda E); index i of an axis reads the
// curve at u_i = (i + 1/2) 512 / r - 1/2.  Loss: masked mean squared error;
// optimiser: AdamW.  Two precisions of the same network: the gmgm_ws_* calls
// run LDS-tiled FP32 FMA products (the reference mode), the gmgm_warmstart_*
// calls BF16 operands on the matrix cores with FP32 accumulation and FP32
// master weights (every product's two operands are rounded to BF16 as they are
// staged).  Every reduction has a fixed order, so a training step is
// deterministic.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gmgm_internal.h"
#include "mfma_util.h"

namespace gmgm_ws {

constexpr int BINS = 512;
constexpr int D_IN = 2 * BINS + 4;
constexpr int D_H = 256;
constexpr int D_OUT = 2 * BINS;
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + (int64_t)D_H * D_IN;
constexpr int64_t OFF_W2 = OFF_B1 + D_H;
constexpr int64_t OFF_B2 = OFF_W2 + (int64_t)D_H * D_H;
constexpr int64_t OFF_W3 = OFF_B2 + D_H;
constexpr int64_t OFF_B3 = OFF_W3 + (int64_t)D_OUT * D_H;
constexpr int64_t N_PARAMS = OFF_B3 + D_OUT;
constexpr int MAX_BATCH = 8192;

__device__ inline double lerp_at(const double* v, int64_t r, double t, const double* mul) {
  // linear interpolation of log(v_i (* mul_i)) at fractional index t in [0, r - 1]
  const int64_t lo = (int64_t)floor(t);
  const int64_t hi = lo + 1 < r ? lo + 1 : r - 1;
  const double f = t - (double)lo;
  const double a = log(mul ? v[lo] * mul[lo] : v[lo]);
  const double b = log(mul ? v[hi] * mul[hi] : v[hi]);
  return a * (1.0 - f) + b * f;
}

__device__ inline double bin_index(int b, int64_t r) {
  double t = (b + 0.5) * (double)r / BINS - 0.5;
  return fmin(fmax(t, 0.0), (double)(r - 1));
}

// out[0:512] = resampled log E_c - s, out[512:1024] = log E_g - s, then 4 scalars.
// With lam_c / lam_g given: the resampled log(lam E) curves (targets), no shift.
__global__ void __launch_bounds__(512) resample_kernel(const double* __restrict__ Ec, const double* __restrict__ lc,
                                                       int64_t rc, const double* __restrict__ Eg,
                                                       const double* __restrict__ lg, int64_t rg, double dc,
                                                       double dg, int with_scalars, float* __restrict__ out,
                                                       int* __restrict__ status) {
  const int b = threadIdx.x;
  const double s = with_scalars ? fmax(log(Ec[0]), log(Eg[0])) : 0.0;
  const double vc = lerp_at(Ec, rc, bin_index(b, rc), lc) - s;
  const double vg = lerp_at(Eg, rg, bin_index(b, rg), lg) - s;
  if (!isfinite(vc) || !isfinite(vg)) atomicCAS(status, 0, DEV_NONFINITE);
  out[b] = (float)vc;
  out[BINS + b] = (float)vg;
  if (with_scalars && b < 4) {
    const double sc[4] = {log((double)rc), log((double)rg), log(dc), log(dg)};
    out[2 * BINS + b] = (float)sc[b];
  }
}

// lam_i = exp(curve(u_i)) / E_i for both axes (u_i = (i + 1/2) 512 / r - 1/2).
__global__ void apply_kernel(const float* __restrict__ curves, const double* __restrict__ E, int64_t r,
                             double* __restrict__ lam) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= r) return;
  double u = (i + 0.5) * BINS / (double)r - 0.5;
  u = fmin(fmax(u, 0.0), (double)(BINS - 1));
  const int lo = (int)floor(u);
  const int hi = lo + 1 < BINS ? lo + 1 : BINS - 1;
  const double f = u - lo;
  const double y = (double)curves[lo] * (1.0 - f) + (double)curves[hi] * f;
  lam[i] = exp(y) / E[i];
}

// C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[n]); op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k],
// op(B)[k][n] = TB ? B[n ldb + k] : B[k ldb + n].  64 x 64 tile, 16 x 16 threads of 4 x 4.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb,
                                                   const float* __restrict__ bias, float* __restrict__ C, int ldc) {
  __shared__ float As[16][68], Bs[16][68];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = tid + 256 * u;            // 0..1023 over a 64 x 16 (A) and 16 x 64 (B) tile
      int mm, kk, nn, kb;
      if (TA) { kk = q >> 6; mm = q & 63; } else { mm = q >> 4; kk = q & 15; }
      if (TB) { nn = q >> 4; kb = q & 15; } else { kb = q >> 6; nn = q & 63; }
      const int gm = m0 + mm, gk = k0 + kk, gn = n0 + nn, gkb = k0 + kb;
      float av = 0.f, bv = 0.f;
      if (gm < M && gk < K) av = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      if (gn < N && gkb < K) bv = TB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn];
      As[kk][mm] = av;
      Bs[kb][nn] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gm = m0 + ty * 4 + i, gn = n0 + tx * 4 + j;
      if (gm < M && gn < N) C[(size_t)gm * ldc + gn] = acc[i][j] + (bias ? bias[gn] : 0.f);
    }
}

// The same product with BF16 operands on the matrix cores: op(A) and op(B)
// are rounded to BF16 (nearest even) as they are staged into LDS, products
// accumulate in FP32 (V_MFMA_F32_32X32X16_BF16), the bias is added in FP32.
// 64 x 64 output tile per workgroup, 4 waves of 32 x 32; the contraction in
// steps of 32 (two MFMAs).  LDS rows hold 32 k (+ 8 of padding) of one m or
// n, so that each lane reads its 8 consecutive k as one 16-byte load.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                        const float* __restrict__ B, int ldb,
                                                        const float* __restrict__ bias, float* __restrict__ C,
                                                        int ldc) {
  constexpr int KT = 32, LDK = KT + 8;
  __shared__ __align__(16) uint16_t As[64][LDK], Bs[64][LDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  v16f acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  for (int k0 = 0; k0 < K; k0 += KT) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = tid + 256 * u;              // 0..2047 over a 64 x 32 tile of each operand
      int mm, kk;
      if (TA) { kk = q >> 6; mm = q & 63; } else { mm = q >> 5; kk = q & 31; }
      int nn, kb;
      if (TB) { nn = q >> 5; kb = q & 31; } else { kb = q >> 6; nn = q & 63; }
      const int gm = m0 + mm, gk = k0 + kk, gn = n0 + nn, gkb = k0 + kb;
      float av = 0.f, bv = 0.f;
      if (gm < M && gk < K) av = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      if (gn < N && gkb < K) bv = TB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn];
      As[mm][kk] = f32_to_bf16_bits(av);
      Bs[nn][kb] = f32_to_bf16_bits(bv);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KT / 16; ++s) {
      const int kq = 16 * s + 8 * (lane >> 5);
      const v8bf a = __builtin_bit_cast(v8bf, *(const uint4*)&As[32 * wm + (lane & 31)][kq]);
      const v8bf b = __builtin_bit_cast(v8bf, *(const uint4*)&Bs[32 * wn + (lane & 31)][kq]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int gm = m0 + 32 * wm + acc_row(v, lane >> 5);
    const int gn = n0 + 32 * wn + (lane & 31);
    if (gm < M && gn < N) C[(size_t)gm * ldc + gn] = acc[v] + (bias ? bias[gn] : 0.f);
  }
}

__device__ inline float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

__global__ void silu_kernel(const float* __restrict__ Z, float* __restrict__ H, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) H[i] = Z[i] * sigm(Z[i]);
}

// dZ = dH * silu'(Z)
__global__ void silu_back_kernel(const float* __restrict__ dH, const float* __restrict__ Z, float* __restrict__ dZ,
                                 int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = sigm(Z[i]);
  dZ[i] = dH[i] * (s * (1.0f + Z[i] * (1.0f - s)));
}

// scal[0] = sum M, scal[1] = sum M (Y - T)^2 (one workgroup, fixed order, FP64)
__global__ void __launch_bounds__(1024) loss_sums_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                         const float* __restrict__ Mk, int64_t n,
                                                         double* __restrict__ scal) {
  __shared__ double r0[16], r1[16];
  double sm = 0, se = 0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double m = Mk ? (double)Mk[i] : 1.0;
    const double d = (double)Y[i] - (double)T[i];
    sm += m;
    se += m * d * d;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sm += __shfl_xor(sm, o, 64);
    se += __shfl_xor(se, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = sm;
    r1[threadIdx.x >> 6] = se;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int w = 0; w < 16; ++w) {
      a += r0[w];
      b += r1[w];
    }
    scal[0] = a;
    scal[1] = b;
    scal[2] = a > 0 ? b / a : 0.0;
  }
}

// dY = 2 M (Y - T) / sum M
__global__ void loss_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ Mk,
                                 int64_t n, const double* __restrict__ scal, float* __restrict__ dY) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double msum = scal[0];
  const double m = Mk ? (double)Mk[i] : 1.0;
  dY[i] = msum > 0 ? (float)(2.0 * m * ((double)Y[i] - (double)T[i]) / msum) : 0.0f;
}

// g[n] = sum_b dZ[b][n] (one thread per column, rows in order)
__global__ void colsum_kernel(const float* __restrict__ dZ, int rows, int N, float* __restrict__ g) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int b = 0; b < rows; ++b) s += dZ[(size_t)b * N + n];
  g[n] = s;
}

// One AdamW update.  The bias corrections 1 - 0.9^t and 1 - 0.999^t and the
// weight decay come from the host (bc1, bc2, wd), or, when bcp is given, from
// bcp[0..2] (written on the device by adam_count_kernel).
__global__ void adamw_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                             const float* __restrict__ g, int64_t n, float lr, float wd, float bc1, float bc2,
                             const float* __restrict__ bcp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (bcp) {
    bc1 = bcp[0];
    bc2 = bcp[1];
    wd = bcp[2];
  }
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  p[i] -= lr * (mh / (sqrtf(vh) + 1e-8f) + wd * p[i]);
}

// Optimiser state of gmgm_warmstart_train_step: a header (update count, weight
// decay) and the two moment vectors.
struct OptHeader {
  int64_t step;
  float weight_decay;
};
constexpr int64_t OPT_M = 256;                                   // byte offset of m
constexpr int64_t OPT_V = OPT_M + N_PARAMS * (int64_t)sizeof(float);
constexpr int64_t OPT_BYTES = OPT_V + N_PARAMS * (int64_t)sizeof(float);

// t = ++step; bc = {1 - 0.9^t, 1 - 0.999^t, weight decay} (FP64 powers, rounded once).
__global__ void adam_count_kernel(OptHeader* __restrict__ h, float* __restrict__ bc) {
  const int64_t t = ++h->step;
  bc[0] = (float)(1.0 - pow(0.9, (double)t));
  bc[1] = (float)(1.0 - pow(0.999, (double)t));
  bc[2] = h->weight_decay;
}

__global__ void opt_init_kernel(char* __restrict__ state, float wd) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) {
    OptHeader* h = (OptHeader*)state;
    h->step = 0;
    h->weight_decay = wd;
  }
  if (i < 2 * N_PARAMS) ((float*)(state + OPT_M))[i] = 0.0f;
}

// Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias of a layer,
// from a SplitMix64 hash of (seed, index).
__device__ inline double hash_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}
__global__ void init_kernel(float* __restrict__ p, uint64_t seed) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N_PARAMS) return;
  const int fan_in = i < OFF_W2 ? D_IN : D_H;
  const double bound = 1.0 / sqrt((double)fan_in);
  p[i] = (float)((2.0 * hash_uniform(seed, (uint64_t)i) - 1.0) * bound);
}

inline unsigned nb(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// bf16 selects the matrix-core product with BF16 operands (the network's
// BF16-weight mode); otherwise FP32 FMA tiles.
template <bool TA, bool TB>
void gemm(hipStream_t st, bool bf16, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
          const float* bias, float* C, int ldc) {
  if (bf16)
    hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB>), dim3(nb(N, 64), nb(M, 64)), dim3(256), 0, st, M, N, K, A, lda,
                       B, ldb, bias, C, ldc);
  else
    hipLaunchKernelGGL((gemm_kernel<TA, TB>), dim3(nb(N, 64), nb(M, 64)), dim3(256), 0, st, M, N, K, A, lda, B,
                       ldb, bias, C, ldc);
}

struct Acts {
  float *Z1, *H1, *Z2, *H2, *Y;
};

gmgm_status acts(gmgm_ctx* c, int batch, Acts* a, float** extra, int64_t extra_floats) {
  void* w;
  const int64_t need = (int64_t)batch * (4 * D_H + D_OUT) + extra_floats;
  GMGM_TRY(ws_get(c, WS_MLP0, (size_t)need * sizeof(float) + 256, &w));
  float* f = (float*)w;
  a->Z1 = f;
  a->H1 = f + (int64_t)batch * D_H;
  a->Z2 = f + (int64_t)batch * 2 * D_H;
  a->H2 = f + (int64_t)batch * 3 * D_H;
  a->Y = f + (int64_t)batch * 4 * D_H;
  *extra = f + (int64_t)batch * (4 * D_H + D_OUT);
  return GMGM_OK;
}

void forward(hipStream_t st, bool bf, const float* P, int B, const float* X, const Acts& a, float* Y) {
  gemm<false, true>(st, bf, B, D_H, D_IN, X, D_IN, P + OFF_W1, D_IN, P + OFF_B1, a.Z1, D_H);
  hipLaunchKernelGGL(silu_kernel, dim3(nb((int64_t)B * D_H)), dim3(256), 0, st, a.Z1, a.H1, (int64_t)B * D_H);
  gemm<false, true>(st, bf, B, D_H, D_H, a.H1, D_H, P + OFF_W2, D_H, P + OFF_B2, a.Z2, D_H);
  hipLaunchKernelGGL(silu_kernel, dim3(nb((int64_t)B * D_H)), dim3(256), 0, st, a.Z2, a.H2, (int64_t)B * D_H);
  gemm<false, true>(st, bf, B, D_OUT, D_H, a.H2, D_H, P + OFF_W3, D_H, P + OFF_B3, Y, D_OUT);
}

}  // namespace gmgm_ws

using namespace gmgm_ws;

extern "C" int64_t gmgm_ws_param_count(void) { return N_PARAMS; }

extern "C" gmgm_status gmgm_ws_init(gmgm_ctx_t c, float* params, uint64_t seed) {
  GMGM_CHECK_CTX(c);
  if (!params) return set_err(c, GMGM_E_ARG, "null pointer argument");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipLaunchKernelGGL(init_kernel, dim3(nb(N_PARAMS)), dim3(256), 0, c->stream, params, seed);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_ws_features(gmgm_ctx_t c, const double* Ec, int64_t rc, const double* Eg, int64_t rg,
                                        double dc, double dg, float* feat) {
  GMGM_CHECK_CTX(c);
  if (!Ec || !Eg || !feat) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (rc < 1 || rg < 1 || !(dc >= 1) || !(dg >= 1) || !std::isfinite(dc) || !std::isfinite(dg))
    return set_err(c, GMGM_E_SHAPE, "need ranks >= 1 and dimensions >= 1");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipLaunchKernelGGL(resample_kernel, dim3(1), dim3(BINS), 0, c->stream, Ec, (const double*)nullptr, rc, Eg,
                     (const double*)nullptr, rg, dc, dg, 1, feat, c->dev_status);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_ws_targets(gmgm_ctx_t c, const double* Ec, const double* lam_c, int64_t rc,
                                       const double* Eg, const double* lam_g, int64_t rg, float* target) {
  GMGM_CHECK_CTX(c);
  if (!Ec || !Eg || !lam_c || !lam_g || !target) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (rc < 1 || rg < 1) return set_err(c, GMGM_E_SHAPE, "need ranks >= 1");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipLaunchKernelGGL(resample_kernel, dim3(1), dim3(BINS), 0, c->stream, Ec, lam_c, rc, Eg, lam_g, rg, 1.0, 1.0, 0,
                     target, c->dev_status);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_ws_forward(gmgm_ctx_t c, const float* params, int32_t batch, const float* feats,
                                       float* out) {
  GMGM_CHECK_CTX(c);
  if (!params || !feats || !out) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (batch < 1 || batch > MAX_BATCH) return set_err(c, GMGM_E_SHAPE, "batch must be in [1, %d]", MAX_BATCH);
  GMGM_HIP(c, hipSetDevice(c->device));
  Acts a;
  float* extra;
  GMGM_TRY(acts(c, batch, &a, &extra, 0));
  forward(c->stream, false, params, batch, feats, a, out);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

namespace gmgm_ws {
// One training step: forward, masked MSE, backward, AdamW.  The update count
// and weight decay come from the host (step >= 1, weight_decay) or, with
// `state`, from the device header (incremented there).
static gmgm_status train_impl(gmgm_ctx* c, bool bf, float* params, float* adam_m, float* adam_v, int64_t step,
                              float weight_decay, OptHeader* state, int32_t batch, const float* feats,
                              const float* target, const float* mask, float lr, double* loss_out,
                              float* grad_out) {
  hipStream_t st = c->stream;
  const int B = batch;
  Acts a;
  float* ex;
  const int64_t nY = (int64_t)B * D_OUT, nH = (int64_t)B * D_H;
  GMGM_TRY(acts(c, B, &a, &ex, nY + 2 * nH + N_PARAMS));
  float *dY = ex, *dH = ex + nY, *dZ = dH + nH, *g = dZ + nH;
  void* ws;
  GMGM_TRY(ws_get(c, WS_MLP1, 64, &ws));
  double* scal = (double*)ws;
  float* bcp = (float*)((char*)ws + 32);

  forward(st, bf, params, B, feats, a, a.Y);
  hipLaunchKernelGGL(loss_sums_kernel, dim3(1), dim3(1024), 0, st, a.Y, target, mask, nY, scal);
  hipLaunchKernelGGL(loss_grad_kernel, dim3(nb(nY)), dim3(256), 0, st, a.Y, target, mask, nY, scal, dY);
  // layer 3
  gemm<true, false>(st, bf, D_OUT, D_H, B, dY, D_OUT, a.H2, D_H, nullptr, g + OFF_W3, D_H);
  hipLaunchKernelGGL(colsum_kernel, dim3(nb(D_OUT)), dim3(256), 0, st, dY, B, D_OUT, g + OFF_B3);
  gemm<false, false>(st, bf, B, D_H, D_OUT, dY, D_OUT, params + OFF_W3, D_H, nullptr, dH, D_H);
  hipLaunchKernelGGL(silu_back_kernel, dim3(nb(nH)), dim3(256), 0, st, dH, a.Z2, dZ, nH);
  // layer 2
  gemm<true, false>(st, bf, D_H, D_H, B, dZ, D_H, a.H1, D_H, nullptr, g + OFF_W2, D_H);
  hipLaunchKernelGGL(colsum_kernel, dim3(nb(D_H)), dim3(256), 0, st, dZ, B, D_H, g + OFF_B2);
  gemm<false, false>(st, bf, B, D_H, D_H, dZ, D_H, params + OFF_W2, D_H, nullptr, dH, D_H);
  hipLaunchKernelGGL(silu_back_kernel, dim3(nb(nH)), dim3(256), 0, st, dH, a.Z1, dZ, nH);
  // layer 1
  gemm<true, false>(st, bf, D_H, D_IN, B, dZ, D_H, feats, D_IN, nullptr, g + OFF_W1, D_IN);
  hipLaunchKernelGGL(colsum_kernel, dim3(nb(D_H)), dim3(256), 0, st, dZ, B, D_H, g + OFF_B1);
  if (grad_out)
    GMGM_HIP(c, hipMemcpyAsync(grad_out, g, N_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, st));
  float bc1 = 1.0f, bc2 = 1.0f;
  if (state) {
    hipLaunchKernelGGL(adam_count_kernel, dim3(1), dim3(1), 0, st, state, bcp);
  } else {
    bc1 = (float)(1.0 - std::pow(0.9, (double)step));
    bc2 = (float)(1.0 - std::pow(0.999, (double)step));
  }
  hipLaunchKernelGGL(adamw_kernel, dim3(nb(N_PARAMS)), dim3(256), 0, st, params, adam_m, adam_v, g, N_PARAMS, lr,
                     weight_decay, bc1, bc2, state ? (const float*)bcp : (const float*)nullptr);
  if (loss_out) {
    GMGM_HIP(c, hipMemcpyAsync(loss_out, scal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    GMGM_HIP(c, hipStreamSynchronize(st));
  }
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}
}  // namespace gmgm_ws

extern "C" gmgm_status gmgm_ws_train_step(gmgm_ctx_t c, float* params, float* adam_m, float* adam_v, int64_t step,
                                          int32_t batch, const float* feats, const float* target, const float* mask,
                                          float lr, float weight_decay, double* loss_out, float* grad_out) {
  GMGM_CHECK_CTX(c);
  if (!params || !adam_m || !adam_v || !feats || !target) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (batch < 1 || batch > MAX_BATCH) return set_err(c, GMGM_E_SHAPE, "batch must be in [1, %d]", MAX_BATCH);
  if (step < 1 || !(lr >= 0) || !(weight_decay >= 0))
    return set_err(c, GMGM_E_ARG, "need step >= 1, lr >= 0, weight_decay >= 0");
  GMGM_HIP(c, hipSetDevice(c->device));
  return train_impl(c, false, params, adam_m, adam_v, step, weight_decay, nullptr, batch, feats, target, mask, lr,
                    loss_out, grad_out);
}

extern "C" int64_t gmgm_warmstart_state_bytes(void) { return OPT_BYTES; }

extern "C" gmgm_status gmgm_warmstart_state_init(gmgm_ctx_t c, void* opt_state, float weight_decay) {
  GMGM_CHECK_CTX(c);
  if (!opt_state) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (!(weight_decay >= 0) || !std::isfinite(weight_decay))
    return set_err(c, GMGM_E_ARG, "weight_decay must be finite and >= 0");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipLaunchKernelGGL(opt_init_kernel, dim3(nb(2 * N_PARAMS)), dim3(256), 0, c->stream, (char*)opt_state,
                     weight_decay);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_warmstart_infer(gmgm_ctx_t c, const void* weights, int32_t batch, const float* feats,
                                            float* out) {
  GMGM_CHECK_CTX(c);
  if (!weights || !feats || !out) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (batch < 1 || batch > MAX_BATCH) return set_err(c, GMGM_E_SHAPE, "batch must be in [1, %d]", MAX_BATCH);
  GMGM_HIP(c, hipSetDevice(c->device));
  Acts a;
  float* extra;
  GMGM_TRY(acts(c, batch, &a, &extra, 0));
  forward(c->stream, true, (const float*)weights, batch, feats, a, out);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_warmstart_train_step(gmgm_ctx_t c, void* weights, void* opt_state, int32_t batch,
                                                 const float* feats, const float* target, const float* mask,
                                                 float lr, float* loss_out) {
  GMGM_CHECK_CTX(c);
  if (!weights || !opt_state || !feats || !target) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (batch < 1 || batch > MAX_BATCH) return set_err(c, GMGM_E_SHAPE, "batch must be in [1, %d]", MAX_BATCH);
  if (!(lr >= 0) || !std::isfinite(lr)) return set_err(c, GMGM_E_ARG, "lr must be finite and >= 0");
  GMGM_HIP(c, hipSetDevice(c->device));
  char* stt = (char*)opt_state;
  double loss = 0.0;
  GMGM_TRY(train_impl(c, true, (float*)weights, (float*)(stt + OPT_M), (float*)(stt + OPT_V), 0, 0.0f,
                      (OptHeader*)stt, batch, feats, target, mask, lr, loss_out ? &loss : nullptr, nullptr));
  if (loss_out) *loss_out = (float)loss;
  return GMGM_OK;
}

extern "C" gmgm_status gmgm_ws_apply(gmgm_ctx_t c, const float* curves, const double* Ec, int64_t rc,
                                     const double* Eg, int64_t rg, double* lam_c, double* lam_g) {
  GMGM_CHECK_CTX(c);
  if (!curves || !Ec || !Eg || !lam_c || !lam_g) return set_err(c, GMGM_E_ARG, "null pointer argument");
  if (rc < 1 || rg < 1) return set_err(c, GMGM_E_SHAPE, "need ranks >= 1");
  GMGM_HIP(c, hipSetDevice(c->device));
  hipLaunchKernelGGL(apply_kernel, dim3(nb(rc)), dim3(256), 0, c->stream, curves, Ec, rc, lam_c);
  hipLaunchKernelGGL(apply_kernel, dim3(nb(rg)), dim3(256), 0, c->stream, curves + BINS, Eg, rg, lam_g);
  GMGM_HIP(c, hipGetLastError());
  return GMGM_OK;
}
