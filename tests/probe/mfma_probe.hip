// Test-only probes: one MFMA with caller-chosen per-lane operands, and host
// wrappers of the library's number-format conversions.
#include <hip/hip_runtime.h>

#include "../../paper_2407_19892_amd/csrc/mfma_util.h"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void probe_kernel(int prec, const unsigned* __restrict__ A, const unsigned* __restrict__ B,
                             float* __restrict__ D) {
  const int l = threadIdx.x;
  v16f acc;
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  if (prec == P_F32) {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(A[l * 8]), __uint_as_float(B[l * 8]), acc,
                                              0, 0, 0);
  } else if (prec == P_BF16) {
    u32x4 a = {A[l * 8], A[l * 8 + 1], A[l * 8 + 2], A[l * 8 + 3]};
    u32x4 b = {B[l * 8], B[l * 8 + 1], B[l * 8 + 2], B[l * 8 + 3]};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b),
                                                 acc, 0, 0, 0);
  } else {
    v8i a, b;
    for (int q = 0; q < 8; ++q) {
      a[q] = (int)A[l * 8 + q];
      b[q] = (int)B[l * 8 + q];
    }
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
  }
  for (int v = 0; v < 16; ++v) D[l * 16 + v] = acc[v];
}

extern "C" int probe_mfma(int prec, const unsigned* A, const unsigned* B, float* D) {
  hipLaunchKernelGGL(probe_kernel, dim3(1), dim3(64), 0, 0, prec, A, B, D);
  return (int)hipDeviceSynchronize();
}

extern "C" unsigned probe_bf16_bits(float x) { return f32_to_bf16_bits(x); }
extern "C" unsigned probe_e4m3_bits(float x) { return f32_to_e4m3_bits(x); }
extern "C" float probe_e4m3_decode(unsigned v) { return e4m3_bits_to_f32((uint8_t)v); }
extern "C" int probe_acc_row(int v, int half) { return acc_row(v, half); }
extern "C" int probe_chunk_k0(int prec, int u, int half) { return chunk_k0(prec, u, half); }
