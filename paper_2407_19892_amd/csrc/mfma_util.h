// MFMA fragments, number formats and wave helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

// Operand precisions of the recomposition sweep.  P_BF16X3 carries each FP32
// operand as a BF16 pair x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) and
// forms hi*hi + hi*lo + lo*hi with three BF16 MFMAs per K step (internal: the
// re-sweep of rows a BF16 / FP8 sweep could not certify).
enum : int { P_F32 = 0, P_BF16 = 1, P_FP8 = 2, P_BF16X3 = 3 };

// Elements of one row held in one 16-byte operand chunk.
__host__ __device__ constexpr int chunk_elems(int prec) { return prec == P_F32 ? 4 : prec == P_FP8 ? 16 : 8; }
// Padded contraction length: a multiple of the K of 4 f32 MFMAs (8), one bf16 MFMA (16)
// or one f8f6f4 MFMA (64).
__host__ __device__ constexpr int k_align(int prec) { return prec == P_F32 ? 8 : prec == P_FP8 ? 64 : 16; }
// 16-byte chunks per lane per 32-row tile: two lanes share a row; the split
// BF16 form holds the high parts in units [0, kpad/16) and the low parts of
// the same k in units [kpad/16, kpad/8).
__host__ __device__ constexpr int units_for(int prec, int kpad) {
  return prec == P_BF16X3 ? kpad / 8 : kpad / chunk_elems(prec) / 2;
}

// 32x32 MFMA accumulator layout: lane l, register v holds
//   row  = 8 * (v / 4) + 4 * (l / 32) + (v % 4),   col = l % 32
// of the 32x32 result (rows come from the A operand, columns from B).
__host__ __device__ constexpr int acc_row(int v, int half) { return 8 * (v / 4) + 4 * half + (v % 4); }

// Operand chunk u of a lane (16 bytes) holds, for row (l % 32) of a 32-row tile, the
// contiguous k range [k0, k0 + chunk_elems) with
//   f32 : u = group g (4 MFMAs of K=2): k0 = 8 g + 4 half        (MFMA 4g+q uses element q)
//   bf16: u = MFMA s (K=16):            k0 = 16 s + 8 half
//         (split form: unit s + kpad/16 holds the low parts of unit s)
//   fp8 : u = 2 s + c, MFMA s (K=64):   k0 = 64 s + 32 half + 16 c
// A and B operands use the same mapping, so each MFMA pairs equal k on both sides.
__host__ __device__ constexpr int chunk_k0(int prec, int u, int half) {
  return prec == P_F32 ? 8 * u + 4 * half
       : prec != P_FP8 ? 16 * u + 8 * half
                        : 64 * (u / 2) + 32 * half + 16 * (u % 2);
}

// ---- number formats (round to nearest even; inputs are finite)
__host__ __device__ inline uint16_t f32_to_bf16_bits(float x) {
  uint32_t b;
  __builtin_memcpy(&b, &x, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// OCP FP8 e4m3 (bias 7, max 448, no infinities); |x| must be <= 448.
__host__ __device__ inline uint8_t f32_to_e4m3_bits(float x) {
  uint32_t b;
  __builtin_memcpy(&b, &x, 4);
  const uint8_t sign = (uint8_t)((b >> 24) & 0x80u);
  float a = x < 0 ? -x : x;
  if (a < 0.015625f) {                      // below 2^-6: subnormal grid m * 2^-9
    float m = a * 512.0f;                   // exact
    int mi = (int)__builtin_rintf(m);       // ties to even
    return (uint8_t)(sign | mi);            // mi == 8 encodes 2^-6 correctly
  }
  int e = (int)((b >> 23) & 0xFFu) - 127;   // -6 .. 8
  uint32_t man = b & 0x7FFFFFu;
  uint32_t r = man >> 20, rem = man & 0xFFFFFu;
  if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) r++;
  if (r == 8u) { r = 0; e++; }
  if (e > 8 || (e == 8 && r > 6u)) { e = 8; r = 6; }   // saturate at 448
  return (uint8_t)(sign | (uint8_t)((e + 7) << 3) | (uint8_t)r);
}

__host__ __device__ inline float e4m3_bits_to_f32(uint8_t v) {
  int s = v >> 7, e = (v >> 3) & 15, m = v & 7;
  float a = e == 0 ? (float)m * (1.0f / 512.0f) : (1.0f + m / 8.0f) * __builtin_ldexpf(1.0f, e - 7);
  return s ? -a : a;
}

// ---- wave helpers
__device__ inline float wave_max_f32(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int wave_sum_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
