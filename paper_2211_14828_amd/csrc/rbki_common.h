// Shared device/host definitions of the rBKI-TK library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/rbkitk.h"

namespace rbki {

// Element storage types the kernels read.
enum Elem : int { E_F64 = 0, E_F32 = 1, E_BF16 = 2, E_FP8 = 3 };

typedef unsigned short bf16_t;   // bfloat16 bit pattern
typedef unsigned char fp8_t;     // OCP e4m3 bit pattern

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(16))) float f32x16_t;
typedef __attribute__((ext_vector_type(2))) float f32x2_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;
typedef __attribute__((ext_vector_type(4))) double f64x4_t;
typedef __attribute__((ext_vector_type(8))) int i32x8_t;

// ---------------------------------------------------------------- bfloat16
// Round-to-nearest-even float -> bfloat16 (NaN kept quiet).
__host__ __device__ inline bf16_t f32_to_bf16(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  uint32_t u = v.u;
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (bf16_t)((u >> 16) | 0x0040u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  union { float f; uint32_t u; } v;
  v.u = ((uint32_t)h) << 16;
  return v.f;
}

// ---------------------------------------------------------------- fp8 e4m3
// OCP e4m3 ("fn"): bias 7, no infinities, max finite 448, NaN = S.1111.111.
// Round-to-nearest-even with saturation to +-448.
__host__ __device__ inline fp8_t f32_to_e4m3(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  uint32_t sign = (v.u >> 24) & 0x80u;
  float a = fabsf(f);
  if (!(a == a)) return (fp8_t)(sign | 0x7Fu);
  if (a >= 448.0f) return (fp8_t)(sign | 0x7Eu);
  // smallest normal 2^-6; subnormal quantum 2^-9
  if (a < 0.015625f) {
    float q = a * 512.0f;                       // in units of 2^-9
    float r = rintf(q);                         // RNE
    return (fp8_t)(sign | (uint32_t)r);         // r <= 8 -> 8 is the min normal 0x08
  }
  union { float f; uint32_t u; } w;
  w.f = a;
  int e = (int)((w.u >> 23) & 0xFF) - 127;      // -6 .. 8
  uint32_t mant = w.u & 0x7FFFFFu;
  // keep 3 mantissa bits, RNE on the 20 dropped bits
  uint32_t keep = mant >> 20;
  uint32_t rest = mant & 0xFFFFFu;
  if (rest > 0x80000u || (rest == 0x80000u && (keep & 1u))) {
    keep += 1;
    if (keep == 8) { keep = 0; e += 1; }
  }
  uint32_t code = ((uint32_t)(e + 7) << 3) | keep;
  if (code > 0x7Eu) code = 0x7Eu;
  return (fp8_t)(sign | code);
}
__host__ __device__ inline float e4m3_to_f32(fp8_t c) {
  uint32_t s = c & 0x80u, e = (c >> 3) & 0xFu, m = c & 7u;
  float v;
  if (e == 0) v = (float)m * 0.001953125f;      // m * 2^-9
  else v = ldexpf(1.0f + (float)m * 0.125f, (int)e - 7);
  return s ? -v : v;
}

// ------------------------------------------------------------ small helpers
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <class T> __device__ inline T warp_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <class T> __device__ inline T warp_max(T v) {
  for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, 64); v = v > w ? v : w; }
  return v;
}

// 1/x and 1/sqrt(x) in float64 from the hardware estimates refined by two
// Newton-Raphson steps each (r <- r (2 - x r); r <- r (3 - x r^2) / 2), full
// double precision from an estimate good to half of it, in a few dependent
// FMAs instead of the correctly rounded divide / square-root sequences.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ inline double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  r = r * fma(-hx * r, r, 1.5);
  r = r * fma(-hx * r, r, 1.5);
  return r;
}

}  // namespace rbki
