// Counter-based Gaussian stream for the sketch matrix Omega (Alg. 1, step 1).
//
// Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel
// random numbers: as easy as 1, 2, 3", SC'11): four 32-bit counter words,
// two key words, ten rounds.  One round multiplies c0 by 0xD2511F53 and c2 by
// 0xCD9E8D57 (64-bit products split into hi/lo halves) and maps
//   (c0, c1, c2, c3) -> (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1, lo(c0*M0));
// the key advances by (0x9E3779B9, 0xBB67AE85) between rounds.
//
// Gaussians by the Box-Muller transform (Box and Muller, 1958).  Stream
// conventions (seed, mode, tag, index) -> value:
//   key      = (seed mod 2^32, seed >> 32)
//   counter  = (lo32(L >> 1), hi32(L >> 1), mode, tag) for linear index L
//   u1, u2   = ((w0 * 2^20 + (w1 >> 12)) + 1/2) * 2^-52 and likewise (w2, w3)
//   z(L)     = sqrt(-2 ln u1) * (cos(2 pi u2) for even L, sin(2 pi u2) for odd L)
// Omega^(n)[j, s] is z at L = s * J_n + j with mode = n and tag = 0; so the
// buffer Omega^T (S x J, row-major) is the stream itself, in order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbki {

struct PhiloxOut { uint32_t w0, w1, w2, w3; };

__host__ __device__ inline void mulhilo32(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}

__host__ __device__ inline PhiloxOut philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                   uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(0xD2511F53u, c0, hi0, lo0);
    mulhilo32(0xCD9E8D57u, c2, hi1, lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  PhiloxOut o = {c0, c1, c2, c3};
  return o;
}

// 52-bit uniform in the open interval (0, 1); exact in double.
__host__ __device__ inline double unit_open(uint32_t wa, uint32_t wb) {
  return ((double)wa * 1048576.0 + (double)(wb >> 12) + 0.5) * 2.220446049250313080847e-16;  // 2^-52
}

// The Box-Muller pair (z(2m), z(2m+1)) for pair index m, in double.
__device__ inline void gauss_pair_f64(uint64_t m, uint32_t mode, uint32_t tag, uint64_t seed,
                                      double& z_even, double& z_odd) {
  PhiloxOut o = philox4x32_10((uint32_t)m, (uint32_t)(m >> 32), mode, tag, (uint32_t)seed,
                              (uint32_t)(seed >> 32));
  double u1 = unit_open(o.w0, o.w1);
  double u2 = unit_open(o.w2, o.w3);
  double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  z_even = r * c;
  z_odd = r * s;
}

// Same pair in single precision (for the float and bfloat16 forms).  The
// uniforms are exact in double; the two arguments that lose accuracy when
// rounded to float are reduced in double first: ln u1 is taken as
// log1p(-(1 - u1)) when u1 >= 1/2, and the angle 2 pi u2 as pi (x - n) with
// n = round(2 u2), so the float arguments carry small absolute errors.
__device__ inline void gauss_pair_f32(uint64_t m, uint32_t mode, uint32_t tag, uint64_t seed,
                                      float& z_even, float& z_odd) {
  PhiloxOut o = philox4x32_10((uint32_t)m, (uint32_t)(m >> 32), mode, tag, (uint32_t)seed,
                              (uint32_t)(seed >> 32));
  const double u1 = unit_open(o.w0, o.w1);
  const double u2 = unit_open(o.w2, o.w3);
  const float ln = u1 < 0.5 ? logf((float)u1) : log1pf(-(float)(1.0 - u1));
  const float r = sqrtf(-2.0f * ln);
  const double x = 2.0 * u2;                  // angle / pi in (0, 2)
  const double nr = rint(x);                  // 0, 1 or 2
  float s, c;
  sincospif((float)(x - nr), &s, &c);
  if (nr == 1.0) { s = -s; c = -c; }          // shift by pi
  z_even = r * c;
  z_odd = r * s;
}

// The same pair for the block-scaled e4m3 sketch, whose values are rounded to
// bfloat16 and then to 3-bit mantissas under a shared power-of-two scale:
// uniforms from the first word of each half (u = (w + 1/2) 2^-32, in float),
// the hardware base-2 logarithm, square root, and sine and cosine of an
// argument in turns (sin(2 pi a)).  The values follow the stream above to
// about 1e-6, far below the bfloat16 step of 2^-8.
__device__ inline void gauss_pair_e4m3(uint64_t m, uint32_t mode, uint32_t tag, uint64_t seed,
                                       float& z_even, float& z_odd) {
  PhiloxOut o = philox4x32_10((uint32_t)m, (uint32_t)(m >> 32), mode, tag, (uint32_t)seed,
                              (uint32_t)(seed >> 32));
  const float u1 = fmaf((float)o.w0, 0x1p-32f, 0x1p-33f);
  const float a = fmaf((float)o.w2, 0x1p-32f, 0x1p-33f);
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));   // -2 ln 2 log2 u1
  z_even = r * __builtin_amdgcn_cosf(a);
  z_odd = r * __builtin_amdgcn_sinf(a);
}

}  // namespace rbki
