// MFMA tile machinery shared by the tensor-reading kernels (gfx950).
//
// Every product here is organised as out[r, c] = sum_k Arow[r][k] * Bcol[c][k]
// with both operands staged in LDS as [row][k] (k contiguous).  A wave owns a
// 64 x 64 block of the output.  Lane layouts (measured on gfx950):
//   32x32 blocks (fp32 x2, bf16 x16, fp8 x64): lane l supplies row l % 32 of
//     A and column l % 32 of B for its half (l / 32) of the K step; the result
//     value v of lane l sits at row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
//   16x16x4 fp64: lane l supplies row/column l % 16 at k = l / 16; result value
//     v sits at row 4 v + l / 16, column l % 16.
// The K order inside a lane is free (it only has to agree between A and B), so
// each lane reads one contiguous run of k from LDS.
#pragma once
#include "rbki_common.h"

namespace rbki {

// Tile geometry: 128 x 128 output per workgroup of 256 threads (4 waves of
// 64 x 64), and one LDS row of 128 bytes of K per operand row.
constexpr int TILE = 128;
constexpr int ROW_BYTES = 128;
constexpr int LDS_PAD_BYTES = 16;
constexpr int LDS_ROW = ROW_BYTES + LDS_PAD_BYTES;   // 144 B: conflict-free 16 B reads

template <int E> struct Mma;

// ---------------------------------------------------------------- fp32
template <> struct Mma<E_F32> {
  typedef float T;
  typedef float Out;                           // accumulator element type
  struct Frag { f32x16_t c[4]; };              // 2 x 2 blocks of 32 x 32
  static constexpr int BK = ROW_BYTES / 4;     // 32 k per LDS tile
  static constexpr int NACC = 64;
  __device__ static inline void zero(Frag& f) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) f.c[i][v] = 0.f;
  }
  __device__ static inline float get(const Frag& f, int j) { return f.c[j >> 4][j & 15]; }
  // rowA, rowB: LDS byte offsets of this lane's rows for the 2 A and 2 B blocks
  __device__ static inline void step(Frag& f, const char* lds_a, const char* lds_b, int lane,
                                     int wr, int wc) {
    const int half = lane >> 5, r = lane & 31;
    // lane reads 16 contiguous floats of its row: k = half*16 + t
    float a[2][16], b[2][16];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const float4* pa = (const float4*)(lds_a + (wr + m * 32 + r) * LDS_ROW + half * 64);
      const float4* pb = (const float4*)(lds_b + (wc + m * 32 + r) * LDS_ROW + half * 64);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float4 va = pa[q], vb = pb[q];
        a[m][4 * q] = va.x; a[m][4 * q + 1] = va.y; a[m][4 * q + 2] = va.z; a[m][4 * q + 3] = va.w;
        b[m][4 * q] = vb.x; b[m][4 * q + 1] = vb.y; b[m][4 * q + 2] = vb.z; b[m][4 * q + 3] = vb.w;
      }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          f.c[m * 2 + n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m][t], b[n][t], f.c[m * 2 + n], 0, 0, 0);
        }
      }
    }
  }
  // output coordinates of accumulator j (relative to the wave's 64x64 block)
  __device__ static inline void coord(int j, int lane, int& row, int& col) {
    int blk = j >> 4, v = j & 15;
    row = (blk >> 1) * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    col = (blk & 1) * 32 + (lane & 31);
  }
};

// ---------------------------------------------------------------- bf16
template <> struct Mma<E_BF16> {
  typedef bf16_t T;
  typedef float Out;
  typedef Mma<E_F32>::Frag Frag;
  static constexpr int BK = ROW_BYTES / 2;     // 64 k per LDS tile
  static constexpr int NACC = 64;
  __device__ static inline void zero(Frag& f) { Mma<E_F32>::zero(f); }
  __device__ static inline float get(const Frag& f, int j) { return f.c[j >> 4][j & 15]; }
  __device__ static inline void step(Frag& f, const char* lds_a, const char* lds_b, int lane,
                                     int wr, int wc) {
    const int half = lane >> 5, r = lane & 31;
    // lane reads 32 contiguous bf16 of its row: 4 MFMA steps of 8
    bf16x8_t a[2][4], b[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const bf16x8_t* pa = (const bf16x8_t*)(lds_a + (wr + m * 32 + r) * LDS_ROW + half * 64);
      const bf16x8_t* pb = (const bf16x8_t*)(lds_b + (wc + m * 32 + r) * LDS_ROW + half * 64);
#pragma unroll
      for (int q = 0; q < 4; ++q) { a[m][q] = pa[q]; b[m][q] = pb[q]; }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          f.c[m * 2 + n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[m][t], b[n][t], f.c[m * 2 + n], 0, 0, 0);
        }
      }
    }
  }
  __device__ static inline void coord(int j, int lane, int& row, int& col) {
    Mma<E_F32>::coord(j, lane, row, col);
  }
};

// ---------------------------------------------------------------- fp64
template <> struct Mma<E_F64> {
  typedef double T;
  typedef double Out;
  struct Frag { f64x4_t c[16]; };              // 4 x 4 blocks of 16 x 16
  static constexpr int BK = ROW_BYTES / 8;     // 16 k per LDS tile
  static constexpr int NACC = 64;
  __device__ static inline void zero(Frag& f) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) f.c[i][v] = 0.0;
  }
  __device__ static inline double get(const Frag& f, int j) { return f.c[j >> 2][j & 3]; }
  __device__ static inline void step(Frag& f, const char* lds_a, const char* lds_b, int lane,
                                     int wr, int wc) {
    const int g = lane >> 4, r = lane & 15;
    // lane reads 4 contiguous doubles of its row: k = g*4 + t
    double a[4][4], b[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const double2* pa = (const double2*)(lds_a + (wr + m * 16 + r) * LDS_ROW + g * 32);
      const double2* pb = (const double2*)(lds_b + (wc + m * 16 + r) * LDS_ROW + g * 32);
      double2 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
      a[m][0] = a0.x; a[m][1] = a0.y; a[m][2] = a1.x; a[m][3] = a1.y;
      b[m][0] = b0.x; b[m][1] = b0.y; b[m][2] = b1.x; b[m][3] = b1.y;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          f.c[m * 4 + n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m][t], b[n][t], f.c[m * 4 + n], 0, 0, 0);
        }
      }
    }
  }
  __device__ static inline void coord(int j, int lane, int& row, int& col) {
    int blk = j >> 2, v = j & 3;
    row = (blk >> 2) * 16 + 4 * v + (lane >> 4);
    col = (blk & 3) * 16 + (lane & 15);
  }
};

}  // namespace rbki
