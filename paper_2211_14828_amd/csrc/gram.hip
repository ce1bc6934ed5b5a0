// Sketch and Gram products of one mode, in a single pass over the tensor.
//
// For the mode-n view [A, I, B] of the row-major tensor (Table 1:
// X_(n)[i, a*B + b] = X[a, i, b], never materialised) this computes
//   C = X_(n) X_(n)^T            (I x I, lower-triangle tiles)     (Remark 1)
//   W = X_(n) Omega^(n)          (I x S, read through Omega^T)     (Alg. 1, step 2)
// as one extended product [X_(n); Omega^T] x X_(n)^T: the output tiles are the
// lower triangle of C plus one tile column per 128 sketch columns.  Each
// workgroup owns one 128 x 128 output tile and one contiguous slice of the
// contraction index (split-K); slices are reduced in a fixed order in float64
// by a second kernel, so results are deterministic.
//
// The contraction index runs over K tiles that never cross an a-slab: for
// B > 1 a tile is (a, b0 .. b0+BK) (rows of X[a] are contiguous in b, masked
// at the slab end); for B == 1 (last mode) a tile is a0 .. a0+BK and the
// operand is transposed while it is staged into LDS.
//
// Workgroups are dispatched round-robin over the 8 XCDs.  When the split count
// is a multiple of 8, all tiles of one split are mapped to the same XCD so the
// slab of X that they share is fetched from HBM once into that XCD's L2.
//
// Thin modes (float32, I <= 64 and S <= 64, e.g. the 64-row modes of a 64^5
// tensor) use one 128 x 64 output tile instead of two 128 x 128 ones: the
// staged operand holds the mode's rows (0..63) and the sketch rows (64..127),
// the other operand is its first 64 rows, so the tile is [C; W^T] and a wave
// computes 64 x 32 of it.  Two thirds of its products are wanted, against a
// sixth for the square tiles.
#include "rbki_kernels.h"
#include "rbki_mma.h"
#include "rbki_philox.h"

namespace rbki {

namespace {

template <int E>
struct Stage {
  typedef typename Mma<E>::T T;
  static constexpr int BK = Mma<E>::BK;
  static constexpr int EPC = 16 / (int)sizeof(T);     // elements per 16-byte chunk
  uint4 chunk[4];
  unsigned valid;                                     // VEC form: bit j = chunk j in range
};

// Load one operand tile (128 rows x BK k) of the mode view into registers.
// omega_rows: rows are sketch columns s (rows of Omega^T, length J).
//
// VEC (rows and row strides a multiple of 16 bytes, so a 16-byte chunk is
// either wholly inside the tile or wholly outside): every lane issues its
// loads unconditionally from a clamped, always valid address and records
// which chunks are real; the mask is applied when the chunks are written to
// LDS.  No load sits under divergent control flow, so all of them stay in
// flight together while the previous K tile is multiplied.  The other form
// reads element by element with per-element bounds.
template <int E, bool VEC>
__device__ inline void load_operand(Stage<E>& st, const GramArgs& g, const void* base, bool omega_rows,
                                    int64_t row0, int64_t nrows, int64_t a, int64_t b0, int64_t kvalid) {
  typedef typename Mma<E>::T T;
  constexpr int EPC = Stage<E>::EPC;
  constexpr int BK = Stage<E>::BK;
  const T* X = (const T*)base;
  const int tid = threadIdx.x;
  if (VEC) st.valid = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    if (g.B > 1 || omega_rows) {
      // chunk c: row c / (BK/EPC), k offset (c % (BK/EPC)) * EPC
      const int row = c / (BK / EPC);
      const int kk = (c % (BK / EPC)) * EPC;
      const int64_t r = row0 + row;
      if (VEC) {
        const bool ok = r < nrows && kk < kvalid;
        const int64_t rc = r < nrows ? r : nrows - 1;
        const int kc = kk < kvalid ? kk : 0;
        const int64_t off = omega_rows ? rc * g.J + (g.B > 1 ? a * g.B + b0 : b0) + kc
                                       : (a * g.I + rc) * g.B + b0 + kc;
        st.chunk[j] = *(const uint4*)(X + off);
        st.valid |= ok ? 1u << j : 0u;
      } else {
        union { uint4 v; T e[EPC]; } u;
        u.v = make_uint4(0, 0, 0, 0);
        if (r < nrows) {
          const int64_t off = omega_rows ? r * g.J + (g.B > 1 ? a * g.B + b0 : b0) + kk
                                         : (a * g.I + r) * g.B + b0 + kk;
#pragma unroll
          for (int e = 0; e < EPC; ++e)
            if (kk + e < kvalid) u.e[e] = X[off + e];
        }
        st.chunk[j] = u.v;
      }
    } else {
      // B == 1, rows of X_(n) are the contiguous index: chunk c covers EPC
      // consecutive rows at one k.
      const int per_k = TILE / EPC;
      const int kk = c / per_k;
      const int row = (c % per_k) * EPC;
      const int64_t r = row0 + row;
      if (VEC) {
        const bool ok = kk < kvalid && r < nrows;
        const int64_t rc = r < nrows ? r : nrows - EPC;
        const int kc = kk < kvalid ? kk : 0;
        st.chunk[j] = *(const uint4*)(X + (b0 + kc) * g.I + rc);   // b0 is a0 here
        st.valid |= ok ? 1u << j : 0u;
      } else {
        union { uint4 v; T e[EPC]; } u;
        u.v = make_uint4(0, 0, 0, 0);
        if (kk < kvalid) {
          const int64_t off = (b0 + kk) * g.I + r;
#pragma unroll
          for (int e = 0; e < EPC; ++e)
            if (r + e < nrows) u.e[e] = X[off + e];
        }
        st.chunk[j] = u.v;
      }
    }
  }
}

template <int E, bool VEC>
__device__ inline void store_operand(const Stage<E>& st, const GramArgs& g, bool omega_rows, char* lds) {
  typedef typename Mma<E>::T T;
  constexpr int EPC = Stage<E>::EPC;
  constexpr int BK = Stage<E>::BK;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    uint4 v = st.chunk[j];
    if (VEC && !((st.valid >> j) & 1u)) v = make_uint4(0, 0, 0, 0);
    if (g.B > 1 || omega_rows) {
      const int row = c / (BK / EPC);
      const int kk = (c % (BK / EPC)) * EPC;
      *(uint4*)(lds + row * LDS_ROW + kk * (int)sizeof(T)) = v;
    } else {
      const int per_k = TILE / EPC;
      const int kk = c / per_k;
      const int row = (c % per_k) * EPC;
      union { uint4 v; T e[EPC]; } u;
      u.v = v;
#pragma unroll
      for (int e = 0; e < EPC; ++e) *(T*)(lds + (row + e) * LDS_ROW + kk * (int)sizeof(T)) = u.e[e];
    }
  }
}

__device__ inline void decode_tile(const GramArgs& g, int tile, int& ti, int& tj, bool& is_w) {
  if (tile < g.ntri) {
    // tile = ti*(ti+1)/2 + tj, tj <= ti
    int t = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
    while ((t + 1) * (t + 2) / 2 <= tile) ++t;
    while (t * (t + 1) / 2 > tile) --t;
    ti = t;
    tj = tile - t * (t + 1) / 2;
    is_w = false;
  } else {
    int w = tile - g.ntri;
    ti = w / g.nw;
    tj = w % g.nw;
    is_w = true;
  }
}

// Thin tile staging (float32): chunk j < 2 of a thread is one of 512 chunks
// of the mode's 64 rows, j >= 2 one of the sketch's 64 rows.
struct ThinStage {
  uint4 chunk[4];
  unsigned valid;
};

template <bool VEC>
__device__ inline void load_thin(ThinStage& st, const GramArgs& g, int64_t a, int64_t b0, int64_t kvalid) {
  const float* X = (const float*)g.X;
  const float* O = (const float*)g.omegaT;
  const int tid = threadIdx.x;
  st.valid = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * (j & 1);
    if (j < 2 && g.B == 1) {
      // the last mode: rows of X_(n) are the contiguous index; chunk c covers
      // 4 consecutive rows at one k
      const int kk = c >> 4, row = (c & 15) * 4;
      const bool ok = kk < kvalid && row < g.I;
      if (VEC) {
        const int64_t rc = row < g.I ? row : g.I - 4;
        const int kc = kk < kvalid ? kk : 0;
        st.chunk[j] = *(const uint4*)(X + (b0 + kc) * g.I + rc);
      } else {
        union { uint4 v; float e[4]; } u;
        u.v = make_uint4(0, 0, 0, 0);
        if (kk < kvalid) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (row + e < g.I) u.e[e] = X[(b0 + kk) * g.I + row + e];
        }
        st.chunk[j] = u.v;
      }
      st.valid |= ok ? 1u << j : 0u;
    } else {
      // row c / 8, k offset (c % 8) * 4; the mode's rows or the sketch's
      const int row = c >> 3, kk = (c & 7) * 4;
      const bool om = j >= 2;
      const int64_t nrows = om ? g.S : g.I;
      const bool ok = row < nrows && kk < kvalid;
      const int64_t kbase = g.B > 1 ? a * g.B + b0 : b0;
      if (VEC) {
        const int64_t rc = row < nrows ? row : nrows - 1;
        const int kc = kk < kvalid ? kk : 0;
        st.chunk[j] = om ? *(const uint4*)(O + rc * g.J + kbase + kc)
                         : *(const uint4*)(X + (a * g.I + rc) * g.B + b0 + kc);
      } else {
        union { uint4 v; float e[4]; } u;
        u.v = make_uint4(0, 0, 0, 0);
        if (row < nrows) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (kk + e < kvalid)
              u.e[e] = om ? O[(int64_t)row * g.J + kbase + kk + e] : X[(a * g.I + row) * g.B + b0 + kk + e];
        }
        st.chunk[j] = u.v;
      }
      st.valid |= ok ? 1u << j : 0u;
    }
  }
}

__device__ inline void store_thin(const ThinStage& st, const GramArgs& g, char* lds) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * (j & 1);
    const uint4 v = ((st.valid >> j) & 1u) ? st.chunk[j] : make_uint4(0, 0, 0, 0);
    if (j < 2 && g.B == 1) {
      const int kk = c >> 4, row = (c & 15) * 4;
      union { uint4 v; float e[4]; } u;
      u.v = v;
#pragma unroll
      for (int e = 0; e < 4; ++e) *(float*)(lds + (row + e) * LDS_ROW + kk * 4) = u.e[e];
    } else {
      const int row = (c >> 3) + (j >= 2 ? 64 : 0), kk = (c & 7) * 4;
      *(uint4*)(lds + row * LDS_ROW + kk * 4) = v;
    }
  }
}

// One K tile of the thin product for a wave's 64 x 32 block: rows wr + 32 m
// + (lane % 32) of the staged operand, columns wc + (lane % 32) of its first
// 64 rows (the 32x32 layout of rbki_mma.h, blocks m = 0, 1).
__device__ inline void thin_step(f32x16_t (&c)[2], const char* lds, int lane, int wr, int wc) {
  const int half = lane >> 5, r = lane & 31;
  float a[2][16], b[16];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const float4* pa = (const float4*)(lds + (wr + m * 32 + r) * LDS_ROW + half * 64);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = pa[q];
      a[m][4 * q] = v.x; a[m][4 * q + 1] = v.y; a[m][4 * q + 2] = v.z; a[m][4 * q + 3] = v.w;
    }
  }
  const float4* pb = (const float4*)(lds + (wc + r) * LDS_ROW + half * 64);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = pb[q];
    b[4 * q] = v.x; b[4 * q + 1] = v.y; b[4 * q + 2] = v.z; b[4 * q + 3] = v.w;
  }
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m) c[m] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m][t], b[t], c[m], 0, 0, 0);
}

template <bool VEC>
__device__ inline void thin_tile(const GramArgs& g, int split, char (&lds)[2][2][TILE * LDS_ROW]) {
  constexpr int BK = Mma<E_F32>::BK;
  const int64_t kt0 = (int64_t)split * g.nkt / g.splits;
  const int64_t kt1 = (int64_t)(split + 1) * g.nkt / g.splits;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 32;
  f32x16_t acc[2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[m][v] = 0.f;
  ThinStage st;
  auto load = [&](int64_t kt) {
    int64_t a, b0, kv;
    if (g.B > 1) {
      a = kt / g.nbt;
      b0 = (kt - a * g.nbt) * BK;
      kv = g.B - b0 < BK ? g.B - b0 : BK;
    } else {
      a = 0;
      b0 = kt * BK;
      kv = g.A - b0 < BK ? g.A - b0 : BK;
    }
    load_thin<VEC>(st, g, a, b0, kv);
  };
  if (kt0 < kt1) {
    load(kt0);
    store_thin(st, g, lds[0][0]);
    __syncthreads();
    for (int64_t kt = kt0; kt < kt1; ++kt) {
      const int buf = (int)((kt - kt0) & 1);
      const bool more = kt + 1 < kt1;
      if (more) load(kt + 1);
      thin_step(acc, lds[buf][0], lane, wr, wc);
      if (more) store_thin(st, g, lds[buf ^ 1][0]);
      __syncthreads();
    }
  }
  // rows 0..63: C (row i, column j); rows 64..127: W^T (row 64 + s, column i)
  float* out = (float*)g.partial + (int64_t)split * (TILE * TILE);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = wr + m * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      out[row * TILE + wc + (lane & 31)] = acc[m][v];
    }
}

template <int E, bool VEC>
__global__ void __launch_bounds__(256, E == E_F64 ? 1 : 2) gram_sketch_kernel(GramArgs g) {
  typedef Mma<E> M;
  typedef typename M::Out Out;
  constexpr int BK = M::BK;
  __shared__ __attribute__((aligned(16))) char lds[2][2][TILE * LDS_ROW];

  if constexpr (E == E_F32) {
    if (g.thin) {
      // one tile: the split is the workgroup (the XCD map gives the same)
      thin_tile<VEC>(g, (int)blockIdx.x, lds);
      return;
    }
  }
  // workgroup -> (split, tile)
  const int w = blockIdx.x;
  int split, tile;
  if (g.xcd_map) {
    const int xcd = w & 7, slot = w >> 3;
    split = xcd + 8 * (slot / g.ntiles);
    tile = slot % g.ntiles;
  } else {
    split = w / g.ntiles;
    tile = w % g.ntiles;
  }
  int ti, tj;
  bool is_w;
  decode_tile(g, tile, ti, tj, is_w);
  const bool diag = !is_w && ti == tj;
  const int64_t r0 = (int64_t)ti * TILE, c0 = (int64_t)tj * TILE;

  const int64_t kt0 = (int64_t)split * g.nkt / g.splits;
  const int64_t kt1 = (int64_t)(split + 1) * g.nkt / g.splits;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;

  typename M::Frag f;
  M::zero(f);

  Stage<E> sa, sb;
  auto kt_coords = [&](int64_t kt, int64_t& a, int64_t& b0, int64_t& kvalid) {
    if (g.B > 1) {
      a = kt / g.nbt;
      b0 = (kt - a * g.nbt) * BK;
      kvalid = g.B - b0 < BK ? g.B - b0 : BK;
    } else {
      a = 0;
      b0 = kt * BK;
      kvalid = g.A - b0 < BK ? g.A - b0 : BK;
    }
  };
  auto load = [&](int64_t kt) {
    int64_t a, b0, kv;
    kt_coords(kt, a, b0, kv);
    load_operand<E, VEC>(sa, g, g.X, false, r0, g.I, a, b0, kv);
    if (is_w) load_operand<E, VEC>(sb, g, g.omegaT, true, c0, g.S, a, b0, kv);
    else if (!diag) load_operand<E, VEC>(sb, g, g.X, false, c0, g.I, a, b0, kv);
  };
  auto store = [&](int buf) {
    store_operand<E, VEC>(sa, g, false, lds[buf][0]);
    if (is_w) store_operand<E, VEC>(sb, g, true, lds[buf][1]);
    else if (!diag) store_operand<E, VEC>(sb, g, false, lds[buf][1]);
  };

  if (kt0 < kt1) {
    load(kt0);
    store(0);
    __syncthreads();
    for (int64_t kt = kt0; kt < kt1; ++kt) {
      const int buf = (int)((kt - kt0) & 1);
      const bool more = kt + 1 < kt1;
      if (more) load(kt + 1);
      M::step(f, lds[buf][0], diag ? lds[buf][0] : lds[buf][1], lane, wr, wc);
      if (more) store(buf ^ 1);
      __syncthreads();
    }
  }

  Out* out = (Out*)g.partial + ((int64_t)split * g.ntiles + tile) * (TILE * TILE);
#pragma unroll
  for (int j = 0; j < M::NACC; ++j) {
    int row, col;
    M::coord(j, lane, row, col);
    out[(wr + row) * TILE + wc + col] = M::get(f, j);
  }
}

// Sum the split-K partials in a fixed order: C (I x I, both triangles) and
// W^T (S x I), float64.
template <class Out>
__global__ void gram_reduce_kernel(GramArgs g, double* C, double* Wt) {
  const int64_t nC = g.I * g.I;
  const int64_t total = nC + (int64_t)g.S * g.I;
  const int64_t stride = (int64_t)TILE * TILE * g.ntiles;
  const Out* P = (const Out*)g.partial;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t tile, idx;
    if (e < nC) {
      int64_t i = e / g.I, j = e - i * g.I;
      int64_t ti = i / TILE, tj = j / TILE;
      if (ti >= tj) {
        tile = ti * (ti + 1) / 2 + tj;
        idx = (i - ti * TILE) * TILE + (j - tj * TILE);
      } else {
        tile = tj * (tj + 1) / 2 + ti;
        idx = (j - tj * TILE) * TILE + (i - ti * TILE);
      }
    } else if (g.thin) {
      int64_t f = e - nC;
      int64_t s = f / g.I, i = f - s * g.I;
      tile = 0;
      idx = (64 + s) * TILE + i;
    } else {
      int64_t f = e - nC;
      int64_t s = f / g.I, i = f - s * g.I;
      int64_t ti = i / TILE, sj = s / TILE;
      tile = g.ntri + ti * g.nw + sj;
      idx = (i - ti * TILE) * TILE + (s - sj * TILE);
    }
    double acc = 0.0;
    for (int sp = 0; sp < g.splits; ++sp) acc += (double)P[sp * stride + tile * (TILE * TILE) + idx];
    if (e < nC) C[e] = acc;
    else Wt[e - nC] = acc;
  }
}

// Omega^T (S x J) in the element type of the product.
template <class T>
__device__ inline T from_double(double v);
template <> __device__ inline double from_double<double>(double v) { return v; }
template <> __device__ inline float from_double<float>(double v) { return (float)v; }

template <int E>
__global__ void omega_kernel(uint64_t seed, uint32_t mode, int64_t total, void* out) {
  const int64_t npairs = (total + 1) / 2;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < npairs;
       m += (int64_t)gridDim.x * blockDim.x) {
    const int64_t L = 2 * m;
    if (E == E_F64) {
      double z0, z1;
      gauss_pair_f64((uint64_t)m, mode, 0u, seed, z0, z1);
      double* o = (double*)out;
      o[L] = z0;
      if (L + 1 < total) o[L + 1] = z1;
    } else {
      float z0, z1;
      gauss_pair_f32((uint64_t)m, mode, 0u, seed, z0, z1);
      if (E == E_F32) {
        float* o = (float*)out;
        o[L] = z0;
        if (L + 1 < total) o[L + 1] = z1;
      } else if (E == E_BF16) {
        bf16_t* o = (bf16_t*)out;
        o[L] = f32_to_bf16(z0);
        if (L + 1 < total) o[L + 1] = f32_to_bf16(z1);
      } else {
        fp8_t* o = (fp8_t*)out;
        o[L] = f32_to_e4m3(z0);
        if (L + 1 < total) o[L + 1] = f32_to_e4m3(z1);
      }
    }
  }
}

__global__ void philox_kernel(const uint32_t* ctr, int64_t count, uint64_t seed, uint32_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    PhiloxOut o = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                                (uint32_t)seed, (uint32_t)(seed >> 32));
    out[4 * i] = o.w0;
    out[4 * i + 1] = o.w1;
    out[4 * i + 2] = o.w2;
    out[4 * i + 3] = o.w3;
  }
}

}  // namespace

// ------------------------------------------------------------------ planning

int gram_bk(int elem) {
  switch (elem) {
    case E_F64: return Mma<E_F64>::BK;
    case E_F32: return Mma<E_F32>::BK;
    default: return Mma<E_BF16>::BK;       // the 128-tile kernel has no fp8 form
  }
}

int elem_size(int elem) { return elem == E_F64 ? 8 : elem == E_F32 ? 4 : elem == E_BF16 ? 2 : 1; }

GramArgs gram_plan(int elem, int64_t A, int64_t I, int64_t B, int S, int cu_count) {
  GramArgs g = {};
  g.A = A;
  g.I = I;
  g.B = B;
  g.J = A * B;
  g.S = S;
  g.nt = (int)ceil_div(I, TILE);
  g.ntri = g.nt * (g.nt + 1) / 2;
  g.nw = S > 0 ? (int)ceil_div(S, TILE) : 0;
  g.ntiles = g.ntri + g.nt * g.nw;
  g.thin = (elem == E_F32 && I <= 64 && S >= 1 && S <= 64) ? 1 : 0;
  if (g.thin) {
    g.nw = 0;
    g.ntiles = 1;
  }
  const int bk = gram_bk(elem);
  if (B > 1) {
    g.nbt = ceil_div(B, bk);
    g.nkt = A * g.nbt;
  } else {
    g.nbt = 0;
    g.nkt = ceil_div(A, bk);
  }
  // split-K: aim for >= 2 workgroups per CU, keep >= 8 K tiles per split
  const int64_t want = ceil_div(2 * (int64_t)cu_count, g.ntiles);
  int64_t splits = want < 1 ? 1 : want;
  const int64_t max_by_k = g.nkt / 8 > 0 ? g.nkt / 8 : 1;
  if (splits > max_by_k) splits = max_by_k;
  if (splits >= 8) splits = (splits + 7) / 8 * 8;
  if (splits > g.nkt) splits = g.nkt > 0 ? g.nkt : 1;
  g.splits = (int)splits;
  g.xcd_map = (g.splits % 8 == 0) ? 1 : 0;
  const int es = elem_size(elem);
  g.vec_ok = ((B > 1 ? B : I) * es) % 16 == 0 && (g.J * es) % 16 == 0 ? 1 : 0;
  return g;
}

size_t gram_partial_bytes(const GramArgs& g, int elem) {
  return (size_t)g.splits * g.ntiles * TILE * TILE * (elem == E_F64 ? 8 : 4);
}

// Vector loads need every row start 16-byte aligned: sizes (vec_ok) and base pointers.
static bool gram_vec(const GramArgs& g) {
  return g.vec_ok && ((uintptr_t)g.X % 16) == 0 && ((uintptr_t)g.omegaT % 16) == 0;
}

template <int E>
static void launch_sketch(const GramArgs& g, unsigned grid, hipStream_t s) {
  if (gram_vec(g)) hipLaunchKernelGGL((gram_sketch_kernel<E, true>), dim3(grid), dim3(256), 0, s, g);
  else hipLaunchKernelGGL((gram_sketch_kernel<E, false>), dim3(grid), dim3(256), 0, s, g);
}

hipError_t launch_gram_main(int elem, const GramArgs& g, hipStream_t s) {
  const unsigned grid = (unsigned)(g.ntiles * g.splits);
  switch (elem) {
    case E_F64: launch_sketch<E_F64>(g, grid, s); break;
    case E_F32: launch_sketch<E_F32>(g, grid, s); break;
    case E_BF16: launch_sketch<E_BF16>(g, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gram_reduce(int elem, const GramArgs& g, double* C, double* Wt, hipStream_t s) {
  const int64_t total = g.I * g.I + (int64_t)g.S * g.I;
  unsigned rgrid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096);
  if (elem == E_F64) hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(rgrid), dim3(256), 0, s, g, C, Wt);
  else hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3(rgrid), dim3(256), 0, s, g, C, Wt);
  return hipGetLastError();
}

hipError_t launch_omega(int elem, uint64_t seed, int mode, int64_t total, void* out, hipStream_t s) {
  const int64_t npairs = (total + 1) / 2;
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(npairs, 256), 16384);
  if (grid == 0) return hipSuccess;
  switch (elem) {
    case E_F64: hipLaunchKernelGGL(omega_kernel<E_F64>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, total, out); break;
    case E_F32: hipLaunchKernelGGL(omega_kernel<E_F32>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, total, out); break;
    case E_BF16: hipLaunchKernelGGL(omega_kernel<E_BF16>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, total, out); break;
    default: hipLaunchKernelGGL(omega_kernel<E_FP8>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, total, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, int64_t count, uint64_t seed, uint32_t* out, hipStream_t s) {
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(count, 256), 4096);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(philox_kernel, dim3(grid), dim3(256), 0, s, ctr, count, seed, out);
  return hipGetLastError();
}

}  // namespace rbki
