// Mode-n products (Alg. 2, step 6: G <- G x_n U^(n)T, and the reconstruction
// G x_n U^(n)) and the fused reconstruction-error reduction, on MFMA.
//
// Both are products out[row, col] = sum_k Aop[row, k] * Bop[col, k] in which
// each operand is strided: either k is its contiguous index ("k-contiguous")
// or the row is ("row-contiguous", transposed while staged into LDS).  A
// mode-n product with U on the view [A, I, B] is, for every a, the product
// Y[a] (R x B) = U^T (R x I) X[a] (I x B); for the last mode (B = 1) it is
// Y (A x R) = X (A x I) U (I x R).  The error pass computes the mode-0
// reconstruction Xhat_(0) = U^(1) H tile by tile and folds (x - xhat)^2 and
// x^2 into float64 partial sums without writing Xhat.
#include "rbki_kernels.h"
#include "rbki_mma.h"

namespace rbki {

namespace {

struct Operand {
  const void* base;
  int64_t row_stride, k_stride;   // one of them is 1
  int64_t batch_stride;
  int64_t rows;                   // valid rows
};

struct ProdArgs {
  Operand a, b;
  int64_t K;                      // contraction length
  int64_t row_tiles, col_tiles;
  // store epilogue
  void* out;
  int64_t out_rs, out_cs, out_bs;
  int64_t out_in, out_inp;        // out_inp > 0: output columns are padded (groups of out_inp, out_in valid)
  // residual epilogue: X (row-major rows x J) of element x_elem
  const void* X;
  int x_elem;
  int64_t xJ;
  double* partial;                // [grid] x 2
  int vec_a, vec_b;
};

// Stage 4 chunks (16 bytes each) of one operand tile in registers.
// VEC (row starts 16-byte aligned, and the sizes make every chunk wholly in
// or wholly out of range): each lane loads unconditionally from a clamped,
// valid address and keeps a validity bit per chunk; the mask is applied when
// the chunks are written to LDS, so no load sits under divergent control flow.
template <int E, bool VEC>
__device__ inline void load_op(uint4* chunk, unsigned& valid, const Operand& op, int64_t batch, int64_t row0,
                               int64_t k0, int64_t K) {
  typedef typename Mma<E>::T T;
  constexpr int EPC = 16 / (int)sizeof(T);
  constexpr int BK = Mma<E>::BK;
  const T* base = (const T*)op.base + batch * op.batch_stride;
  const int tid = threadIdx.x;
  valid = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    if (op.k_stride == 1) {
      const int row = c / (BK / EPC);
      const int kk = (c % (BK / EPC)) * EPC;
      const int64_t r = row0 + row, k = k0 + kk;
      if (VEC) {
        const int64_t rc = r < op.rows ? r : op.rows - 1;
        const int64_t kc = k < K ? k : 0;
        chunk[j] = *(const uint4*)(base + rc * op.row_stride + kc);
        valid |= (r < op.rows && k < K) ? 1u << j : 0u;
      } else {
        union { uint4 v; T e[EPC]; } u;
        u.v = make_uint4(0, 0, 0, 0);
        if (r < op.rows) {
          const T* p = base + r * op.row_stride + k;
#pragma unroll
          for (int e = 0; e < EPC; ++e)
            if (k + e < K) u.e[e] = p[e];
        }
        chunk[j] = u.v;
        valid |= 1u << j;
      }
    } else {
      const int per_k = TILE / EPC;
      const int kk = c / per_k;
      const int row = (c % per_k) * EPC;
      const int64_t r = row0 + row, k = k0 + kk;
      if (VEC) {
        const int64_t rc = r < op.rows ? r : op.rows - EPC;
        const int64_t kc = k < K ? k : 0;
        chunk[j] = *(const uint4*)(base + kc * op.k_stride + rc);
        valid |= (r < op.rows && k < K) ? 1u << j : 0u;
      } else {
        union { uint4 v; T e[EPC]; } u;
        u.v = make_uint4(0, 0, 0, 0);
        if (k < K) {
          const T* p = base + k * op.k_stride + r;
#pragma unroll
          for (int e = 0; e < EPC; ++e)
            if (r + e < op.rows) u.e[e] = p[e];
        }
        chunk[j] = u.v;
        valid |= 1u << j;
      }
    }
  }
}

template <int E>
__device__ inline void store_op(const uint4* chunk, unsigned valid, const Operand& op, char* lds) {
  typedef typename Mma<E>::T T;
  constexpr int EPC = 16 / (int)sizeof(T);
  constexpr int BK = Mma<E>::BK;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    const uint4 v = ((valid >> j) & 1u) ? chunk[j] : make_uint4(0, 0, 0, 0);
    if (op.k_stride == 1) {
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

template <class T> __device__ inline double load_x(const void* X, int64_t i);
template <> __device__ inline double load_x<double>(const void* X, int64_t i) { return ((const double*)X)[i]; }
template <> __device__ inline double load_x<float>(const void* X, int64_t i) { return (double)((const float*)X)[i]; }
template <> __device__ inline double load_x<bf16_t>(const void* X, int64_t i) {
  return (double)bf16_to_f32(((const bf16_t*)X)[i]);
}

// EPI = 0: store; EPI = 1: residual with X of type XT
template <int E, int EPI, class XT, bool VEC>
__global__ void __launch_bounds__(256, E == E_F64 ? 1 : 2) prod_kernel(ProdArgs p) {
  typedef Mma<E> M;
  typedef typename M::Out Out;
  constexpr int BK = M::BK;
  __shared__ __attribute__((aligned(16))) char lds[2][2][TILE * LDS_ROW];
  __shared__ double red[2][4];

  const int64_t tile = blockIdx.x;
  const int64_t batch = blockIdx.y;
  const int64_t rt = tile % p.row_tiles, ct = tile / p.row_tiles;
  const int64_t r0 = rt * TILE, c0 = ct * TILE;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;

  typename M::Frag f;
  M::zero(f);
  uint4 ca[4], cb[4];
  unsigned va, vb;
  const int64_t nk = ceil_div(p.K, BK);
  load_op<E, VEC>(ca, va, p.a, batch, r0, 0, p.K);
  load_op<E, VEC>(cb, vb, p.b, batch, c0, 0, p.K);
  store_op<E>(ca, va, p.a, lds[0][0]);
  store_op<E>(cb, vb, p.b, lds[0][1]);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) {
      load_op<E, VEC>(ca, va, p.a, batch, r0, (kt + 1) * BK, p.K);
      load_op<E, VEC>(cb, vb, p.b, batch, c0, (kt + 1) * BK, p.K);
    }
    M::step(f, lds[buf][0], lds[buf][1], lane, wr, wc);
    if (more) {
      store_op<E>(ca, va, p.a, lds[buf ^ 1][0]);
      store_op<E>(cb, vb, p.b, lds[buf ^ 1][1]);
    }
    __syncthreads();
  }

  if (EPI == 0) {
    Out* out = (Out*)p.out + batch * p.out_bs;
#pragma unroll
    for (int j = 0; j < M::NACC; ++j) {
      int row, col;
      M::coord(j, lane, row, col);
      const int64_t r = r0 + wr + row;
      int64_t c = c0 + wc + col;
      if (r < p.a.rows && c < p.b.rows) {
        if (p.out_inp > 0) {                       // padded column -> true column
          const int64_t hi = c / p.out_inp, lo = c - hi * p.out_inp;
          if (lo >= p.out_in) continue;
          c = hi * p.out_in + lo;
        }
        out[r * p.out_rs + c * p.out_cs] = M::get(f, j);
      }
    }
  } else {
    double res = 0.0, nrm = 0.0;
#pragma unroll
    for (int j = 0; j < M::NACC; ++j) {
      int row, col;
      M::coord(j, lane, row, col);
      const int64_t r = r0 + wr + row, c = c0 + wc + col;
      if (r < p.a.rows && c < p.b.rows) {
        const double x = load_x<XT>(p.X, r * p.xJ + c);
        const double d = x - (double)M::get(f, j);
        res = fma(d, d, res);
        nrm = fma(x, x, nrm);
      }
    }
    res = warp_sum(res);
    nrm = warp_sum(nrm);
    if (lane == 0) {
      red[0][wave] = res;
      red[1][wave] = nrm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int64_t g = blockIdx.y * (int64_t)gridDim.x + blockIdx.x;
      p.partial[2 * g] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      p.partial[2 * g + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
  }
}

// Fixed-order sum of the per-workgroup partials.
__global__ void sum_pairs_kernel(const double* partial, int64_t n, double* out) {
  __shared__ double sr[16], sn[16];
  double r = 0.0, q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    r += partial[2 * i];
    q += partial[2 * i + 1];
  }
  r = warp_sum(r);
  q = warp_sum(q);
  if ((threadIdx.x & 63) == 0) {
    sr[threadIdx.x >> 6] = r;
    sn[threadIdx.x >> 6] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a += sr[w];
      b += sn[w];
    }
    out[0] = a;
    out[1] = b;
  }
}

// ------------------------------------------------------------------------
// Streaming reconstruction-error pass for R <= 64.  Workgroup w owns columns
// j0 .. j0+127 of X_(0) (I x J) and walks every 128-row tile of it: H(:,
// j0..j0+127) is staged once in LDS as [j][k], the rows of U (I x 64,
// zero-padded) are read straight from L2 into MFMA fragments, and the tile of
// X is requested before the MFMAs so that its HBM reads are in flight while
// Xhat = U H is formed.  (x - xhat)^2 and x^2 are accumulated in float64;
// Xhat is never written.  PE is the product type: float32 (32x32x2 MFMA) or,
// for the precision forms, split bfloat16: each operand is hi + lo with both
// parts bfloat16, and U H = Uh Hh + Uh Hl + Ul Hh on 32x32x16 MFMA with
// float32 accumulation (relative error about 2^-16; a fifth of the
// matrix-core time of the float32 form).
struct ResArgs {
  const void* Up;       // I x 64 row-major, columns >= R zero: float32, or split
                        // bfloat16 (hi parts, then the I x 64 lo parts)
  const float* H;       // R x J row-major
  const void* X;        // I x J row-major
  int64_t I, J;
  int R, nkt;           // nkt = ceil(R / 32) K tiles of 32 (float32 products)
  double* partial;      // [gridDim.x] x 2
};

template <class XT>
__device__ inline float x_to_f(XT v);
template <> __device__ inline float x_to_f<float>(float v) { return v; }
template <> __device__ inline float x_to_f<bf16_t>(bf16_t v) { return bf16_to_f32(v); }

// The split-bfloat16 form: each workgroup owns 64 columns j0.. of X_(0),
// their H block split into bfloat16 hi + lo parts in LDS; wave w walks the
// 16-row tiles w, w + 4, ... and forms Xhat (16 x 64) of a tile as four
// 16 x 16 blocks on 16x16x32 bfloat16 MFMA, K = 64 in two steps, three
// products (Ul Hh + Uh Hl + Uh Hh).  Column c of block n is X column
// j0 + 4 c + n (H is staged in that order), so a lane's four values of a row
// are four consecutive X values, one 16-byte load.  The bound is the bytes in
// flight: with small tiles each wave has X three tiles ahead and U one tile
// ahead, two workgroups per compute unit (1.05 ms alone at 1000^3, against
// 1.16 ms with 32-row tiles one tile ahead; three workgroups per compute unit
// spill registers and took 1.55 ms).  The loads are unconditional (a tile past the
// wave's last is clamped to it) so that the wait before each product counts
// only the loads issued after its operands'.
constexpr int RS_COLS = 64;
constexpr int RS_LDS_ROW = 72;       // bf16 per LDS row: 64 k + 16 bytes of padding
constexpr int RS_TR = 16;            // rows per tile
struct ResSplitArgs {
  const bf16_t* Uh;     // I x 64 (columns >= R zero), hi parts
  const bf16_t* Ul;     // lo parts
  const float* H;       // R x J row-major
  const void* X;        // I x J row-major
  int64_t I, J;
  int R;
  double* partial;      // [gridDim.x] x 2
};

// four consecutive values of X as floats (VEC: one 16-byte or 8-byte load)
template <class XT, bool VEC>
__device__ inline float4 load_x4(const XT* p);
template <> __device__ inline float4 load_x4<float, true>(const float* p) { return *(const float4*)p; }
template <> __device__ inline float4 load_x4<float, false>(const float* p) { return make_float4(p[0], p[1], p[2], p[3]); }
template <> __device__ inline float4 load_x4<bf16_t, true>(const bf16_t* p) {
  const uint2 v = *(const uint2*)p;
  return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u), __uint_as_float(v.y << 16),
                     __uint_as_float(v.y & 0xFFFF0000u));
}
template <> __device__ inline float4 load_x4<bf16_t, false>(const bf16_t* p) {
  return make_float4(bf16_to_f32(p[0]), bf16_to_f32(p[1]), bf16_to_f32(p[2]), bf16_to_f32(p[3]));
}

template <class XT, bool VEC>
__global__ void __launch_bounds__(256, 2) residual_split_kernel(ResSplitArgs a) {
  __shared__ __attribute__((aligned(16))) bf16_t hh[RS_COLS * RS_LDS_ROW];
  __shared__ __attribute__((aligned(16))) bf16_t hl[RS_COLS * RS_LDS_ROW];
  __shared__ double red[2][4];
  // the wave index is uniform across the wave: readfirstlane lets the
  // compiler keep row pointers and loop counters in scalar registers
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c16 = lane & 15, g = lane >> 4;
  const int64_t j0 = (int64_t)blockIdx.x * RS_COLS;

  // H block -> LDS as [p][k], row p = 16 n + c holding column j0 + 4 c + n:
  // a thread takes 4 consecutive columns at one k
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = tid + 256 * q;
    const int kk = c >> 4, jj = (c & 15) * 4;
    const bool ok = kk < a.R && j0 + jj < a.J;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok) v = *(const float4*)(a.H + (int64_t)kk * a.J + j0 + jj);
    const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int p = 16 * e + (jj >> 2);
      const bf16_t hi = f32_to_bf16(vv[e]);
      hh[p * RS_LDS_ROW + kk] = hi;
      hl[p * RS_LDS_ROW + kk] = f32_to_bf16(vv[e] - bf16_to_f32(hi));
    }
  }
  __syncthreads();

  const XT* X = (const XT*)a.X;
  const int64_t NT = ceil_div(a.I, RS_TR);
  const int ns = NT > wave ? (int)((NT - wave + 3) / 4) : 0;      // this wave's tiles wave + 4 s
  if (ns > 0) {
    const bool whole_cols = j0 + RS_COLS <= a.J;
    // this lane's first column, clamped into the matrix (columns past J are masked)
    const int64_t jl = std::min<int64_t>(j0 + 4 * c16, a.J - 4 > 0 ? a.J - 4 : 0);
    auto tile_of = [&](int s) { return (int64_t)wave + 4 * (int64_t)std::min(s, ns - 1); };
    // X: rows 16 t + 4 g + v (clamped), columns jl .. jl + 3
    auto load_x = [&](int s, float4 (&xv)[4]) {
      const int64_t i0 = tile_of(s) * RS_TR + 4 * g;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + v < a.I ? i0 + v : a.I - 1;
        xv[v] = load_x4<XT, VEC>(X + i * a.J + jl);
      }
    };
    // U fragments: row 16 t + c16, k = 32 ks + 8 g .. + 7, hi then lo
    auto load_u = [&](int s, bf16x8_t (&u)[4]) {
      int64_t iu = tile_of(s) * RS_TR + c16;
      iu = iu < a.I ? iu : a.I - 1;
      const bf16_t* ph = a.Uh + iu * 64 + 8 * g;
      const bf16_t* pl = a.Ul + iu * 64 + 8 * g;
      u[0] = *(const bf16x8_t*)ph;
      u[1] = *(const bf16x8_t*)(ph + 32);
      u[2] = *(const bf16x8_t*)pl;
      u[3] = *(const bf16x8_t*)(pl + 32);
    };
    double res = 0.0, nrm = 0.0;
    auto tile = [&](int s, const bf16x8_t (&u)[4], const float4 (&xv)[4]) {
      f32x4_t acc[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[n] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const int row = (16 * n + c16) * RS_LDS_ROW + 32 * ks + 8 * g;
          const bf16x8_t bh = *(const bf16x8_t*)(hh + row);
          const bf16x8_t bl = *(const bf16x8_t*)(hl + row);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u[2 + ks], bh, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u[ks], bl, acc[n], 0, 0, 0);
          acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(u[ks], bh, acc[n], 0, 0, 0);
        }
      // item v of acc[n]: row 16 t + 4 g + v, column j0 + 4 c16 + n
      const int64_t i0 = ((int64_t)wave + 4 * (int64_t)s) * RS_TR + 4 * g;
      if (whole_cols && i0 - 4 * g + RS_TR <= a.I) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float xs[4] = {xv[v].x, xv[v].y, xv[v].z, xv[v].w};
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            const double x = (double)xs[n];
            const double d = x - (double)acc[n][v];
            res = fma(d, d, res);
            nrm = fma(x, x, nrm);
          }
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float xs[4] = {xv[v].x, xv[v].y, xv[v].z, xv[v].w};
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            // the loaded column is jl + n; it is the tile's column only when unclamped
            const bool ok = i0 + v < a.I && j0 + 4 * c16 + n < a.J && jl == j0 + 4 * c16;
            const double x = ok ? (double)xs[n] : 0.0;
            const double d = ok ? x - (double)acc[n][v] : 0.0;
            res = fma(d, d, res);
            nrm = fma(x, x, nrm);
          }
        }
      }
    };
    // X three tiles ahead, U one tile ahead; the register sets rotate with s
    float4 x0[4], x1[4], x2[4], x3[4];
    bf16x8_t ua[4], ub[4];
    load_x(0, x0);
    load_u(0, ua);
    load_x(1, x1);
    load_x(2, x2);
    auto step = [&](int s, const bf16x8_t (&ucur)[4], bf16x8_t (&unext)[4], const float4 (&xcur)[4],
                    float4 (&xfar)[4]) {
      load_u(s + 1, unext);
      load_x(s + 3, xfar);
      if (s < ns) tile(s, ucur, xcur);
    };
    for (int s = 0; s < ns; s += 4) {
      step(s, ua, ub, x0, x3);
      step(s + 1, ub, ua, x1, x0);
      step(s + 2, ua, ub, x2, x1);
      step(s + 3, ub, ua, x3, x2);
    }
    res = warp_sum(res);
    nrm = warp_sum(nrm);
    if (lane == 0) {
      red[0][wave] = res;
      red[1][wave] = nrm;
    }
  } else if (lane == 0) {
    red[0][wave] = 0.0;
    red[1][wave] = 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    a.partial[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    a.partial[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

template <class XT, int PE>
__global__ void __launch_bounds__(256, PE == E_F32 ? 2 : 1) residual_kernel(ResArgs a) {
  __shared__ __attribute__((aligned(16))) char ldsB[2][TILE * LDS_ROW];
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, lr = lane & 31;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  const int64_t j0 = (int64_t)blockIdx.x * TILE;

  // H block -> LDS, transposed: chunk c holds 4 consecutive j at one k.
  // float32: [k / 32][j][k % 32]; bfloat16: [j][k] (64 k in one row)
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int c = tid + 256 * q;
    const int kk = c >> 5, jj = (c & 31) * 4;
    const bool ok = kk < a.R && j0 + jj < a.J;
    const int kc = kk < a.R ? kk : 0;
    const int64_t jc = j0 + jj < a.J ? j0 + jj : 0;
    float4 v = *(const float4*)(a.H + (int64_t)kc * a.J + jc);
    if (!ok) v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (PE == E_F32) {
      char* base = ldsB[kk >> 5] + (kk & 31) * 4;
      *(float*)(base + (jj + 0) * LDS_ROW) = v.x;
      *(float*)(base + (jj + 1) * LDS_ROW) = v.y;
      *(float*)(base + (jj + 2) * LDS_ROW) = v.z;
      *(float*)(base + (jj + 3) * LDS_ROW) = v.w;
    } else {
      // hi parts in ldsB[0], lo parts in ldsB[1], [j][k] with 64 k per row
      const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bf16_t hi = f32_to_bf16(vv[e]);
        *(bf16_t*)(ldsB[0] + kk * 2 + (jj + e) * LDS_ROW) = hi;
        *(bf16_t*)(ldsB[1] + kk * 2 + (jj + e) * LDS_ROW) = f32_to_bf16(vv[e] - bf16_to_f32(hi));
      }
    }
  }
  __syncthreads();

  const XT* X = (const XT*)a.X;
  double res = 0.0, nrm = 0.0;
  const int64_t nit = ceil_div(a.I, TILE);
  // a tile of X in the accumulator layout (rows clamped into the matrix)
  auto load_x = [&](int64_t it, XT (&xv)[64]) {
    const int64_t i0 = it * TILE;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
      int row, col;
      Mma<E_F32>::coord(j, lane, row, col);
      int64_t i = i0 + wr + row, jj = j0 + wc + col;
      i = i < a.I ? i : a.I - 1;
      jj = jj < a.J ? jj : a.J - 1;
      xv[j] = X[i * a.J + jj];
    }
  };
  // Xhat tile = U(i0.., :) H(:, j0..), then (x - xhat)^2 and x^2 into the
  // sums; rows past I (a tile past the end included) add nothing
  auto tile = [&](int64_t it, const XT (&xv)[64]) {
    const int64_t i0 = it * TILE;
    Mma<E_F32>::Frag f;
    Mma<E_F32>::zero(f);
    if (PE == E_F32) {
      const float* Up = (const float*)a.Up;
      for (int kt = 0; kt < a.nkt; ++kt) {
        float av[2][16], bv[2][16];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          int64_t i = i0 + wr + m * 32 + lr;
          i = i < a.I ? i : a.I - 1;
          const float4* pa = (const float4*)(Up + i * 64 + kt * 32 + half * 16);
          const float4* pb = (const float4*)(ldsB[kt] + (wc + m * 32 + lr) * LDS_ROW + half * 64);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 va = pa[q], vb = pb[q];
            av[m][4 * q] = va.x; av[m][4 * q + 1] = va.y; av[m][4 * q + 2] = va.z; av[m][4 * q + 3] = va.w;
            bv[m][4 * q] = vb.x; bv[m][4 * q + 1] = vb.y; bv[m][4 * q + 2] = vb.z; bv[m][4 * q + 3] = vb.w;
          }
        }
#pragma unroll
        for (int t = 0; t < 16; ++t)
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
              f.c[m * 2 + n] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[m][t], bv[n][t], f.c[m * 2 + n], 0, 0, 0);
      }
    } else {
      // lane half h takes k = 32 h .. 32 h + 31 of both operands, 8 per MFMA
      const bf16_t* Uh = (const bf16_t*)a.Up;
      const bf16_t* Ul = Uh + a.I * 64;
      bf16x8_t ah[2][4], al[2][4];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        int64_t i = i0 + wr + m * 32 + lr;
        i = i < a.I ? i : a.I - 1;
        const bf16x8_t* ph = (const bf16x8_t*)(Uh + i * 64 + half * 32);
        const bf16x8_t* pl = (const bf16x8_t*)(Ul + i * 64 + half * 32);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ah[m][q] = ph[q];
          al[m][q] = pl[q];
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        bf16x8_t bh[2], bl[2];
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          bh[n] = ((const bf16x8_t*)(ldsB[0] + (wc + n * 32 + lr) * LDS_ROW + half * 64))[t];
          bl[n] = ((const bf16x8_t*)(ldsB[1] + (wc + n * 32 + lr) * LDS_ROW + half * 64))[t];
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n) {
            f.c[m * 2 + n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[m][t], bh[n], f.c[m * 2 + n], 0, 0, 0);
            f.c[m * 2 + n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[m][t], bl[n], f.c[m * 2 + n], 0, 0, 0);
            f.c[m * 2 + n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[m][t], bh[n], f.c[m * 2 + n], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int j = 0; j < 64; ++j) {
      int row, col;
      Mma<E_F32>::coord(j, lane, row, col);
      const bool ok = i0 + wr + row < a.I && j0 + wc + col < a.J;
      const double x = ok ? (double)x_to_f<XT>(xv[j]) : 0.0;
      const double d = ok ? x - (double)Mma<E_F32>::get(f, j) : 0.0;
      res = fma(d, d, res);
      nrm = fma(x, x, nrm);
    }
  };
  if (PE == E_F32) {
    for (int64_t it = 0; it < nit; ++it) {
      XT xv[64];
      load_x(it, xv);
      tile(it, xv);
    }
  } else {
    // two tiles per round, each tile's X requested a tile ahead of its use
    XT xa[64], xb[64];
    load_x(0, xa);
    for (int64_t it = 0; it < nit; it += 2) {
      load_x(it + 1 < nit ? it + 1 : nit - 1, xb);
      tile(it, xa);
      load_x(it + 2 < nit ? it + 2 : nit - 1, xa);
      tile(it + 1, xb);
    }
  }
  res = warp_sum(res);
  nrm = warp_sum(nrm);
  if (lane == 0) {
    red[0][wave] = res;
    red[1][wave] = nrm;
  }
  __syncthreads();
  if (tid == 0) {
    a.partial[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    a.partial[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// U (given as Ut, R x I float32) -> Up (I x 64, zero-padded columns): float32,
// or split bfloat16 (hi = rounded value, lo = rounded remainder, the lo block
// after the hi block)
template <class T>
__global__ void pad_u_kernel(const float* Ut, int64_t R, int64_t I, T* Up) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < I * 64;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e >> 6, k = e & 63;
    const float v = k < R ? Ut[k * I + i] : 0.f;
    if constexpr (sizeof(T) == 4) {
      Up[e] = v;
    } else {
      const bf16_t hi = f32_to_bf16(v);
      Up[e] = hi;
      Up[I * 64 + e] = f32_to_bf16(v - bf16_to_f32(hi));
    }
  }
}

template <class S, class D> __device__ inline D conv(S v);
template <> __device__ inline float conv<double, float>(double v) { return (float)v; }
template <> __device__ inline double conv<float, double>(float v) { return (double)v; }
template <> __device__ inline float conv<float, float>(float v) { return v; }
template <> __device__ inline double conv<double, double>(double v) { return v; }
template <> __device__ inline bf16_t conv<float, bf16_t>(float v) { return f32_to_bf16(v); }
template <> __device__ inline bf16_t conv<double, bf16_t>(double v) { return f32_to_bf16((float)v); }
template <> __device__ inline float conv<bf16_t, float>(bf16_t v) { return bf16_to_f32(v); }
template <> __device__ inline double conv<bf16_t, double>(bf16_t v) { return (double)bf16_to_f32(v); }
template <> __device__ inline bf16_t conv<bf16_t, bf16_t>(bf16_t v) { return v; }

template <class S, class D>
__global__ void convert_kernel(const S* src, D* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = conv<S, D>(src[i]);
}

// ------------------------------------------------------------------------
// First mode product of the precision forms from the mode's K-blocked copy
// (the Gram operand, [K tile][ipad rows][64 bytes], bfloat16 or block-scaled
// e4m3): Y[a, r, b] = sum_i U[i, r] X[a, i, b], R <= 64.  A workgroup owns 64
// padded columns (one e4m3 K tile or two bfloat16 ones) and all R rows of Y.
// The contraction over the ipad rows runs in chunks of 256: each chunk is
// decoded to bfloat16 and transposed into LDS as [column][row] (a thread
// decodes 8 rows x 8 columns and writes 8 16-byte column pieces).  Wave w
// takes positions 64 w .. 64 w + 63 of every chunk for the whole 64 x 64
// block (2 x 2 32x32x16 bfloat16 MFMA tiles, one row tile when R <= 32); the
// four partial blocks are added through LDS at the end of the block.  A
// workgroup takes a run of consecutive blocks and walks their chunks as one
// stream, so the loads run ahead across block ends and the next block's first
// chunks arrive while a block's partials are added.  The loads are ordered for the in-order retirement of
// vector loads: the chunk two steps ahead is in flight while a chunk is
// multiplied, and a wave's U pieces for the next step are loaded one step
// ahead into registers, so no MFMA waits on a load issued after an X load.
// U (bfloat16, zero past R and I) is stored in the order the waves read it:
// for chunk ch, wave w, k step s and row tile t, the 64 lanes' 8-value pieces
// are 1 KB contiguous, so a U load reads whole cache lines.
struct FirstArgs {
  const unsigned char* X;    // blocked copy
  const unsigned char* sc;   // e4m3 scales (the Gram operand's layout), or null
  const bf16_t* U;           // fragment order, 64 x ipad values
  float* Y;                  // [A][R][B]
  int64_t ipad, Bp, B, IN, INp;
  int64_t nblk;              // 64-column blocks
  int bpw;                   // consecutive blocks per workgroup
  int R;
};

constexpr int F_CH = 256;                    // rows per chunk
constexpr int F_ROW = F_CH * 2 + 16;         // LDS bytes per column row (padded)
constexpr int F_PART = 65;                   // floats per row of a partial block in LDS
constexpr int FIRST_RUN = 4;                 // 64-column blocks per workgroup
static_assert(4 * 64 * F_PART * 4 <= 2 * 64 * F_ROW, "the partial blocks reuse the chunk buffers");

// two floats -> packed bfloat16 (a in the low half), rounded to nearest even
__device__ inline uint32_t pack_bf16x2(float a, float b) {
  typedef __attribute__((ext_vector_type(2))) float f2v;
  typedef __attribute__((ext_vector_type(2))) __bf16 b2v;
  const b2v h = __builtin_convertvector((f2v){a, b}, b2v);
  return __builtin_bit_cast(uint32_t, h);
}

// one thread's share of a chunk: 8 rows x 16 bytes (bfloat16) or 8 bytes
// (e4m3, in .x .y) and, for e4m3, the 8 rows' scale bytes
struct FirstRaw {
  uint4 v[8];
  uint2 scl;
};

template <int E, bool TWO>
__global__ void __launch_bounds__(256, 2) ttm_first_kernel(FirstArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[2][64 * F_ROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // staging: thread (rl, cg) takes rows rl + 32 e (e = 0..7) of the chunk and
  // columns 8 cg .. 8 cg + 7.  Row rl + 32 e goes to chunk position 8 rl + e
  // (the contraction order inside a chunk is free; U is stored in the same
  // order), so a thread writes 8 consecutive positions of every column, and
  // its 8 e4m3 scales are 8 consecutive bytes of the scale layout.  rl runs
  // fastest over the lanes: the 8 lanes of a group write 8 consecutive 16-byte
  // pieces of one column row (distinct LDS banks), and a wave still loads 8
  // whole 64-byte rows.
  const int rl = (wave << 3) | (lane & 7), cg = lane >> 3;
  const int half = lane >> 5, lr = lane & 31;
  const int kw = wave * 64 + half * 8;             // this lane's first position in a chunk
  const int nch = (int)(a.ipad / F_CH);
  // this workgroup's stream: step s is chunk s % nch of block first + s / nch
  const int64_t first = (int64_t)blockIdx.x * a.bpw;
  const int nmine = (int)std::min<int64_t>(a.bpw, a.nblk - first);
  const int S = nmine * nch;
  if (S <= 0) return;
  auto block_of = [&](int s) { return first + s / nch; };

  auto load_x = [&](int s, FirstRaw& x) {
    const int64_t blk = block_of(s);
    const int ch = s % nch;
    const int64_t row0 = (int64_t)ch * F_CH;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t i = row0 + rl + 32 * e;
      if (E == E_FP8) {
        const uint2 v = *(const uint2*)(a.X + (blk * a.ipad + i) * 64 + cg * 8);
        x.v[e] = make_uint4(v.x, v.y, 0u, 0u);
      } else {
        const int64_t kt = blk * 2 + (cg >> 2);
        x.v[e] = *(const uint4*)(a.X + (kt * a.ipad + i) * 64 + (cg & 3) * 16);
      }
    }
    if (E == E_FP8) {
      // scale byte e of row rl + 32 e: [K tile][256-row tile][half][row % 32][row / 32]
      const int64_t tile = (blk * a.ipad + row0) >> 8;
      x.scl = *(const uint2*)(a.sc + (tile * 2 + (cg >> 2)) * 256 + rl * 8);
    }
  };
  // U pieces of a chunk: [k step][row tile] (rows lr and 32 + lr, positions
  // kw + 16 s .. + 7)
  auto load_u = [&](int ch, bf16x8_t (&u)[4][2]) {
    const bf16_t* p = a.U + ((int64_t)ch * 4 + wave) * 4096 + lane * 8;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      u[s][0] = *(const bf16x8_t*)(p + s * 1024);
      if (TWO) u[s][1] = *(const bf16x8_t*)(p + s * 1024 + 512);
    }
  };
  // decode and write the transposed pieces: column 8 cg + c, positions 8 rl .. 8 rl + 7
  // (dword j of a piece: positions 2 j and 2 j + 1, the even one in the low half)
  auto store = [&](char* buf, const FirstRaw& x) {
    uint32_t o[8][4];                              // [column][position pair]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e0 = 2 * j, e1 = 2 * j + 1;
      if (E == E_FP8) {
        // the scaled conversion gives code * 2^(byte - 127) exactly (a zero
        // byte is 2^-127); the products are e4m3 values times powers of two,
        // exact in bf16 except below bf16's subnormal range (runs of scale
        // byte 0, which hold zeros), so the packing rounds nothing else
        const uint32_t sw = j < 2 ? x.scl.x : x.scl.y;
        const float s0 = __uint_as_float(((sw >> (16 * (j & 1))) & 0xFFu) << 23);
        const float s1 = __uint_as_float(((sw >> (16 * (j & 1) + 8)) & 0xFFu) << 23);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const f32x2_t f0 = (p & 1) ? __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)(p < 2 ? x.v[e0].x : x.v[e0].y), s0, true)
                                     : __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)(p < 2 ? x.v[e0].x : x.v[e0].y), s0, false);
          const f32x2_t f1 = (p & 1) ? __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)(p < 2 ? x.v[e1].x : x.v[e1].y), s1, true)
                                     : __builtin_amdgcn_cvt_scalef32_pk_f32_fp8((int)(p < 2 ? x.v[e1].x : x.v[e1].y), s1, false);
          o[2 * p][j] = pack_bf16x2(f0.x, f1.x);
          o[2 * p + 1][j] = pack_bf16x2(f0.y, f1.y);
        }
      } else {
        const uint32_t wa[4] = {x.v[e0].x, x.v[e0].y, x.v[e0].z, x.v[e0].w};
        const uint32_t wb[4] = {x.v[e1].x, x.v[e1].y, x.v[e1].z, x.v[e1].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          o[2 * q][j] = (wa[q] & 0xFFFFu) | (wb[q] << 16);
          o[2 * q + 1][j] = (wa[q] >> 16) | (wb[q] & 0xFFFF0000u);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
      *(uint4*)(buf + (cg * 8 + c) * F_ROW + rl * 16) = make_uint4(o[c][0], o[c][1], o[c][2], o[c][3]);
  };

  f32x16_t acc[2][2];                              // [row tile][column tile]
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[t][c][v] = 0.f;
  auto mma = [&](const char* buf, const bf16x8_t (&u)[4][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = kw + 16 * s;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const bf16x8_t bv = *(const bf16x8_t*)(buf + (c * 32 + lr) * F_ROW + k * 2);
        acc[0][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(u[s][0], bv, acc[0][c], 0, 0, 0);
        if (TWO) acc[1][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(u[s][1], bv, acc[1][c], 0, 0, 0);
      }
    }
  };
  // the sum of the four waves' partial blocks of block blk -> Y (the chunk
  // buffers are free when it starts; it ends with the block's partials read)
  auto finish = [&](int64_t blk) {
    // partial blocks [wave][row][column]; value v of lane l: row
    // 8 (v / 4) + 4 (l / 32) + v % 4 of the tile, column l % 32
    float* part = (float*)&lds[0][0];
#pragma unroll
    for (int t = 0; t < (TWO ? 2 : 1); ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int r = t * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
          part[(wave * 64 + r) * F_PART + c * 32 + lr] = acc[t][c][v];
          acc[t][c][v] = 0.f;
        }
    __syncthreads();
    const int col = tid & 63;
    const int64_t g0 = blk * 64;                   // first padded column (over all a)
    const int64_t av_ = g0 / a.Bp, bp0 = g0 - av_ * a.Bp;
    const int64_t bp = bp0 + col;
    const int64_t hi = bp / a.INp, lo = bp - hi * a.INp;
    if (lo < a.IN) {
      float* out = a.Y + av_ * a.R * a.B + hi * a.IN + lo;
#pragma unroll
      for (int j = 0; j < (TWO ? 16 : 8); ++j) {
        const int r = (tid >> 6) + 4 * j;
        if (r < a.R) {
          float sum = 0.f;
#pragma unroll
          for (int w = 0; w < 4; ++w) sum += part[(w * 64 + r) * F_PART + col];
          out[(int64_t)r * a.B] = sum;
        }
      }
    }
    __syncthreads();
  };
  // stream step s: issue U of step s + 1 then X of step s + 2, multiply step
  // s's chunk, then write step s + 1's chunk (loaded one step earlier) to the
  // other LDS buffer; at a block's last chunk its partials are added first.
  // The loads are unconditional (a step past the end is clamped to the last
  // one, an L2 hit) so that the wait before each MFMA counts only the loads
  // issued after its operand's.
  auto step = [&](int s, const bf16x8_t (&ucur)[4][2], bf16x8_t (&unext)[4][2], const FirstRaw& have,
                  FirstRaw& next) {
    const int ch = s % nch;
    const bool last = ch + 1 == nch;
    load_u(last ? 0 : ch + 1, unext);
    load_x(min(s + 2, S - 1), next);
    mma(lds[s & 1], ucur);
    if (last) {
      __syncthreads();
      finish(block_of(s));
    }
    if (s + 1 < S) store(lds[(s + 1) & 1], have);
    __syncthreads();
  };

  FirstRaw x0, x1;
  bf16x8_t u0[4][2], u1[4][2];
  load_u(0, u0);
  load_x(0, x0);
  load_x(min(1, S - 1), x1);
  store(lds[0], x0);
  __syncthreads();
  int s = 0;
  for (; s + 1 < S; s += 2) {
    step(s, u0, u1, x1, x0);
    step(s + 1, u1, u0, x0, x1);
  }
  if (s < S) step(s, u0, u1, x1, x0);             // odd length: the last step
}

// U (given as Ut, R x I float64) -> bfloat16 in ttm_first_kernel's read
// order: element 8 (64 (2 (4 (4 ch + w) + s) + t) + l) + e is row
// 32 t + l % 32 at chunk position 64 w + 16 s + 8 (l / 32) + e, and position
// 8 q + e' of a 256-row chunk holds row q + 32 e' of U; zero past R and I
__global__ void u_first_kernel(const double* Ut, int64_t R, int64_t I, int64_t ipad, bf16_t* U) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < 64 * ipad;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(idx & 7), l = (int)((idx >> 3) & 63), t = (int)((idx >> 9) & 1);
    const int s = (int)((idx >> 10) & 3), w = (int)((idx >> 12) & 3);
    const int64_t ch = idx >> 14;
    const int64_t r = 32 * t + (l & 31);
    const int pc = 64 * w + 16 * s + 8 * (l >> 5) + e;     // position in the chunk
    const int64_t i = ch * F_CH + (pc >> 3) + 32 * (pc & 7);
    U[idx] = (r < R && i < I) ? f32_to_bf16((float)Ut[r * I + i]) : (bf16_t)0;
  }
}

// Last-mode product with a short output and a long contraction, float32:
// Y (A x R) = X (A x I) U (I x R) for R <= 64, U given as Ut (R x I).  The
// generic tile has one workgroup per 128 x 128 output block, so A = 2500,
// R = 50, I = 1000 ran on 20 workgroups with a serial loop over I.  Here a
// workgroup owns 32 rows of X, its four waves split the contraction into
// four ranges, and each wave forms the 32 x 64 block of its range on
// 32x32x2 float32 MFMA; the partial blocks are added through LDS in a fixed
// order.  Within a run of 8 contraction indices kb.., lane half h supplies
// the indices kb + 4 h + t at step t (t = 0..3), so each lane reads 4
// consecutive values of its X row and of its Ut row (16 bytes when I is a
// multiple of 4); both operands come straight from memory.
constexpr int LM_ROWS = 32;
struct LastArgs {
  const float* X;       // A x I row-major
  const float* Ut;      // R x I row-major
  float* Y;             // A x R row-major
  int64_t A, I;
  int R;
  int64_t krange;       // contraction indices per wave, a multiple of 8
};

template <bool VEC>
__global__ void __launch_bounds__(256) lastmode_small_kernel(LastArgs a) {
  __shared__ float part[4][LM_ROWS][65];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, lr = lane & 31;
  const int64_t a0 = (int64_t)blockIdx.x * LM_ROWS;
  const int64_t arow = a0 + lr < a.A ? a0 + lr : a.A - 1;       // clamped; rows past A are not stored
  const float* xr = a.X + arow * a.I;
  const float* ur[2];
  bool uok[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int r = c * 32 + lr;
    uok[c] = r < a.R;
    ur[c] = a.Ut + (int64_t)(uok[c] ? r : 0) * a.I;
  }
  const int64_t k0 = (int64_t)wave * a.krange;
  const int64_t k1 = std::min<int64_t>(k0 + a.krange, a.I);
  f32x16_t acc[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
  auto load4 = [&](const float* row, int64_t k, bool ok) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (VEC) {
      if (ok && k < k1) v = *(const float4*)(row + k);
    } else if (ok) {
      if (k < k1) v.x = row[k];
      if (k + 1 < k1) v.y = row[k + 1];
      if (k + 2 < k1) v.z = row[k + 2];
      if (k + 3 < k1) v.w = row[k + 3];
    }
    return v;
  };
  for (int64_t kb = k0; kb < k1; kb += 8) {
    const int64_t k = kb + 4 * half;
    const float4 xv = load4(xr, k, true);
    const float4 u0 = load4(ur[0], k, uok[0]);
    const float4 u1 = load4(ur[1], k, uok[1]);
    const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
    const float us0[4] = {u0.x, u0.y, u0.z, u0.w}, us1[4] = {u1.x, u1.y, u1.z, u1.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[t], us0[t], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[t], us1[t], acc[1], 0, 0, 0);
    }
  }
  // value v of lane l: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32 of the tile
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) part[wave][8 * (v >> 2) + 4 * half + (v & 3)][c * 32 + lr] = acc[c][v];
  __syncthreads();
  const int col = tid & 63;
  if (col < a.R) {
#pragma unroll
    for (int j = 0; j < LM_ROWS / 4; ++j) {
      const int row = (tid >> 6) + 4 * j;
      if (a0 + row < a.A)
        a.Y[(a0 + row) * a.R + col] = (part[0][row][col] + part[1][row][col]) + (part[2][row][col] + part[3][row][col]);
    }
  }
}

// Last-mode product with a short contraction and a wide output, float32:
// Y (A x R) = X (A x I) U (I x R) for I <= 64, U given as Ut (R x I) (the
// expansion G x_N U^(N) of the reconstruction, 50000 x 50 times 50 x 1000 at
// 1000^3, which the generic tile ran at a fifth of the write rate).  A
// workgroup owns 64 rows of X and 128 columns of Y: its X rows and Ut rows
// are each one contiguous run of memory, copied to LDS with coalesced loads;
// wave w forms the 32 x 64 block at rows 32 (w / 2), columns 64 (w % 2) on
// 32x32x2 float32 MFMA over the whole contraction (lane half h supplies the
// indices kb + 4 h + t at step t, as in lastmode_small_kernel).
constexpr int EX_ROWS = 64;
constexpr int EX_COLS = 128;
struct ExpArgs {
  const float* X;       // A x I row-major
  const float* Ut;      // R x I row-major
  float* Y;             // A x R row-major
  int64_t A, R;
  int I;                // <= 64
};

__global__ void __launch_bounds__(256) expand_small_kernel(ExpArgs a) {
  __shared__ __attribute__((aligned(16))) float xs[EX_ROWS * 64];
  __shared__ __attribute__((aligned(16))) float us[EX_COLS * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, lr = lane & 31;
  // consecutive workgroups take the column blocks of the same rows, so they
  // write whole output rows together
  const int64_t c0 = (int64_t)blockIdx.x * EX_COLS, a0 = (int64_t)blockIdx.y * EX_ROWS;
  const int I = a.I;
  // the runs: rows a0.. of X and c0.. of Ut, I values each (packed in LDS
  // with the same row length I)
  auto copy = [&](const float* src, int64_t n, float* dst) {
    if (((uintptr_t)src & 15) == 0) {
      const int64_t n4 = n >> 2;
      for (int64_t q = tid; q < n4; q += 256) *(float4*)(dst + 4 * q) = *(const float4*)(src + 4 * q);
      for (int64_t q = 4 * n4 + tid; q < n; q += 256) dst[q] = src[q];
    } else {
      for (int64_t q = tid; q < n; q += 256) dst[q] = src[q];
    }
  };
  copy(a.X + a0 * I, std::min<int64_t>(EX_ROWS, a.A - a0) * I, xs);
  copy(a.Ut + c0 * I, std::min<int64_t>(EX_COLS, a.R - c0) * I, us);
  __syncthreads();
  // rows past A and columns past R read stale LDS values: their outputs are
  // not stored, and the contraction past I is masked
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 64;
  const float* xr = xs + (wr + lr) * I;
  const float* u0r = us + (wc + lr) * I;
  const float* u1r = us + (wc + 32 + lr) * I;
  f32x16_t acc[2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
  const int nk = (I + 7) / 8;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j < nk) {
      float xv[4], u0[4], u1[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 8 * j + 4 * half + t;
        const bool ok = k < I;
        const int kc = ok ? k : 0;
        xv[t] = ok ? xr[kc] : 0.f;
        u0[t] = ok ? u0r[kc] : 0.f;
        u1[t] = ok ? u1r[kc] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[t], u0[t], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[t], u1[t], acc[1], 0, 0, 0);
      }
    }
  }
  // value v of lane l: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32 of the tile
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int64_t col = c0 + wc + c * 32 + lr;
    if (col >= a.R) continue;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = a0 + wr + 8 * (v >> 2) + 4 * half + (v & 3);
      if (row < a.A) a.Y[row * a.R + col] = acc[c][v];
    }
  }
}

template <int E, int EPI, class XT>
hipError_t launch_prod(const ProdArgs& p, int64_t batches, hipStream_t s) {
  // the batch index runs on grid.y (at most 65535 per launch)
  typedef typename Mma<E>::T T;
  typedef typename Mma<E>::Out Out;
  for (int64_t b0 = 0; b0 < batches; b0 += 65535) {
    const int64_t nb = std::min<int64_t>(65535, batches - b0);
    ProdArgs q = p;
    q.a.base = (const T*)p.a.base + b0 * p.a.batch_stride;
    q.b.base = (const T*)p.b.base + b0 * p.b.batch_stride;
    if (EPI == 0) q.out = (Out*)p.out + b0 * p.out_bs;
    dim3 grid((unsigned)(p.row_tiles * p.col_tiles), (unsigned)nb);
    if (p.vec_a && p.vec_b) hipLaunchKernelGGL((prod_kernel<E, EPI, XT, true>), grid, dim3(256), 0, s, q);
    else hipLaunchKernelGGL((prod_kernel<E, EPI, XT, false>), grid, dim3(256), 0, s, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

size_t ttm_work_bytes(int, int64_t, int64_t, int64_t, int64_t) { return 0; }

hipError_t launch_ttm(int elem, const void* X, int64_t A, int64_t I, int64_t B, const void* Ut, int64_t R,
                      void* Y, void*, size_t, hipStream_t s) {
  const int es = elem_size(elem);
  ProdArgs p = {};
  p.K = I;
  int64_t batches;
  if (B > 1) {
    // Y[a] (R x B) = Ut (R x I) . X[a] (I x B): rows r, cols b
    p.a = {Ut, I, 1, 0, R};
    p.b = {X, 1, B, I * B, B};
    p.out = Y;
    p.out_rs = B;
    p.out_cs = 1;
    p.out_bs = R * B;
    p.row_tiles = ceil_div(R, TILE);
    p.col_tiles = ceil_div(B, TILE);
    p.vec_a = (I * es) % 16 == 0 && aligned16(Ut);
    p.vec_b = (B * es) % 16 == 0 && aligned16(X);
    batches = A;
  } else {
    if (elem == E_F32 && R <= 64 && I >= 256) {
      // long contraction, short output: waves split the contraction
      LastArgs la;
      la.X = (const float*)X;
      la.Ut = (const float*)Ut;
      la.Y = (float*)Y;
      la.A = A;
      la.I = I;
      la.R = (int)R;
      la.krange = ceil_div(ceil_div(I, 4), 8) * 8;
      const int64_t wgs = ceil_div(A, LM_ROWS);
      if (wgs > 0x7fffffff) return hipErrorInvalidValue;
      const bool vec = I % 4 == 0 && aligned16(X) && aligned16(Ut);
      if (vec) hipLaunchKernelGGL(lastmode_small_kernel<true>, dim3((unsigned)wgs), dim3(256), 0, s, la);
      else hipLaunchKernelGGL(lastmode_small_kernel<false>, dim3((unsigned)wgs), dim3(256), 0, s, la);
      return hipGetLastError();
    }
    if (elem == E_F32 && I <= 64 && R > 64) {
      // short contraction, wide output
      ExpArgs ea;
      ea.X = (const float*)X;
      ea.Ut = (const float*)Ut;
      ea.Y = (float*)Y;
      ea.A = A;
      ea.R = R;
      ea.I = (int)I;
      const int64_t gx = ceil_div(R, EX_COLS), gy = ceil_div(A, EX_ROWS);
      if (gx > 0x7fffffff || gy > 65535) return hipErrorInvalidValue;
      hipLaunchKernelGGL(expand_small_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, ea);
      return hipGetLastError();
    }
    // Y (A x R) = X (A x I) . U (I x R): rows a, cols r
    p.a = {X, I, 1, 0, A};
    p.b = {Ut, I, 1, 0, R};
    p.out = Y;
    p.out_rs = R;
    p.out_cs = 1;
    p.out_bs = 0;
    p.row_tiles = ceil_div(A, TILE);
    p.col_tiles = ceil_div(R, TILE);
    p.vec_a = (I * es) % 16 == 0 && aligned16(X);
    p.vec_b = (I * es) % 16 == 0 && aligned16(Ut);
    batches = 1;
  }
  switch (elem) {
    case E_F64: return launch_prod<E_F64, 0, double>(p, batches, s);
    case E_F32: return launch_prod<E_F32, 0, float>(p, batches, s);
    case E_BF16: return launch_prod<E_BF16, 0, float>(p, batches, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ttm_padded(const void* Xpad, int64_t A, int64_t I, int64_t B, int64_t IN, const void* Ut,
                             int64_t R, void* Y, hipStream_t s) {
  const int64_t INp = pad64(IN);
  ProdArgs p = {};
  p.K = I;
  int64_t batches;
  if (B > 1) {
    // Y[a] (R x B) = Ut (R x I) . Xpad[a] (I x Bp): rows r, padded columns mapped back
    const int64_t Bp = (B / IN) * INp;
    p.a = {Ut, I, 1, 0, R};
    p.b = {Xpad, 1, Bp, I * Bp, Bp};
    p.out = Y;
    p.out_rs = B;
    p.out_cs = 1;
    p.out_bs = R * B;
    p.out_in = IN;
    p.out_inp = INp;
    p.row_tiles = ceil_div(R, TILE);
    p.col_tiles = ceil_div(Bp, TILE);
    p.vec_a = (I * 2) % 16 == 0 && aligned16(Ut);
    p.vec_b = aligned16(Xpad);
    batches = A;
  } else {
    // last mode: Y (A x R) = Xpad (A x I, row pitch I_Npad) . U (I x R)
    p.a = {Xpad, INp, 1, 0, A};
    p.b = {Ut, I, 1, 0, R};
    p.out = Y;
    p.out_rs = R;
    p.out_cs = 1;
    p.out_bs = 0;
    p.row_tiles = ceil_div(A, TILE);
    p.col_tiles = ceil_div(R, TILE);
    p.vec_a = (I * 2) % 16 == 0 && aligned16(Xpad);
    p.vec_b = (I * 2) % 16 == 0 && aligned16(Ut);
    batches = 1;
  }
  return launch_prod<E_BF16, 0, float>(p, batches, s);
}

hipError_t launch_ttm_first_blocked(int elem, const void* xb, const void* scales, int64_t A, int64_t I,
                                    int64_t B, int64_t IN, const double* Ut, int64_t R, void* U16, void* Y,
                                    hipStream_t s) {
  if (R < 1 || R > 64 || (elem != E_FP8 && elem != E_BF16)) return hipErrorInvalidValue;
  const int64_t INp = pad64(IN), ipad = block_rows(I);
  const int64_t Bp = (B / IN) * INp;
  hipLaunchKernelGGL(u_first_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(64 * ipad, 256), 2048)), dim3(256), 0,
                     s, Ut, R, I, ipad, (bf16_t*)U16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FirstArgs fa;
  fa.X = (const unsigned char*)xb;
  fa.sc = (const unsigned char*)scales;
  fa.U = (const bf16_t*)U16;
  fa.Y = (float*)Y;
  fa.ipad = ipad;
  fa.Bp = Bp;
  fa.B = B;
  fa.IN = IN;
  fa.INp = INp;
  fa.R = (int)R;
  const int64_t blocks = A * Bp / 64;
  fa.nblk = blocks;
  if (blocks < 1) return hipSuccess;
  // runs of FIRST_RUN blocks: long enough to amortise a workgroup's start
  // (its first loads and LDS fill), short enough that the dispatcher balances
  // the grid against kernels running beside it
  fa.bpw = FIRST_RUN;
  const int64_t wgs = ceil_div(blocks, (int64_t)FIRST_RUN);
  if (wgs > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)wgs), block(256);
  if (elem == E_FP8) {
    if (R > 32) hipLaunchKernelGGL((ttm_first_kernel<E_FP8, true>), grid, block, 0, s, fa);
    else hipLaunchKernelGGL((ttm_first_kernel<E_FP8, false>), grid, block, 0, s, fa);
  } else {
    if (R > 32) hipLaunchKernelGGL((ttm_first_kernel<E_BF16, true>), grid, block, 0, s, fa);
    else hipLaunchKernelGGL((ttm_first_kernel<E_BF16, false>), grid, block, 0, s, fa);
  }
  return hipGetLastError();
}

size_t residual_work_bytes(int64_t I, int64_t J) {
  const int64_t tiles = std::max<int64_t>(ceil_div(I, TILE) * ceil_div(J, TILE), ceil_div(J, RS_COLS));
  return (size_t)tiles * 16 + 256 + (size_t)I * 64 * 4 + 64;
}

hipError_t launch_residual(int x_elem, const void* X, int op_elem, const void* Ut, const void* H, int64_t I,
                           int64_t J, int64_t R, double* out, void* work, size_t, hipStream_t s, bool bf16_products) {
  const int64_t tiles = std::max<int64_t>(ceil_div(I, TILE) * ceil_div(J, TILE), ceil_div(J, RS_COLS));
  double* partial = (double*)work;
  if (op_elem == E_F32 && R <= 64 && (x_elem == E_F32 || x_elem == E_BF16) && J % 4 == 0 && aligned16(H) &&
      ceil_div(J, TILE) <= 0x7fffffff) {
    // streaming form
    void* Up = (char*)work + ((tiles * 16 + 255) / 256) * 256;
    const dim3 pgrid((unsigned)std::min<int64_t>(ceil_div(I * 64, 256), 4096));
    if (bf16_products) hipLaunchKernelGGL(pad_u_kernel<bf16_t>, pgrid, dim3(256), 0, s, (const float*)Ut, R, I, (bf16_t*)Up);
    else hipLaunchKernelGGL(pad_u_kernel<float>, pgrid, dim3(256), 0, s, (const float*)Ut, R, I, (float*)Up);
    ResArgs ra;
    ra.Up = Up;
    ra.H = (const float*)H;
    ra.X = X;
    ra.I = I;
    ra.J = J;
    ra.R = (int)R;
    ra.nkt = (int)ceil_div(R, 32);
    ra.partial = partial;
    dim3 grid((unsigned)ceil_div(J, TILE));
    if (bf16_products) {
      ResSplitArgs rs;
      rs.Uh = (const bf16_t*)Up;
      rs.Ul = (const bf16_t*)Up + I * 64;
      rs.H = (const float*)H;
      rs.X = X;
      rs.I = I;
      rs.J = J;
      rs.R = (int)R;
      rs.partial = partial;
      grid = dim3((unsigned)ceil_div(J, RS_COLS));
      // VEC: every row starts on a 4-value boundary, so a lane's 4 values are one load
      const bool vec = J % 4 == 0 && aligned16(X);
      if (x_elem == E_F32) {
        if (vec) hipLaunchKernelGGL((residual_split_kernel<float, true>), grid, dim3(256), 0, s, rs);
        else hipLaunchKernelGGL((residual_split_kernel<float, false>), grid, dim3(256), 0, s, rs);
      } else {
        if (vec) hipLaunchKernelGGL((residual_split_kernel<bf16_t, true>), grid, dim3(256), 0, s, rs);
        else hipLaunchKernelGGL((residual_split_kernel<bf16_t, false>), grid, dim3(256), 0, s, rs);
      }
    } else {
      if (x_elem == E_F32) hipLaunchKernelGGL((residual_kernel<float, E_F32>), grid, dim3(256), 0, s, ra);
      else hipLaunchKernelGGL((residual_kernel<bf16_t, E_F32>), grid, dim3(256), 0, s, ra);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(1024), 0, s, (const double*)partial, (int64_t)grid.x, out);
    return hipGetLastError();
  }
  const int es = elem_size(op_elem);
  ProdArgs p = {};
  p.K = R;
  // Xhat[i, j] = sum_r U[i, r] H[r, j]: rows i from Ut (R x I, row-contiguous),
  // cols j from H (R x J, row-contiguous)
  p.a = {Ut, 1, I, 0, I};
  p.b = {H, 1, J, 0, J};
  p.row_tiles = ceil_div(I, TILE);
  p.col_tiles = ceil_div(J, TILE);
  p.vec_a = (I * es) % 16 == 0 && aligned16(Ut);
  p.vec_b = (J * es) % 16 == 0 && aligned16(H);
  p.X = X;
  p.x_elem = x_elem;
  p.xJ = J;
  p.partial = partial;
  hipError_t e;
  if (op_elem == E_F64) {
    if (x_elem != E_F64) return hipErrorInvalidValue;
    e = launch_prod<E_F64, 1, double>(p, 1, s);
  } else if (op_elem == E_F32) {
    if (x_elem == E_F32) e = launch_prod<E_F32, 1, float>(p, 1, s);
    else if (x_elem == E_BF16) e = launch_prod<E_F32, 1, bf16_t>(p, 1, s);
    else e = launch_prod<E_F32, 1, double>(p, 1, s);
  } else if (op_elem == E_BF16) {
    if (x_elem == E_F32) e = launch_prod<E_BF16, 1, float>(p, 1, s);
    else if (x_elem == E_BF16) e = launch_prod<E_BF16, 1, bf16_t>(p, 1, s);
    else e = launch_prod<E_BF16, 1, double>(p, 1, s);
  } else {
    return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int64_t n = p.row_tiles * p.col_tiles;
  hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(1024), 0, s, (const double*)partial, n, out);
  return hipGetLastError();
}

hipError_t convert_tensor(int src_elem, const void* src, int dst_elem, void* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 65536);
#define CV(SE, ST, DE, DT)                                                                                    \
  if (src_elem == SE && dst_elem == DE) {                                                                     \
    hipLaunchKernelGGL((convert_kernel<ST, DT>), dim3(grid), dim3(256), 0, s, (const ST*)src, (DT*)dst, n); \
    return hipGetLastError();                                                                                 \
  }
  CV(E_F64, double, E_F32, float)
  CV(E_F32, float, E_F64, double)
  CV(E_F32, float, E_F32, float)
  CV(E_F64, double, E_F64, double)
  CV(E_F32, float, E_BF16, bf16_t)
  CV(E_F64, double, E_BF16, bf16_t)
  CV(E_BF16, bf16_t, E_F32, float)
  CV(E_BF16, bf16_t, E_F64, double)
  CV(E_BF16, bf16_t, E_BF16, bf16_t)
#undef CV
  return hipErrorInvalidValue;
}

}  // namespace rbki
