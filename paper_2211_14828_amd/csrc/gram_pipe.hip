// bf16 Gram + sketch products of one mode (Remark 1: C = X_(n) X_(n)^T; Alg. 1,
// step 2: W = X_(n) Omega^(n)), streamed through LDS by direct global->LDS
// loads in a four-stage ring.
//
// Operands.  The products read zero-padded bf16 copies of the tensor, built
// once per decomposition:
//   * Xpad: X viewed as (T / I_N) rows of its last dimension I_N, each row
//     padded with zeros to I_Npad (a multiple of 64).  Mode n < N-1 reads it
//     as [A_n, I_n, Bp_n] with Bp_n = (B_n / I_N) I_Npad: row (a, i) is
//     contiguous, and the padding adds zero columns to X_(n), which change
//     neither C nor W.
//   * Xt: the last mode, X_(N) stored as I_N rows of A_pad = (T / I_N)
//     rounded up to a multiple of 64, zero-padded.
//   * Omega^T in the same padded column layout (zero in padded columns).
// Every K tile (32 columns) is therefore whole: no bounds checks, no masking.
// Rows past I_n (the last row tile) and sketch rows past S read a clamped,
// valid row; the outputs they produce are never reduced.
//
// Tiles.  A workgroup (4 waves) owns one 256 x 256 lower-triangle tile of C
// and a slice of the contraction (split-K).  Off-diagonal tiles give each
// wave a 128 x 128 block (4 x 4 MFMA 32x32x16 tiles).  In a diagonal tile the
// upper-right 128 x 128 block is the transpose of the lower-left one, so that
// wave computes the 256 x 64 sketch block W(rows, 0..63) instead (S <= 64).
// All tiles cost the same, and the number of splits is chosen so that tiles x
// splits fills whole rounds of the 256 compute units.
//
// Pipeline.  Stage s of the ring holds K tile kt (A rows and B rows, 64 bytes
// each) in its own LDS array.  While tile kt is multiplied, tiles kt+1..kt+3
// are in flight.  The loads go straight to LDS (no register staging); one
// barrier per K tile orders them.  Within a row the four 16-byte chunks are
// XOR-swizzled with bits 2..3 of the row index, so the 32 rows read by one
// MFMA operand load hit distinct LDS banks.
//
// Split-K partials (float32) are reduced in a fixed order in float64 by a
// second kernel: results are deterministic.
#include "rbki_kernels.h"
#include "rbki_mma.h"
#include "rbki_philox.h"

namespace rbki {

namespace {

typedef __attribute__((address_space(3))) void lds_void;

constexpr int PT = 256;          // tile rows
constexpr int PK = 32;           // k per stage
constexpr int PROW = 64;         // bytes per row per stage
constexpr int PSTAGE = PT * PROW;   // 16 KB per operand per stage
constexpr int PW = 64;           // sketch columns computed by the spare diagonal wave

__shared__ __attribute__((aligned(1024))) char pa0[PSTAGE];
__shared__ __attribute__((aligned(1024))) char pa1[PSTAGE];
__shared__ __attribute__((aligned(1024))) char pa2[PSTAGE];
__shared__ __attribute__((aligned(1024))) char pa3[PSTAGE];
__shared__ __attribute__((aligned(1024))) char pb0[PSTAGE];
__shared__ __attribute__((aligned(1024))) char pb1[PSTAGE];
__shared__ __attribute__((aligned(1024))) char pb2[PSTAGE];
__shared__ __attribute__((aligned(1024))) char pb3[PSTAGE];

template <int ST> __device__ inline char* stage_a() {
  if constexpr (ST == 0) return pa0;
  else if constexpr (ST == 1) return pa1;
  else if constexpr (ST == 2) return pa2;
  else return pa3;
}
template <int ST> __device__ inline char* stage_b() {
  if constexpr (ST == 0) return pb0;
  else if constexpr (ST == 1) return pb1;
  else if constexpr (ST == 2) return pb2;
  else return pb3;
}

// s_waitcnt with only the vector-memory counter constrained (<= n, n < 64).
template <int N> __device__ inline void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}
__device__ inline void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14)); }

// swizzled byte offset of logical 16-byte chunk c of row r in a stage
__device__ inline int swz(int r, int c) { return r * PROW + ((c ^ ((r >> 2) & 3)) << 4); }

struct PipeCtx {
  const bf16_t* X;        // padded operand view [A, I, Bp]
  const bf16_t* Om;       // padded Omega^T, S rows of Jp
  int64_t IBp, Bp;        // slab stride I * Bp, row pitch
  int64_t na, nk0;        // next K tile to load: slab a, first column k0
  int64_t left;           // K tiles of this split not yet loaded (the last one is reloaded after)
  int64_t offa[4], offb[4];   // per-lane element offsets of this lane's rows and chunks
  int wave;
};

// Advance the next K tile (a, k0) by one tile, holding at the split's last.
__device__ __attribute__((always_inline)) inline void advance(PipeCtx& c) {
  if (c.left > 1) {
    c.nk0 += PK;
    if (c.nk0 == c.Bp) { c.nk0 = 0; ++c.na; }
    --c.left;
  }
}

// Issue the loads of the next K tile into stage ST: A rows r0..r0+255 (4
// loads per wave), B rows c0..c0+255 (off-diagonal, 4 per wave) or sketch rows
// 0..63 (diagonal, 1 per wave).  Lane l of load q covers row 16 q + l / 4
// and the 16-byte chunk at position l % 4 of that row.
template <bool DIAG, int ST>
__device__ __attribute__((always_inline)) inline void issue(PipeCtx& c) {
  const bf16_t* xa = c.X + c.na * c.IBp + c.nk0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    __builtin_amdgcn_global_load_lds((const void*)(xa + c.offa[j]),
                                     (lds_void*)(stage_a<ST>() + (j * 4 + c.wave) * 1024), 16, 0, 0);
  if (DIAG) {
    __builtin_amdgcn_global_load_lds((const void*)(c.Om + c.na * c.Bp + c.nk0 + c.offb[0]),
                                     (lds_void*)(stage_b<ST>() + c.wave * 1024), 16, 0, 0);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(xa + c.offb[j]),
                                       (lds_void*)(stage_b<ST>() + (j * 4 + c.wave) * 1024), 16, 0, 0);
  }
  advance(c);
}

// Multiply the K tile held in stage ST (two MFMA K steps of 16).
//   C waves (WW false): acc[m][n] += A(ra + 32 m) . B(rb + 32 n)
//   sketch wave (WW true): acc[m][n] += A(128 (n / 2) + 32 m) . Omega(32 (n % 2))
template <bool DIAG, bool WW, int ST>
__device__ __attribute__((always_inline)) inline void compute(f32x16_t (&acc)[4][4], int lane, int ra, int rb) {
  const char* la = stage_a<ST>();
  const char* lb = (DIAG && !WW) ? stage_a<ST>() : stage_b<ST>();
  const int half = lane >> 5, lr = lane & 31;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int ch = 2 * t + half;
    if (WW) {
      bf16x8_t av[8], bv[2];
#pragma unroll
      for (int m = 0; m < 8; ++m) av[m] = *(const bf16x8_t*)(la + swz(m * 32 + lr, ch));
#pragma unroll
      for (int n = 0; n < 2; ++n) bv[n] = *(const bf16x8_t*)(lb + swz(n * 32 + lr, ch));
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m + 4 * (n >> 1)], bv[n & 1], acc[m][n], 0, 0, 0);
    } else {
      bf16x8_t av[4], bv[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        av[m] = *(const bf16x8_t*)(la + swz(ra + m * 32 + lr, ch));
        bv[m] = *(const bf16x8_t*)(lb + swz(rb + m * 32 + lr, ch));
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[m], bv[n], acc[m][n], 0, 0, 0);
    }
  }
}

// One K step of the ring: wait for stage ST, barrier, refill the stage that
// was read in the previous step, multiply stage ST if this step is real.
template <bool DIAG, bool WW, int ST>
__device__ __attribute__((always_inline)) inline void ring_step(PipeCtx& c, f32x16_t (&acc)[4][4], bool real,
                                                                int lane, int ra, int rb) {
  constexpr int PER = DIAG ? 5 : 8;          // loads per wave per stage
  wait_vm<2 * PER>();
  __builtin_amdgcn_s_barrier();
  issue<DIAG, (ST + 3) & 3>(c);
  if (real) compute<DIAG, WW, ST>(acc, lane, ra, rb);
  wait_lgkm0();
}

template <bool DIAG, bool WW>
__device__ __attribute__((always_inline)) inline void ring(PipeCtx& c, f32x16_t (&acc)[4][4], int64_t nk, int lane,
                                                           int ra, int rb) {
  issue<DIAG, 0>(c);
  issue<DIAG, 1>(c);
  issue<DIAG, 2>(c);
  for (int64_t k = 0; k < nk; k += 4) {
    ring_step<DIAG, WW, 0>(c, acc, true, lane, ra, rb);
    ring_step<DIAG, WW, 1>(c, acc, k + 1 < nk, lane, ra, rb);
    ring_step<DIAG, WW, 2>(c, acc, k + 2 < nk, lane, ra, rb);
    ring_step<DIAG, WW, 3>(c, acc, k + 3 < nk, lane, ra, rb);
  }
  // every load must have landed before the workgroup's LDS is released
  wait_vm<0>();
  __builtin_amdgcn_s_barrier();
}

template <bool DIAG>
__device__ __attribute__((always_inline)) inline void run_tile(const GramArgs& g, int split, int ti, int tj) {
  PipeCtx c;
  c.X = (const bf16_t*)g.X;
  c.Om = (const bf16_t*)g.omegaT;
  c.IBp = g.I * g.B;
  c.Bp = g.B;
  c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t kt0 = (int64_t)split * g.nkt / g.splits;
  const int64_t kt1 = (int64_t)(split + 1) * g.nkt / g.splits;     // kt1 > kt0 (splits <= nkt)
  c.na = kt0 / g.nbt;
  c.nk0 = (kt0 - c.na * g.nbt) * PK;
  c.left = kt1 - kt0;
  const int64_t r0 = (int64_t)ti * PT, c0 = (int64_t)tj * PT;
  {
    const int rl = lane >> 2, p = lane & 3;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = (j * 4 + c.wave) * 16 + rl;
      const int ch = p ^ ((row >> 2) & 3);
      int64_t ra_ = r0 + row, rb_ = c0 + row;
      ra_ = ra_ < g.I ? ra_ : g.I - 1;        // rows past I: a valid row, output discarded
      rb_ = rb_ < g.I ? rb_ : g.I - 1;
      c.offa[j] = ra_ * g.B + ch * 8;
      c.offb[j] = rb_ * g.B + ch * 8;
    }
    if (DIAG) {
      const int row = c.wave * 16 + rl;       // sketch row 0..63
      const int sr = row < g.S ? row : g.S - 1;
      c.offb[0] = (int64_t)sr * g.J + (p ^ ((row >> 2) & 3)) * 8;
    }
  }
  const bool wwave = DIAG && c.wave == 1;
  // C blocks: off-diagonal waves (w/2, w%2); diagonal waves 0, 2, 3 take
  // blocks (0,0), (1,0), (1,1)
  const int ra = DIAG ? (c.wave == 0 ? 0 : 128) : (c.wave >> 1) * 128;
  const int rb = DIAG ? (c.wave == 3 ? 128 : 0) : (c.wave & 1) * 128;

  f32x16_t acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[m][n][v] = 0.f;

  const int64_t nk = kt1 - kt0;
  if (DIAG) {
    if (wwave) ring<true, true>(c, acc, nk, lane, ra, rb);
    else ring<true, false>(c, acc, nk, lane, ra, rb);
  } else {
    ring<false, false>(c, acc, nk, lane, ra, rb);
  }

  const int half = lane >> 5, lr = lane & 31;
  if (wwave) {
    // sketch block: rows 0..255 of the tile, columns 0..63
    float* out = (float*)g.partial + (int64_t)split * g.part_stride + g.wpart_off + (int64_t)ti * PT * PW;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = (n >> 1) * 128 + m * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
          const int col = (n & 1) * 32 + lr;
          out[row * PW + col] = acc[m][n][v];
        }
  } else {
    const int tile = ti * (ti + 1) / 2 + tj;
    float* out = (float*)g.partial + (int64_t)split * g.part_stride + (int64_t)tile * PT * PT;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = ra + m * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
          const int col = rb + n * 32 + lr;
          out[row * PT + col] = acc[m][n][v];
        }
  }
}

__device__ inline void decode_tri(int tile, int& ti, int& tj) {
  int t = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
  while ((t + 1) * (t + 2) / 2 <= tile) ++t;
  while (t * (t + 1) / 2 > tile) --t;
  ti = t;
  tj = tile - t * (t + 1) / 2;
}

__global__ void __launch_bounds__(256, 1) gram_pipe_kernel(GramArgs g) {
  const int w = blockIdx.x;
  int split, tile;
  if (g.xcd_map) {
    // consecutive workgroups go to consecutive XCDs: keep the tiles of one
    // split (which share its K range) on one XCD
    const int xcd = w & 7, slot = w >> 3;
    split = xcd + 8 * (slot / g.ntiles);
    tile = slot % g.ntiles;
  } else {
    split = w / g.ntiles;
    tile = w % g.ntiles;
  }
  int ti, tj;
  decode_tri(tile, ti, tj);
  if (ti == tj) run_tile<true>(g, split, ti, tj);
  else run_tile<false>(g, split, ti, tj);
}

// C (I x I, both triangles) and W^T (S x I) from the partials, float64,
// summed over the splits in a fixed order.  Threads walk the partial layout
// (tile by tile, row-major inside a tile), so every split's reads are
// coalesced; each lower-triangle value is written to C(i, j) and C(j, i).
__global__ void gram_pipe_reduce_kernel(GramArgs g, double* C, double* Wt) {
  const int64_t nCp = (int64_t)g.ntri * PT * PT;
  const int64_t nWp = (int64_t)g.nt * PT * PW;
  const float* P = (const float*)g.partial;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nCp + nWp;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j, s = -1;
    if (e < nCp) {
      const int tile = (int)(e / (PT * PT));
      const int w = (int)(e - (int64_t)tile * PT * PT);
      int ti, tj;
      decode_tri(tile, ti, tj);
      i = (int64_t)ti * PT + (w >> 8);
      j = (int64_t)tj * PT + (w & (PT - 1));
      if (i >= g.I || j >= g.I || j > i) continue;   // padding rows, or the unused block of a diagonal tile
    } else {
      const int64_t f = e - nCp;
      const int64_t ti = f / (PT * PW);
      const int w = (int)(f - ti * PT * PW);
      i = ti * PT + w / PW;
      s = w % PW;
      if (i >= g.I || s >= g.S) continue;
      j = 0;
    }
    double acc = 0.0;
    const int64_t off = e < nCp ? e : g.wpart_off + (e - nCp);
    for (int sp = 0; sp < g.splits; ++sp) acc += (double)P[sp * g.part_stride + off];
    if (s < 0) {
      C[i * g.I + j] = acc;
      C[j * g.I + i] = acc;
    } else {
      Wt[s * g.I + i] = acc;
    }
  }
}

// Padded bf16 copies of X viewed as R rows of length L (R = T / I_N, L = I_N):
// Xpad (R x Lp) and Xt (L x Rp), zeros in the padding.  64 x 64 tiles through LDS.
template <class T>
__global__ void pad_copies_kernel(const T* X, int64_t R, int64_t L, bf16_t* Xpad, int64_t Lp, bf16_t* Xt,
                                  int64_t Rp) {
  __shared__ float tile[64][65];
  const int64_t tl = Lp / 64;
  const int64_t br = blockIdx.x / tl, bl = blockIdx.x - br * tl;
  const int64_t r0 = br * 64, l0 = bl * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int y = ty; y < 64; y += 4) {
    const int64_t r = r0 + y, l = l0 + tx;
    float v = 0.f;
    if (r < R && l < L) {
      if constexpr (sizeof(T) == 2) v = bf16_to_f32(((const bf16_t*)X)[r * L + l]);
      else v = (float)X[r * L + l];
    }
    tile[y][tx] = v;
    if (Xpad && r < R) Xpad[r * Lp + l] = f32_to_bf16(v);
  }
  if (!Xt) return;
  __syncthreads();
  for (int y = ty; y < 64; y += 4) {
    const int64_t l = l0 + y, r = r0 + tx;
    if (l < L) Xt[l * Rp + r] = f32_to_bf16(tile[tx][y]);
  }
}

// Omega^T (S x J) of one mode in the padded column layout (S x Jp): the
// value of stream index L = s J + j goes to column jp(j); padded columns
// must be zero beforehand.  B = 1: jp = j.  B > 1: j = a B + b with
// b = bh I_N + bl, jp = a Bp + bh I_Npad + bl.
__global__ void omega_pad_kernel(uint64_t seed, uint32_t mode, int64_t S, int64_t J, int64_t B, int64_t IN,
                                 int64_t INp, int64_t Jp, bf16_t* out) {
  const int64_t total = S * J;
  const int64_t npairs = (total + 1) / 2;
  const int64_t Bp = B > 1 ? (B / IN) * INp : 1;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < npairs;
       m += (int64_t)gridDim.x * blockDim.x) {
    float z[2];
    gauss_pair_f32((uint64_t)m, mode, 0u, seed, z[0], z[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t L = 2 * m + h;
      if (L >= total) break;
      const int64_t s = L / J, j = L - s * J;
      int64_t jp = j;
      if (B > 1) {
        const int64_t a = j / B, b = j - a * B;
        const int64_t bh = b / IN, bl = b - bh * IN;
        jp = a * Bp + bh * INp + bl;
      }
      out[s * Jp + jp] = f32_to_bf16(z[h]);
    }
  }
}

}  // namespace

int64_t pad64(int64_t v) { return (v + 63) / 64 * 64; }

GramArgs gram_plan_pipe(int64_t A, int64_t I, int64_t Bp, int S, int cu_count) {
  GramArgs g = {};
  g.A = A;
  g.I = I;
  g.B = Bp;
  g.J = A * Bp;
  g.S = S;
  g.nt = (int)ceil_div(I, PT);
  g.ntri = g.nt * (g.nt + 1) / 2;
  g.ntiles = g.ntri;
  g.nbt = Bp / PK;
  g.nkt = A * g.nbt;
  // splits: minimise rounds(tiles x splits over the CUs) x (K tiles per split
  // + a fixed cost of 8 tiles) + the partials each split adds to the
  // reduction (a 256 x 256 float tile costs about 0.12 K-tile times);
  // multiples of 8 keep the XCD mapping
  const int64_t cu = cu_count > 0 ? cu_count : 256;
  int64_t best = 1;
  double best_cost = 1e300;
  for (int64_t s = 1; s <= 512 && s <= g.nkt; ++s) {
    if (s > 8 && s % 8) continue;
    const int64_t rounds = ceil_div(g.ntiles * s, cu);
    const double cost = (double)rounds * ((double)g.nkt / (double)s + 8.0) + 0.12 * (double)(g.ntiles * s);
    if (cost < best_cost * 0.999) { best_cost = cost; best = s; }
  }
  g.splits = (int)best;
  g.xcd_map = (g.splits % 8 == 0) ? 1 : 0;
  g.wpart_off = (int64_t)g.ntri * PT * PT;
  g.part_stride = g.wpart_off + (int64_t)g.nt * PT * PW;
  return g;
}

size_t gram_pipe_partial_bytes(const GramArgs& g) { return (size_t)g.splits * g.part_stride * 4; }

bool gram_pipe_ok(int64_t I, int S) { return S >= 1 && S <= PW && I > 128; }

hipError_t launch_gram_pipe(const GramArgs& g, hipStream_t s) {
  if (g.nkt < 1 || g.splits > g.nkt || g.S > PW || g.B % PK) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gram_pipe_kernel, dim3((unsigned)(g.ntiles * g.splits)), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_gram_pipe_reduce(const GramArgs& g, double* C, double* Wt, hipStream_t s) {
  const int64_t total = (int64_t)g.ntri * PT * PT + (int64_t)g.nt * PT * PW;
  unsigned rgrid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096);
  hipLaunchKernelGGL(gram_pipe_reduce_kernel, dim3(rgrid), dim3(256), 0, s, g, C, Wt);
  return hipGetLastError();
}

hipError_t launch_pad_copies(int src_elem, const void* X, int64_t R, int64_t L, void* Xpad, void* Xt, hipStream_t s) {
  const int64_t Lp = pad64(L), Rp = pad64(R);
  const int64_t blocks = (Rp / 64) * (Lp / 64);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  switch (src_elem) {
    case E_F64:
      hipLaunchKernelGGL(pad_copies_kernel<double>, grid, dim3(256), 0, s, (const double*)X, R, L, (bf16_t*)Xpad, Lp,
                         (bf16_t*)Xt, Rp);
      break;
    case E_F32:
      hipLaunchKernelGGL(pad_copies_kernel<float>, grid, dim3(256), 0, s, (const float*)X, R, L, (bf16_t*)Xpad, Lp,
                         (bf16_t*)Xt, Rp);
      break;
    default:
      hipLaunchKernelGGL(pad_copies_kernel<bf16_t>, grid, dim3(256), 0, s, (const bf16_t*)X, R, L, (bf16_t*)Xpad, Lp,
                         (bf16_t*)Xt, Rp);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_omega_pad(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t Jp,
                            void* out, hipStream_t s) {
  hipError_t e = fill_zero(out, (size_t)S * Jp * 2, s);
  if (e != hipSuccess) return e;
  const int64_t npairs = (S * J + 1) / 2;
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(npairs, 256), 16384);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(omega_pad_kernel, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN, pad64(IN), Jp,
                     (bf16_t*)out);
  return hipGetLastError();
}

}  // namespace rbki
