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
// FP8 form.  The same kernel runs on e4m3 copies: a stage row then holds 64
// values, one MFMA K step of 64 (block-scaled 32x32x64 f8f6f4).  Every run
// of 32 values along a storage row has its own power-of-two (E8M0) scale,
// chosen so that the run's largest magnitude maps to at most 448.  For each
// mode the scales are gathered once into [K tile][row][2] order, so each
// wave fetches the scales of 128 rows for a stage with one more 4-byte
// direct-to-LDS load.
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

__shared__ __attribute__((aligned(16))) unsigned char psa0[512];
__shared__ __attribute__((aligned(16))) unsigned char psa1[512];
__shared__ __attribute__((aligned(16))) unsigned char psa2[512];
__shared__ __attribute__((aligned(16))) unsigned char psa3[512];
__shared__ __attribute__((aligned(16))) unsigned char psb0[512];
__shared__ __attribute__((aligned(16))) unsigned char psb1[512];
__shared__ __attribute__((aligned(16))) unsigned char psb2[512];
__shared__ __attribute__((aligned(16))) unsigned char psb3[512];

template <int ST> __device__ inline unsigned char* stage_sa() {
  if constexpr (ST == 0) return psa0;
  else if constexpr (ST == 1) return psa1;
  else if constexpr (ST == 2) return psa2;
  else return psa3;
}
template <int ST> __device__ inline unsigned char* stage_sb() {
  if constexpr (ST == 0) return psb0;
  else if constexpr (ST == 1) return psb1;
  else if constexpr (ST == 2) return psb2;
  else return psb3;
}

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
  const char* X;          // padded operand view [A, I, Bp] (bytes)
  const char* Om;         // padded Omega^T, S rows of Jp (bytes)
  int64_t IBp, Bp;        // slab stride I * Bp and row pitch, in elements
  int64_t na, nk0;        // next K tile to load: slab a, first column k0 (elements)
  int64_t left;           // K tiles of this split not yet loaded (the last one is reloaded after)
  int64_t kt;             // global index of the next K tile (scale lookup)
  int64_t offa[4], offb[4];   // per-lane byte offsets of this lane's rows and chunks
  const unsigned char* sc;    // fp8: this lane's scale source at K tile 0
  int64_t sc_step;            // fp8: bytes per K tile of that source
  int sc_dst;                 // fp8: 0..3 = A scales low/high half, B scales low/high half
  int wave;
};

template <int E> struct PipeElem {
  static constexpr int ES = E == E_FP8 ? 1 : 2;      // bytes per value
  static constexpr int KT = PROW / ES;               // values per stage row
};

// Advance the next K tile (a, k0) by one tile, holding at the split's last.
template <int E>
__device__ __attribute__((always_inline)) inline void advance(PipeCtx& c) {
  if (c.left > 1) {
    c.nk0 += PipeElem<E>::KT;
    if (c.nk0 == c.Bp) { c.nk0 = 0; ++c.na; }
    ++c.kt;
    --c.left;
  }
}

// Issue the loads of the next K tile into stage ST: A rows r0..r0+255 (4
// loads per wave), B rows c0..c0+255 (off-diagonal, 4 per wave) or sketch rows
// 0..63 (diagonal, 1 per wave), and for fp8 one load of scales per wave.
// Lane l of load q covers row 16 q + l / 4 and the 16-byte chunk at position
// l % 4 of that row.
template <int E, bool DIAG, int ST>
__device__ __attribute__((always_inline)) inline void issue(PipeCtx& c) {
  constexpr int ES = PipeElem<E>::ES;
  const char* xa = c.X + (c.na * c.IBp + c.nk0) * ES;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    __builtin_amdgcn_global_load_lds((const void*)(xa + c.offa[j]),
                                     (lds_void*)(stage_a<ST>() + (j * 4 + c.wave) * 1024), 16, 0, 0);
  if (DIAG) {
    __builtin_amdgcn_global_load_lds((const void*)(c.Om + (c.na * c.Bp + c.nk0) * ES + c.offb[0]),
                                     (lds_void*)(stage_b<ST>() + c.wave * 1024), 16, 0, 0);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(xa + c.offb[j]),
                                       (lds_void*)(stage_b<ST>() + (j * 4 + c.wave) * 1024), 16, 0, 0);
  }
  if (E == E_FP8) {
    unsigned char* dst = (c.sc_dst < 2 ? stage_sa<ST>() : stage_sb<ST>()) + (c.sc_dst & 1) * 256;
    __builtin_amdgcn_global_load_lds((const void*)(c.sc + c.kt * c.sc_step), (lds_void*)dst, 4, 0, 0);
  }
  advance<E>(c);
}

// fp8 operand of the block-scaled 32x32x64 MFMA (layout measured on gfx950):
// lane half h supplies K values 16h..16h+15 in its bytes 0..15 and
// 32+16h..47+16h in its bytes 16..31, and the scale of K block b (values
// 32b..32b+31) is the one passed by lane half b.  So half h takes chunks h
// and 2+h of the stage row (the h-th 16 values of each 32-value run) and
// passes the scale of run h.
__device__ inline i32x8_t frag8(const char* l, int row, int half) {
  union { i32x8_t v; uint4 q[2]; } u;
  u.q[0] = *(const uint4*)(l + swz(row, half));
  u.q[1] = *(const uint4*)(l + swz(row, 2 + half));
  return u.v;
}

// Multiply the K tile held in stage ST.
//   C waves (WW false): acc[m][n] += A(ra + 32 m) . B(rb + 32 n)
//   sketch wave (WW true): acc[m][n] += A(128 (n / 2) + 32 m) . Omega(32 (n % 2))
// bf16: two MFMA K steps of 16 per stage; fp8: one block-scaled K step of 64
// (operands as frag8 describes).
template <int E, bool DIAG, bool WW, int ST>
__device__ __attribute__((always_inline)) inline void compute(f32x16_t (&acc)[4][4], int lane, int ra, int rb) {
  const char* la = stage_a<ST>();
  const char* lb = (DIAG && !WW) ? stage_a<ST>() : stage_b<ST>();
  const int half = lane >> 5, lr = lane & 31;
  if constexpr (E == E_FP8) {
    const unsigned char* sa = stage_sa<ST>();
    const unsigned char* sb = (DIAG && !WW) ? stage_sa<ST>() : stage_sb<ST>();
    if (WW) {
      i32x8_t av[8], bv[2];
      int ea[8], eb[2];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        av[m] = frag8(la, m * 32 + lr, half);
        ea[m] = sa[(m * 32 + lr) * 2 + half];
      }
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        bv[n] = frag8(lb, n * 32 + lr, half);
        eb[n] = sb[(n * 32 + lr) * 2 + half];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              av[m + 4 * (n >> 1)], bv[n & 1], acc[m][n], 0, 0, 0, ea[m + 4 * (n >> 1)], 0, eb[n & 1]);
    } else {
      i32x8_t av[4], bv[4];
      int ea[4], eb[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        av[m] = frag8(la, ra + m * 32 + lr, half);
        bv[m] = frag8(lb, rb + m * 32 + lr, half);
        ea[m] = sa[(ra + m * 32 + lr) * 2 + half];
        eb[m] = sb[(rb + m * 32 + lr) * 2 + half];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          acc[m][n] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av[m], bv[n], acc[m][n], 0, 0, 0, ea[m], 0,
                                                                      eb[n]);
    }
  } else {
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
}

// One K step of the ring: wait for stage ST, barrier, refill the stage that
// was read in the previous step, multiply stage ST if this step is real.
template <int E, bool DIAG, bool WW, int ST>
__device__ __attribute__((always_inline)) inline void ring_step(PipeCtx& c, f32x16_t (&acc)[4][4], bool real,
                                                                int lane, int ra, int rb) {
  constexpr int PER = (DIAG ? 5 : 8) + (E == E_FP8 ? 1 : 0);   // loads per wave per stage
  wait_vm<2 * PER>();
  __builtin_amdgcn_s_barrier();
  issue<E, DIAG, (ST + 3) & 3>(c);
  if (real) compute<E, DIAG, WW, ST>(acc, lane, ra, rb);
  wait_lgkm0();
}

template <int E, bool DIAG, bool WW>
__device__ __attribute__((always_inline)) inline void ring(PipeCtx& c, f32x16_t (&acc)[4][4], int64_t nk, int lane,
                                                           int ra, int rb) {
  issue<E, DIAG, 0>(c);
  issue<E, DIAG, 1>(c);
  issue<E, DIAG, 2>(c);
  for (int64_t k = 0; k < nk; k += 4) {
    ring_step<E, DIAG, WW, 0>(c, acc, true, lane, ra, rb);
    ring_step<E, DIAG, WW, 1>(c, acc, k + 1 < nk, lane, ra, rb);
    ring_step<E, DIAG, WW, 2>(c, acc, k + 2 < nk, lane, ra, rb);
    ring_step<E, DIAG, WW, 3>(c, acc, k + 3 < nk, lane, ra, rb);
  }
  // every load must have landed before the workgroup's LDS is released
  wait_vm<0>();
  __builtin_amdgcn_s_barrier();
}

template <int E, bool DIAG>
__device__ __attribute__((always_inline)) inline void run_tile(const GramArgs& g, int split, int ti, int tj) {
  constexpr int ES = PipeElem<E>::ES;
  PipeCtx c;
  c.X = (const char*)g.X;
  c.Om = (const char*)g.omegaT;
  c.IBp = g.I * g.B;
  c.Bp = g.B;
  c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t kt0 = (int64_t)split * g.nkt / g.splits;
  const int64_t kt1 = (int64_t)(split + 1) * g.nkt / g.splits;     // kt1 > kt0 (splits <= nkt)
  c.na = kt0 / g.nbt;
  c.nk0 = (kt0 - c.na * g.nbt) * PipeElem<E>::KT;
  c.left = kt1 - kt0;
  c.kt = kt0;
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
      c.offa[j] = ra_ * g.B * ES + ch * 16;
      c.offb[j] = rb_ * g.B * ES + ch * 16;
    }
    if (DIAG) {
      const int row = c.wave * 16 + rl;       // sketch row 0..63
      const int sr = row < g.S ? row : g.S - 1;
      c.offb[0] = (int64_t)sr * g.J * ES + (p ^ ((row >> 2) & 3)) * 16;
    }
    if (E == E_FP8) {
      // scales: [K tile][Ipad rows][2] for X, [K tile][64][2] for Omega; a lane
      // fetches 4 bytes = the two runs of two consecutive rows
      const int64_t ipad = (int64_t)g.nt * PT;
      if (DIAG && c.wave >= 2) {
        const int l = lane < 32 ? lane : 31;
        c.sc = g.xexp_om + 4 * l;
        c.sc_step = 64 * 2;
        c.sc_dst = c.wave == 2 ? 2 : 3;       // wave 3 reloads the same bytes into an unused half
      } else {
        const int64_t base = (c.wave < 2 ? r0 : c0) + (c.wave & 1) * 128 + 2 * lane;
        c.sc = g.xexp + 2 * base;
        c.sc_step = ipad * 2;
        c.sc_dst = c.wave;
      }
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
    if (wwave) ring<E, true, true>(c, acc, nk, lane, ra, rb);
    else ring<E, true, false>(c, acc, nk, lane, ra, rb);
  } else {
    ring<E, false, false>(c, acc, nk, lane, ra, rb);
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

template <int E>
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
  if (ti == tj) run_tile<E, true>(g, split, ti, tj);
  else run_tile<E, false>(g, split, ti, tj);
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

// Omega^T (S x J) of one mode in the padded column layout (S x Jp): the
// value of stream index L = s J + j goes to column jp(j); padded columns
// must be zero beforehand.  B = 1: jp = j.  B > 1: j = a B + b with
// b = bh I_N + bl, jp = a Bp + bh I_Npad + bl.
// Index arithmetic in 32 bits when every index fits (the common case), else 64.
template <class IT>
__global__ void omega_pad_kernel(uint64_t seed, uint32_t mode, int64_t S, int64_t J_, int64_t B_, int64_t IN_,
                                 int64_t INp_, int64_t Jp, bf16_t* out) {
  const IT J = (IT)J_, B = (IT)B_, IN = (IT)IN_, INp = (IT)INp_;
  const int64_t total = S * J_;
  const int64_t npairs = (total + 1) / 2;
  const IT Bp = B > 1 ? (B / IN) * INp : 1;
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < npairs;
       m += (int64_t)gridDim.x * blockDim.x) {
    float z[2];
    gauss_pair_f32((uint64_t)m, mode, 0u, seed, z[0], z[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t L = 2 * m + h;
      if (L >= total) break;
      const IT Lt = (IT)L;
      const IT sv = Lt / J, j = Lt - sv * J;
      IT jp = j;
      if (B > 1) {
        const IT a = j / B, b = j - a * B;
        const IT bh = b / IN, bl = b - bh * IN;
        jp = a * Bp + bh * INp + bl;
      }
      out[(int64_t)sv * Jp + jp] = f32_to_bf16(z[h]);
    }
  }
}

// E8M0 scale byte for a run whose largest magnitude is amax: the smallest
// power of two 2^s with amax / 2^s <= 448 (the largest e4m3 value), biased
// by 127.  With amax = f 2^e, f in [0.5, 1): s = e - 9 if f <= 0.875, else
// e - 8 (448 = 0.875 2^9).  An all-zero run gets the smallest scale.
__device__ inline int e8m0_for(float amax) {
  if (!(amax > 0.f)) return 0;
  int e;
  const float f = frexpf(amax, &e);
  int s = f <= 0.875f ? e - 9 : e - 8;
  s = s < -127 ? -127 : (s > 127 ? 127 : s);
  return s + 127;
}

// max over each half (32 lanes) of a wave
__device__ inline float half_max(float v) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// 2^-s for the scale exponent s in [-127, 127] (exact; 2^-127 is subnormal)
__device__ inline float pow2_neg(int s) {
  return s < 127 ? __uint_as_float((uint32_t)(127 - s) << 23) : __uint_as_float(0x00400000u);
}

// e8m0_for with the exponent read from the float's bits (normal amax)
__device__ inline int e8m0_fast(float amax) {
  const uint32_t u = __float_as_uint(amax);
  const int ex = (int)((u >> 23) & 0xFF);
  if (ex == 0 || ex == 0xFF) return e8m0_for(amax);
  const int e = ex - 126;                                  // amax = f 2^e, f = 1.m / 2
  int sc = ((u & 0x7FFFFFu) <= 0x600000u ? e - 9 : e - 8);   // f <= 0.875 <=> 1.m <= 1.75
  sc = sc < -127 ? -127 : (sc > 127 ? 127 : sc);
  return sc + 127;
}

// max over the 8 lanes of an aligned group
__device__ inline float group8_max(float v) {
  v = fmaxf(v, __shfl_xor(v, 1, 64));
  v = fmaxf(v, __shfl_xor(v, 2, 64));
  v = fmaxf(v, __shfl_xor(v, 4, 64));
  return v;
}

// Four values -> packed e4m3 (scale byte sc, shared by the 8 lanes of a run of 32)
__device__ inline uint32_t pack_e4m3(const float* v, int sc) {
  const float mul = pow2_neg(sc - 127);
  uint32_t w = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) w |= (uint32_t)f32_to_e4m3(v[k] * mul) << (8 * k);
  return w;
}

__device__ inline uint2 pack_bf16(const float* v) {
  return make_uint2((uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16),
                    (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16));
}

// Padded copies of X viewed as R rows of length L (R = T / I_N, L = I_N), in
// bf16 and / or e4m3 with per-32 scales, any output may be null:
//   Xpad, Xp8 (+ Sp): R x Lp, zero padding;  Xt, Xt8 (+ St): L x Rp.
// 64 x 64 tiles through LDS; a thread handles 4 consecutive values (16 per
// tile row), so a run of 32 is 8 lanes of one wave.
template <class T>
__global__ void __launch_bounds__(256) pad_copies_kernel(const T* X, int64_t R, int64_t L, bool vec, bf16_t* Xpad,
                                                         int64_t Lp, bf16_t* Xt, int64_t Rp, fp8_t* Xp8,
                                                         unsigned char* Sp, fp8_t* Xt8, unsigned char* St) {
  __shared__ float tile[64][65];
  const int64_t tl = Lp / 64;
  const int64_t br = blockIdx.x / tl, bl = blockIdx.x - br * tl;
  const int64_t r0 = br * 64, l0 = bl * 64;
  const int t = threadIdx.x, q4 = (t & 15) * 4;
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    const int y = pass * 16 + (t >> 4);
    const int64_t r = r0 + y, l = l0 + q4;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (r < R) {
      const T* src = X + r * L + l;
      if (vec && l + 3 < L) {
        if constexpr (sizeof(T) == 4) {
          const float4 f = *(const float4*)src;
          v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
        } else if constexpr (sizeof(T) == 2) {
          const uint2 h = *(const uint2*)src;
          v[0] = bf16_to_f32((bf16_t)(h.x & 0xFFFF)); v[1] = bf16_to_f32((bf16_t)(h.x >> 16));
          v[2] = bf16_to_f32((bf16_t)(h.y & 0xFFFF)); v[3] = bf16_to_f32((bf16_t)(h.y >> 16));
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = (float)src[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (l + k < L) {
            if constexpr (sizeof(T) == 2) v[k] = bf16_to_f32(((const bf16_t*)src)[k]);
            else v[k] = (float)src[k];
          }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) tile[y][q4 + k] = v[k];
    // the run's scale: all lanes take part (rows past R hold zeros)
    int sc = 0;
    if (Xp8) sc = e8m0_fast(group8_max(fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])))));
    if (r < R) {
      if (Xpad) *(uint2*)(Xpad + r * Lp + l) = pack_bf16(v);
      if (Xp8) {
        *(uint32_t*)(Xp8 + r * Lp + l) = pack_e4m3(v, sc);
        if ((t & 7) == 0) Sp[r * (Lp / 32) + (l >> 5)] = (unsigned char)sc;
      }
    }
  }
  if (!Xt && !Xt8) return;
  __syncthreads();
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    const int y = pass * 16 + (t >> 4);            // output row l0 + y, values r0 + q4 .. + 3
    const int64_t l = l0 + y, r = r0 + q4;
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = tile[q4 + k][y];
    int sc = 0;
    if (Xt8) sc = e8m0_fast(group8_max(fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])))));
    if (l < L) {
      if (Xt) *(uint2*)(Xt + l * Rp + r) = pack_bf16(v);
      if (Xt8) {
        *(uint32_t*)(Xt8 + l * Rp + r) = pack_e4m3(v, sc);
        if ((t & 7) == 0) St[l * (Rp / 32) + (r >> 5)] = (unsigned char)sc;
      }
    }
  }
}

// bf16 rows (total a multiple of 32) -> e4m3 + per-32 scales; one wave per 64 values.
__global__ void quantize_rows_kernel(const bf16_t* src, int64_t total, fp8_t* q, unsigned char* scales) {
  const int lane = threadIdx.x & 63;
  const int64_t nchunk = (total + 63) / 64;
  for (int64_t ch = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); ch < nchunk;
       ch += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    const int64_t i = ch * 64 + lane;
    const float v = i < total ? bf16_to_f32(src[i]) : 0.f;
    const int sc = e8m0_for(half_max(fabsf(v)));
    if (i < total) {
      q[i] = f32_to_e4m3(ldexpf(v, 127 - sc));
      if ((lane & 31) == 0) scales[i >> 5] = (unsigned char)sc;
    }
  }
}

// out[kt][i][h] = plane[((a I + min(i, I-1)) Bp + k0) / 32 + h], kt = a (Bp / 64) + k0 / 64;
// IT: the index type (32 bits when the plane and the output fit)
template <class IT>
__global__ void gather_scales_kernel(const unsigned char* plane, int64_t I_, int64_t Bp_, int64_t ipad_,
                                     int64_t total, unsigned char* out) {
  const IT I = (IT)I_, Bp = (IT)Bp_, ipad = (IT)ipad_;
  const IT nbt = Bp / 64;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const IT et = (IT)e;
    const IT h = et & 1;
    const IT ri = et >> 1;
    const IT kt = ri / ipad, i = ri - kt * ipad;
    const IT a = kt / nbt, k0 = (kt - a * nbt) * 64;
    const IT ic = i < I ? i : I - 1;
    out[e] = plane[((uint64_t)(a * I + ic) * (uint64_t)Bp + k0) / 32 + h];
  }
}

}  // namespace

int64_t pad64(int64_t v) { return (v + 63) / 64 * 64; }

GramArgs gram_plan_pipe(int elem, int64_t A, int64_t I, int64_t Bp, int S, int cu_count) {
  GramArgs g = {};
  g.A = A;
  g.I = I;
  g.B = Bp;
  g.J = A * Bp;
  g.S = S;
  g.nt = (int)ceil_div(I, PT);
  g.ntri = g.nt * (g.nt + 1) / 2;
  g.ntiles = g.ntri;
  g.nbt = Bp / (elem == E_FP8 ? 64 : PK);
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

hipError_t launch_gram_pipe(int elem, const GramArgs& g, hipStream_t s) {
  if (g.nkt < 1 || g.splits > g.nkt || g.S > PW || g.B % 64) return hipErrorInvalidValue;
  if (elem == E_FP8) {
    if (!g.xexp || !g.xexp_om) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gram_pipe_kernel<E_FP8>, dim3((unsigned)(g.ntiles * g.splits)), dim3(256), 0, s, g);
  } else {
    hipLaunchKernelGGL(gram_pipe_kernel<E_BF16>, dim3((unsigned)(g.ntiles * g.splits)), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

hipError_t launch_pad_copies_fp8(int src_elem, const void* X, int64_t R, int64_t L, void* Xpad, void* Xt, void* Xp8,
                                 void* Sp, void* Xt8, void* St, hipStream_t s) {
  const int64_t Lp = pad64(L), Rp = pad64(R);
  const int64_t blocks = (Rp / 64) * (Lp / 64);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  const int es = src_elem == E_F64 ? 8 : src_elem == E_F32 ? 4 : 2;
  const bool vec = (L % 4) == 0 && ((uintptr_t)X % (4 * es)) == 0;
#define PCF(T)                                                                                                   \
  hipLaunchKernelGGL(pad_copies_kernel<T>, grid, dim3(256), 0, s, (const T*)X, R, L, vec, (bf16_t*)Xpad, Lp,      \
                     (bf16_t*)Xt, Rp, (fp8_t*)Xp8, (unsigned char*)Sp, (fp8_t*)Xt8, (unsigned char*)St)
  switch (src_elem) {
    case E_F64: PCF(double); break;
    case E_F32: PCF(float); break;
    default: PCF(bf16_t); break;
  }
#undef PCF
  return hipGetLastError();
}

hipError_t launch_quantize_rows_fp8(const void* src, int64_t rows, int64_t cols, void* q, void* scales,
                                    hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  if (cols % 32) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(ceil_div(total, 64), 4), 16384);
  hipLaunchKernelGGL(quantize_rows_kernel, dim3(grid), dim3(256), 0, s, (const bf16_t*)src, total, (fp8_t*)q,
                     (unsigned char*)scales);
  return hipGetLastError();
}

hipError_t launch_gather_scales(const void* plane, int64_t A, int64_t I, int64_t Bp, int64_t ipad, void* out,
                                hipStream_t s) {
  if (Bp % 64 || ipad < I) return hipErrorInvalidValue;
  const int64_t total = A * (Bp / 64) * ipad * 2;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 16384);
  if (total < ((int64_t)1 << 31) && A * I < ((int64_t)1 << 31))
    hipLaunchKernelGGL(gather_scales_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, (const unsigned char*)plane, I, Bp,
                       ipad, total, (unsigned char*)out);
  else
    hipLaunchKernelGGL(gather_scales_kernel<uint64_t>, dim3(grid), dim3(256), 0, s, (const unsigned char*)plane, I, Bp,
                       ipad, total, (unsigned char*)out);
  return hipGetLastError();
}

hipError_t launch_gram_pipe_reduce(const GramArgs& g, double* C, double* Wt, hipStream_t s) {
  const int64_t total = (int64_t)g.ntri * PT * PT + (int64_t)g.nt * PT * PW;
  unsigned rgrid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096);
  hipLaunchKernelGGL(gram_pipe_reduce_kernel, dim3(rgrid), dim3(256), 0, s, g, C, Wt);
  return hipGetLastError();
}

hipError_t launch_pad_copies(int src_elem, const void* X, int64_t R, int64_t L, void* Xpad, void* Xt, hipStream_t s) {
  return launch_pad_copies_fp8(src_elem, X, R, L, Xpad, Xt, nullptr, nullptr, nullptr, nullptr, s);
}

hipError_t launch_omega_pad(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t Jp,
                            void* out, hipStream_t s) {
  hipError_t e = fill_zero(out, (size_t)S * Jp * 2, s);
  if (e != hipSuccess) return e;
  const int64_t npairs = (S * J + 1) / 2;
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(npairs, 256), 16384);
  if (grid == 0) return hipSuccess;
  if (S * J < ((int64_t)1 << 31) && Jp < ((int64_t)1 << 31))
    hipLaunchKernelGGL(omega_pad_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), Jp, (bf16_t*)out);
  else
    hipLaunchKernelGGL(omega_pad_kernel<uint64_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), Jp, (bf16_t*)out);
  return hipGetLastError();
}

}  // namespace rbki
