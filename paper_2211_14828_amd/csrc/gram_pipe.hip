// bf16 Gram + sketch products of one mode (Remark 1: C = X_(n) X_(n)^T; Alg. 1,
// step 2: W = X_(n) Omega^(n)), streamed through LDS by direct global->LDS
// loads in a four-stage ring.
//
// Operands.  For each mode the products read a K-blocked copy of the
// mode's unfolding, built just before its Gram pass:
//   * the columns of X_(n) are taken in the zero-padded order of the view
//     [A_n, I_n, Bp_n], Bp_n = (B_n / I_N) I_Npad (I_Npad = I_N rounded up to
//     64; the last mode: A = 1, Bp = T / I_N rounded up to 64).  Padding adds
//     zero columns, which change neither C nor W;
//   * K tile kt holds 64 bytes of every row (32 bf16 or 64 e4m3 values), and
//     the copy is stored [kt][row][64 bytes] with the rows padded with zeros
//     to whole 256-row tiles.  One wave's 1 KB load of 16 rows is then one
//     contiguous block of whole cache lines (a row-major copy costs a 128-byte
//     line for every 64-byte row chunk, about half the load throughput);
//   * Omega^T in the same column order, blocked [kt][64 sketch rows][64
//     bytes], rows past S zero.
// Every K tile is therefore whole: no bounds checks, no masking.
//
// Tiles.  A workgroup (4 waves) owns one 256 x 256 lower-triangle tile of C
// and a slice of the contraction (split-K).  Off-diagonal tiles give each
// wave a 128 x 128 block (4 x 4 MFMA 32x32x16 tiles).  In a diagonal tile the
// upper-right 128 x 128 block is the transpose of the lower-left one, so that
// wave computes the 256 x 64 sketch block W(rows, 0..63) instead (S <= 64).
// All tiles cost the same, and the number of splits is chosen so that tiles x
// splits fills whole rounds of the 256 compute units.  The tiles of one split
// share its K range, so they run on one XCD (one L2); when whole splits leave
// spare compute units on every XCD (10 tiles: 3 splits, 30 of 32 units), the
// spare units take further splits whose tiles are spread over several XCDs.
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
// chosen so that the run's largest magnitude maps to at most 448.  The copy
// stores the scales of a K tile and 256-row tile as [half][row % 32][row / 32]
// (512 bytes; half: the first or second run of 32 of the 64-value row), the
// sketch's as [half][row % 32][4] (rows 0..63: bytes 0, 1; 256 bytes).  A
// lane's four fragments of a 128-row block then take their scales from one
// 4-byte LDS read, held in one register: the MFMA's scale op_sel picks the
// byte (measured on gfx950: op_sel k selects byte k).  Each wave fetches 256
// bytes of scales for a stage with one more 4-byte direct-to-LDS load.
//
// Split-K partials (float32) are reduced in a fixed order in float64 by a
// second kernel: results are deterministic.
#include <type_traits>

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
  const char* xk;         // next K tile of the blocked operand
  const char* ok;         // next K tile of the blocked sketch
  int64_t xstep, ostep;   // bytes per K tile of each
  int64_t left;           // K tiles of this split not yet loaded (the last one is reloaded after)
  int64_t kt;             // global index of the next K tile (scale lookup)
  int offa[4], offb[4];   // per-lane byte offsets of this lane's rows and chunks within a K tile
  const unsigned char* sc;    // fp8: this lane's scale source at K tile 0
  int64_t sc_step;            // fp8: bytes per K tile of that source
  int sc_dst;                 // fp8: 0..3 = A scales low/high half, B scales low/high half
  int wave;
};

template <int E> struct PipeElem {
  static constexpr int ES = E == E_FP8 ? 1 : 2;      // bytes per value
  static constexpr int KT = PROW / ES;               // values per stage row
};

// Advance the next K tile by one, holding at the split's last.  Branch-free:
// a branch would split the K step into basic blocks, and the compiler then
// sinks the MFMAs of several steps past their barriers into one block (all
// their fragments live at once, and no overlap with the loads).
__device__ __attribute__((always_inline)) inline void advance(PipeCtx& c) {
  const int64_t d = c.left > 1 ? 1 : 0;
  c.xk += d * c.xstep;
  c.ok += d * c.ostep;
  c.kt += d;
  c.left -= d;
}

// Issue the loads of the next K tile into stage ST: A rows r0..r0+255 (4
// loads per wave), B rows c0..c0+255 (off-diagonal, 4 per wave) or sketch rows
// 0..63 (diagonal, 1 per wave), and for fp8 one load of scales per wave.
// Lane l of load q covers row 16 q + l / 4 and the 16-byte chunk at position
// l % 4 of that row.
template <int E, bool DIAG, int ST>
__device__ __attribute__((always_inline)) inline void issue(PipeCtx& c) {
#pragma unroll
  for (int j = 0; j < 4; ++j)
    __builtin_amdgcn_global_load_lds((const void*)(c.xk + c.offa[j]),
                                     (lds_void*)(stage_a<ST>() + (j * 4 + c.wave) * 1024), 16, 0, 0);
  if (DIAG) {
    __builtin_amdgcn_global_load_lds((const void*)(c.ok + c.offb[0]), (lds_void*)(stage_b<ST>() + c.wave * 1024),
                                     16, 0, 0);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(c.xk + c.offb[j]),
                                       (lds_void*)(stage_b<ST>() + (j * 4 + c.wave) * 1024), 16, 0, 0);
  }
  if (E == E_FP8) {
    unsigned char* dst = (c.sc_dst < 2 ? stage_sa<ST>() : stage_sb<ST>()) + (c.sc_dst & 1) * 256;
    __builtin_amdgcn_global_load_lds((const void*)(c.sc + c.kt * c.sc_step), (lds_void*)dst, 4, 0, 0);
  }
  advance(c);
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

// Operand fragments of one K tile, held in registers.
//   C waves (WW false): A rows ra + 32 m and B rows rb + 32 n, m, n < 4
//   sketch wave (WW true): A rows 32 m, m < 8, and sketch rows 32 n, n < 2
// bf16 keeps the two MFMA K steps of 16 of a stage; fp8 one block-scaled K
// step of 64 with the E8M0 scale of each fragment's lane half.
template <int E, bool WW> struct Frags;
template <> struct Frags<E_FP8, false> { i32x8_t a[4], b[4]; int ea, eb; };   // scales: byte m of ea / eb
template <> struct Frags<E_FP8, true> { i32x8_t a[8], b[2]; int ea[2], eb; };
template <> struct Frags<E_BF16, false> { bf16x8_t a[2][4], b[2][4]; };
template <> struct Frags<E_BF16, true> { bf16x8_t a[2][8], b[2][2]; };

// The packed scales of the fp8 fragments of the K tile in stage ST.
template <bool DIAG, bool WW, int ST>
__device__ __attribute__((always_inline)) inline void load_scales(Frags<E_FP8, WW>& f, int lane, int ra, int rb) {
  const int half = lane >> 5, lr = lane & 31;
  const int sl = (half * 32 + lr) * 8;             // this lane's 8 bytes of a 256-row tile
  if constexpr (WW) {
    f.ea[0] = *(const int*)(stage_sa<ST>() + sl);
    f.ea[1] = *(const int*)(stage_sa<ST>() + sl + 4);
    f.eb = *(const int*)(stage_sb<ST>() + (half * 32 + lr) * 4);
  } else {
    f.ea = *(const int*)(stage_sa<ST>() + sl + (ra >> 5));
    f.eb = *(const int*)((DIAG ? stage_sa<ST>() : stage_sb<ST>()) + sl + (rb >> 5));
  }
}

// Read the fragments of the K tile held in stage ST (fp8 operands as frag8
// describes).  Fragment rows are r0 + 32 m + (lane % 32) with r0 a multiple of
// 32, so the swizzle depends on the lane only and every address is a per-lane
// base plus a constant.
template <int E, bool DIAG, bool WW, int ST>
__device__ __attribute__((always_inline)) inline void load_frags(Frags<E, WW>& f, int lane, int ra, int rb) {
  const char* la = stage_a<ST>();
  const char* lb = (DIAG && !WW) ? stage_a<ST>() : stage_b<ST>();
  const int half = lane >> 5, lr = lane & 31;
  constexpr int NA = WW ? 8 : 4, NB = WW ? 2 : 4;
  const int a0 = WW ? 0 : ra, b0 = WW ? 0 : rb;
  const int sw = (lr >> 2) & 3;
  const char* pa = la + (a0 + lr) * PROW;
  const char* pb = lb + (b0 + lr) * PROW;
  if constexpr (E == E_FP8) {
    const int c0 = (half ^ sw) << 4, c1 = ((2 + half) ^ sw) << 4;
#pragma unroll
    for (int m = 0; m < NA; ++m) {
      union { i32x8_t v; uint4 q[2]; } u;
      u.q[0] = *(const uint4*)(pa + m * 32 * PROW + c0);
      u.q[1] = *(const uint4*)(pa + m * 32 * PROW + c1);
      f.a[m] = u.v;
    }
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      union { i32x8_t v; uint4 q[2]; } u;
      u.q[0] = *(const uint4*)(pb + n * 32 * PROW + c0);
      u.q[1] = *(const uint4*)(pb + n * 32 * PROW + c1);
      f.b[n] = u.v;
    }
    load_scales<DIAG, WW, ST>(f, lane, ra, rb);
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int ch = ((2 * t + half) ^ sw) << 4;
#pragma unroll
      for (int m = 0; m < NA; ++m) f.a[t][m] = *(const bf16x8_t*)(pa + m * 32 * PROW + ch);
#pragma unroll
      for (int n = 0; n < NB; ++n) f.b[t][n] = *(const bf16x8_t*)(pb + n * 32 * PROW + ch);
    }
  }
}

// Compile-time loop: f(integral_constant<int, T>) for T = B .. N-1.
template <int B, int N> struct Unroll {
  template <class F> __device__ __attribute__((always_inline)) static void run(F&& f) {
    if constexpr (B < N) {
      f(std::integral_constant<int, B>{});
      Unroll<B + 1, N>::run(f);
    }
  }
};

// One DMA of the loads issue() makes for stage ST (q < loads per wave).
template <int E, bool DIAG, int ST, int q>
__device__ __attribute__((always_inline)) inline void dma_one(PipeCtx& c) {
  if constexpr (q < 4) {
    __builtin_amdgcn_global_load_lds((const void*)(c.xk + c.offa[q]),
                                     (lds_void*)(stage_a<ST>() + (q * 4 + c.wave) * 1024), 16, 0, 0);
  } else if constexpr (DIAG ? q == 4 : q < 8) {
    if constexpr (DIAG)
      __builtin_amdgcn_global_load_lds((const void*)(c.ok + c.offb[0]), (lds_void*)(stage_b<ST>() + c.wave * 1024),
                                       16, 0, 0);
    else
      __builtin_amdgcn_global_load_lds((const void*)(c.xk + c.offb[DIAG ? 0 : q - 4]),
                                       (lds_void*)(stage_b<ST>() + ((DIAG ? 0 : q - 4) * 4 + c.wave) * 1024), 16, 0, 0);
  } else if constexpr (E == E_FP8) {
    unsigned char* dst = (c.sc_dst < 2 ? stage_sa<ST>() : stage_sb<ST>()) + (c.sc_dst & 1) * 256;
    __builtin_amdgcn_global_load_lds((const void*)(c.sc + c.kt * c.sc_step), (lds_void*)dst, 4, 0, 0);
  }
}

// Fragment f (< NA + NB) of the K tile in stage ST (load_frags, one at a time).
template <int E, bool DIAG, bool WW, int ST, int f>
__device__ __attribute__((always_inline)) inline void frag_one(Frags<E, WW>& fr, int lane, int ra, int rb) {
  constexpr int NA = WW ? 8 : 4;
  const int half = lane >> 5, lr = lane & 31;
  const int sw = (lr >> 2) & 3;
  constexpr bool isa = f < NA;
  constexpr int idx = isa ? f : f - NA;
  const int r0 = isa ? (WW ? 0 : ra) : (WW ? 0 : rb);
  const char* base = (isa || (DIAG && !WW)) ? stage_a<ST>() : stage_b<ST>();
  const char* pr = base + (r0 + idx * 32 + lr) * PROW;
  if constexpr (E == E_FP8) {
    union { i32x8_t v; uint4 q[2]; } u;
    u.q[0] = *(const uint4*)(pr + ((half ^ sw) << 4));
    u.q[1] = *(const uint4*)(pr + (((2 + half) ^ sw) << 4));
    if constexpr (isa) fr.a[idx] = u.v;
    else fr.b[idx] = u.v;
    if constexpr (f == NA) load_scales<DIAG, WW, ST>(fr, lane, ra, rb);   // with the first fragment read
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const bf16x8_t v = *(const bf16x8_t*)(pr + (((2 * t + half) ^ sw) << 4));
      if constexpr (isa) fr.a[t][idx] = v;
      else fr.b[t][idx] = v;
    }
  }
}

// MFMA tile t (< 16) of one K tile: (m, n) = (t / 4, t % 4), as in mma().
template <int E, bool WW, int t>
__device__ __attribute__((always_inline)) inline void mma_one(f32x16_t (&acc)[4][4], const Frags<E, WW>& f) {
  constexpr int m = t >> 2, n = t & 3;
  constexpr int ia = WW ? m + 4 * (n >> 1) : m, ib = WW ? (n & 1) : n;
  if constexpr (E == E_FP8) {
    int ea;
    if constexpr (WW) ea = f.ea[ia >> 2];
    else ea = f.ea;
    acc[m][n] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(f.a[ia], f.b[ib], acc[m][n], 0, 0, ia & 3, ea, ib & 3,
                                                                f.eb);
  } else {
    acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[0][ia], f.b[0][ib], acc[m][n], 0, 0, 0);
    acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[1][ia], f.b[1][ib], acc[m][n], 0, 0, 0);
  }
}

// Which fragment of the next tile is read after MFMA slot t (-1: none).  MFMAs
// run m-major (t = 4 m + n), so the current tile's A fragments die one by one
// (C waves: a[m] after slot 4 m + 3; the sketch wave: a[m] after 4 m + 1 and
// a[m + 4] after 4 m + 3) and the next tile's A fragments are read right
// after, into the freed registers; its B fragments (live to the end of the
// step) are read first.  Fragment index: a[i] = i, b[j] = NA + j.
template <bool WW> __device__ constexpr int next_frag_at(int t) {
  if (WW) {
    constexpr int at[16] = {8, 9, 0, -1, 4, -1, 1, -1, 5, -1, 2, -1, 6, 3, 7, -1};
    return at[t];
  } else {
    constexpr int at[16] = {4, 5, 6, 7, 0, -1, -1, -1, 1, -1, -1, -1, 2, 3, -1, -1};
    return at[t];
  }
}

// K step k of the ring (ST = k mod 4).  On entry the fragments of tile k are
// in `cur` and tiles k+1..k+3 are loaded or in flight.  Wait for tile k+1,
// barrier (every wave has read tile k into registers and sees tile k+1),
// then multiply tile k while refilling stage ST with tile k+4 and reading
// tile k+1 into `nxt`.  A global->LDS load holds the wave's issue until the
// address unit accepts it, so the loads and the LDS reads are interleaved one
// by one with the MFMAs (scheduling barriers keep the order): the address
// unit works while the matrix cores run, and the next tile's LDS reads are
// in flight under this tile's MFMAs.  REAL false (past the end of the split)
// skips the MFMAs.
template <int E, bool DIAG, bool WW, int ST, bool REAL>
__device__ __attribute__((always_inline)) inline void ring_step(PipeCtx& c, f32x16_t (&acc)[4][4],
                                                                const Frags<E, WW>& cur, Frags<E, WW>& nxt,
                                                                int lane, int ra, int rb) {
  constexpr int PER = (DIAG ? 5 : 8) + (E == E_FP8 ? 1 : 0);   // loads per wave per stage
  wait_vm<2 * PER>();
  __builtin_amdgcn_s_barrier();
  Unroll<0, 16>::run([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    constexpr int f = next_frag_at<WW>(t);
    if constexpr (REAL) mma_one<E, WW, t>(acc, cur);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (t < PER) dma_one<E, DIAG, ST, t>(c);
    if constexpr (f >= 0) frag_one<E, DIAG, WW, (ST + 1) & 3, f>(nxt, lane, ra, rb);
    __builtin_amdgcn_sched_barrier(0);
  });
  advance(c);
  wait_lgkm0();
}

template <int E, bool DIAG, bool WW>
__device__ __attribute__((always_inline)) inline void ring(PipeCtx& c, f32x16_t (&acc)[4][4], int64_t nk, int lane,
                                                           int ra, int rb) {
  constexpr int PER = (DIAG ? 5 : 8) + (E == E_FP8 ? 1 : 0);
  issue<E, DIAG, 0>(c);
  issue<E, DIAG, 1>(c);
  issue<E, DIAG, 2>(c);
  issue<E, DIAG, 3>(c);
  Frags<E, WW> f0, f1;
  wait_vm<3 * PER>();
  __builtin_amdgcn_s_barrier();
  load_frags<E, DIAG, WW, 0>(f0, lane, ra, rb);
  wait_lgkm0();
  int64_t k = 0;
  for (; k + 4 <= nk; k += 4) {
    ring_step<E, DIAG, WW, 0, true>(c, acc, f0, f1, lane, ra, rb);
    ring_step<E, DIAG, WW, 1, true>(c, acc, f1, f0, lane, ra, rb);
    ring_step<E, DIAG, WW, 2, true>(c, acc, f0, f1, lane, ra, rb);
    ring_step<E, DIAG, WW, 3, true>(c, acc, f1, f0, lane, ra, rb);
  }
  if (k < nk) {                                   // 1..3 tiles left
    ring_step<E, DIAG, WW, 0, true>(c, acc, f0, f1, lane, ra, rb);
    if (k + 1 < nk) ring_step<E, DIAG, WW, 1, true>(c, acc, f1, f0, lane, ra, rb);
    else ring_step<E, DIAG, WW, 1, false>(c, acc, f1, f0, lane, ra, rb);
    if (k + 2 < nk) ring_step<E, DIAG, WW, 2, true>(c, acc, f0, f1, lane, ra, rb);
    else ring_step<E, DIAG, WW, 2, false>(c, acc, f0, f1, lane, ra, rb);
  }
  // every load must have landed before the workgroup's LDS is released
  wait_vm<0>();
  __builtin_amdgcn_s_barrier();
}

template <int E, bool DIAG>
__device__ __attribute__((always_inline)) inline void run_tile(const GramArgs& g, int split, int ti, int tj) {
  PipeCtx c;
  c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t kt0 = (int64_t)split * g.nkt / g.splits;
  const int64_t kt1 = (int64_t)(split + 1) * g.nkt / g.splits;     // kt1 > kt0 (splits <= nkt)
  const int64_t ipad = (int64_t)g.nt * PT;                          // rows of a K tile of the operand
  c.xstep = ipad * PROW;
  c.ostep = (int64_t)PW * PROW;
  c.xk = (const char*)g.X + kt0 * c.xstep;
  c.ok = (const char*)g.omegaT + kt0 * c.ostep;
  c.left = kt1 - kt0;
  c.kt = kt0;
  const int r0 = ti * PT, c0 = tj * PT;
  {
    // rows past I and sketch rows past S are zero in the blocked copies
    const int rl = lane >> 2, p = lane & 3;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = (j * 4 + c.wave) * 16 + rl;
      const int ch = p ^ ((row >> 2) & 3);
      c.offa[j] = (r0 + row) * PROW + ch * 16;
      c.offb[j] = (c0 + row) * PROW + ch * 16;
    }
    if (DIAG) {
      const int row = c.wave * 16 + rl;       // sketch row 0..63
      c.offb[0] = row * PROW + (p ^ ((row >> 2) & 3)) * 16;
    }
    if (E == E_FP8) {
      // scales: [K tile][Ipad rows][2] for X, [K tile][64][2] for Omega; a lane
      // fetches 4 bytes = the two runs of two consecutive rows
      // per K tile: 512 bytes per 256-row tile of the operand, 256 for the
      // sketch; waves 0, 1 fetch the A tile's, waves 2, 3 the B tile's (or,
      // in a diagonal tile, wave 2 the sketch's and wave 3 the same bytes
      // again into an unused half, so that every wave issues the same loads)
      if (DIAG && c.wave >= 2) {
        c.sc = g.xexp_om + 4 * lane;
        c.sc_step = 256;
        c.sc_dst = c.wave == 2 ? 2 : 3;
      } else {
        const int tile = c.wave < 2 ? ti : tj;
        c.sc = g.xexp + (int64_t)tile * 512 + (c.wave & 1) * 256 + 4 * lane;
        c.sc_step = (int64_t)g.nt * 512;
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
    // split (which share its K range) on one XCD; the spare slots of every
    // XCD take the extra splits' tiles in turn (slots past them are idle)
    const int xcd = w & 7, slot = w >> 3;
    if (g.xleft == 0 || slot < g.xbase * g.ntiles) {
      split = xcd + 8 * (slot / g.ntiles);
      tile = slot % g.ntiles;
    } else {
      const int e = xcd * g.xleft + (slot - g.xbase * g.ntiles);
      if (e >= (g.splits - 8 * g.xbase) * g.ntiles) return;
      split = 8 * g.xbase + e / g.ntiles;
      tile = e % g.ntiles;
    }
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

// Omega^T (S x J) of one mode, blocked: the value of stream index L = s J + j
// goes to padded column jp(j), stored at [jp / KT][s][jp % KT] (KT values per
// 64 sketch rows of a K tile); padded columns and rows s >= S must be zero
// beforehand.  B = 1: jp = j.  B > 1: j = a B + b with b = bh I_N + bl,
// jp = a Bp + bh I_Npad + bl.
// Index arithmetic in 32 bits when every index fits (the common case), else 64.
template <class IT>
__global__ void omega_block_kernel(uint64_t seed, uint32_t mode, int64_t S, int64_t J_, int64_t B_, int64_t IN_,
                                   int64_t INp_, int KT, bf16_t* out) {
  const IT J = (IT)J_, B = (IT)B_, IN = (IT)IN_, INp = (IT)INp_;
  const int64_t total = S * J_;
  const int64_t npairs = (total + 1) / 2;
  const IT Bp = B > 1 ? (B / IN) * INp : 1;
  const IT kt_sz = (IT)KT;
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
      const IT kt = jp / kt_sz, kk = jp - kt * kt_sz;
      out[((int64_t)kt * PW + sv) * KT + kk] = f32_to_bf16(z[h]);
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

// e4m3 bytes of a and b (low two bytes of the result, a first) by the
// hardware conversion: round to nearest even into OCP e4m3, the same bytes as
// f32_to_e4m3 for finite |x| <= 448 (every input here is scaled into that
// range; non-finite inputs give NaN codes instead of saturating).
__device__ inline uint32_t e4m3x2(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

// Four values -> packed e4m3 (scale byte sc, shared by the 8 lanes of a run of 32)
__device__ inline uint32_t pack_e4m3(const float* v, int sc) {
  const float mul = pow2_neg(sc - 127);
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0] * mul, v[1] * mul, 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[2] * mul, v[3] * mul, lo, true);
}

// Four values X[off .. off+3] as float; values at or past `avail` (the
// elements left in the row) are zero.  vec: X and the row length are such
// that every 4-aligned offset is 4-element aligned (float4 / 8-byte loads).
template <class T>
__device__ inline void load4(const T* X, int64_t off, int64_t avail, bool vec, float* v) {
  const T* src = X + off;
  if (vec && avail >= 4) {
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
    for (int k = 0; k < 4; ++k) {
      if (k < avail) {
        if constexpr (sizeof(T) == 2) v[k] = bf16_to_f32(((const bf16_t*)src)[k]);
        else v[k] = (float)src[k];
      } else {
        v[k] = 0.f;
      }
    }
  }
}

// Sixteen values src[0 .. 15] as float, every one inside X; src is aligned
// to four elements.
template <class T>
__device__ inline void load16(const T* src, float* v) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 f = ((const float4*)src)[k];
      v[4 * k] = f.x; v[4 * k + 1] = f.y; v[4 * k + 2] = f.z; v[4 * k + 3] = f.w;
    }
  } else if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint2 h = ((const uint2*)src)[k];
      v[4 * k] = bf16_to_f32((bf16_t)(h.x & 0xFFFF)); v[4 * k + 1] = bf16_to_f32((bf16_t)(h.x >> 16));
      v[4 * k + 2] = bf16_to_f32((bf16_t)(h.y & 0xFFFF)); v[4 * k + 3] = bf16_to_f32((bf16_t)(h.y >> 16));
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double2 d = ((const double2*)src)[k];
      v[2 * k] = (float)d.x; v[2 * k + 1] = (float)d.y;
    }
  }
}

__device__ inline uint2 pack_bf16(const float* v) {
  return make_uint2((uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16),
                    (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16));
}

// Padded bf16 copies of X viewed as R rows of length L (R = T / I_N,
// L = I_N), either may be null: Xpad R x Lp (the first mode product reads it,
// and the bf16 Gram fallback of the leading modes), Xt L x Rp (the bf16 Gram
// fallback of the last mode); zero padding.  64 x 64 tiles through LDS; a
// thread handles 4 consecutive values.
template <class T>
__global__ void __launch_bounds__(256) pad_copies_kernel(const T* X, int64_t R, int64_t L, bool vec, bf16_t* Xpad,
                                                         int64_t Lp, bf16_t* Xt, int64_t Rp) {
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
    if (r < R) load4(X, r * L + l, L - l, vec, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) tile[y][q4 + k] = v[k];
    if (r < R && Xpad) *(uint2*)(Xpad + r * Lp + l) = pack_bf16(v);
  }
  if (!Xt) return;
  __syncthreads();
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    const int y = pass * 16 + (t >> 4);            // output row l0 + y, values r0 + q4 .. + 3
    const int64_t l = l0 + y, r = r0 + q4;
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = tile[q4 + k][y];
    if (l < L) *(uint2*)(Xt + l * Rp + r) = pack_bf16(v);
  }
}

// Position of the scale of run h of row `rowid` (= K tile x rows + row, rows a
// multiple of 256) in the operand's scale layout [K tile][256-row tile][h]
// [row % 32][row / 32 within the tile].
__device__ inline int64_t scale_pos(int64_t rowid, int h) {
  const int rr = (int)(rowid & 255);
  return ((rowid >> 8) * 2 + h) * 256 + (rr & 31) * 8 + (rr >> 5);
}

// 16 output bytes of a blocked copy: VPC values (16 e4m3 or 8 bf16), for
// e4m3 with the scale of its run of 32 (the lane and its neighbour lane^1
// hold the two halves of a run).  Returns the scale byte (e4m3) or 0.
// The same 16 bytes, returned instead of stored (sc: the scale byte, or 0).
template <int E>
__device__ inline uint4 encode_chunk(const float* v, int& sc) {
  if constexpr (E == E_FP8) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) m = fmaxf(m, fabsf(v[k]));
    m = fmaxf(m, __shfl_xor(m, 1, 64));
    sc = e8m0_fast(m);
    return make_uint4(pack_e4m3(v, sc), pack_e4m3(v + 4, sc), pack_e4m3(v + 8, sc), pack_e4m3(v + 12, sc));
  } else {
    sc = 0;
    const uint2 lo = pack_bf16(v), hi = pack_bf16(v + 4);
    return make_uint4(lo.x, lo.y, hi.x, hi.y);
  }
}

template <int E>
__device__ inline int store_chunk(const float* v, char* dst, bool store = true) {
  if constexpr (E == E_FP8) {
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) m = fmaxf(m, fabsf(v[k]));
    m = fmaxf(m, __shfl_xor(m, 1, 64));
    const int sc = e8m0_fast(m);
    uint4 w;
    w.x = pack_e4m3(v, sc);
    w.y = pack_e4m3(v + 4, sc);
    w.z = pack_e4m3(v + 8, sc);
    w.w = pack_e4m3(v + 12, sc);
    if (store) *(uint4*)dst = w;
    return sc;
  } else {
    const uint2 lo = pack_bf16(v), hi = pack_bf16(v + 4);
    if (store) *(uint4*)dst = make_uint4(lo.x, lo.y, hi.x, hi.y);
    return 0;
  }
}

// Blocked copies of every pipelined mode's unfolding in one pass over X.  X
// is read as H x L rows of its last dimension (L = I_{N-1}, the last leading
// dimension; H the product of the others; row r = h L + l) and I_N columns c.
//  - Leading mode n < N-1: row r of its view [A_n, I_n, B_n] is (a, i, bh)
//    with r = (a I_n + i) Bh_n + bh, Bh_n = B_n / I_N; padded column
//    b' = bh I_Npad + c holds X[r][c] (zero for c >= I_N).  Copy n is
//    [kt][i][64 bytes] with kt = a (Bh_n I_Npad / KT) + b' / KT, rows padded
//    to ipad_n (the padding rows are zeroed separately).
//  - The last mode: operand row c (zero for c >= I_N, up to its ipad), K
//    index k = h Lp + l with Lp = pad64(L) (zero for l >= L), so that every
//    K tile lies inside one run of L rows; copy [k / KT][c][64 bytes].
// e4m3 scales in the layout scale_pos describes.  xpad (nullable): the
// row-major padded bf16 copy.
//
// A workgroup takes 64 rows l0 .. l0+63 by 64 columns c0 .. c0+63 (l0, c0
// multiples of 64) for four consecutive h in turn: thread t reads 16 values
// of row l0 + t/4 and writes the leading copies' chunks from registers (four
// threads fill the 64 bytes of a row chunk; neighbouring l are neighbouring
// rows of mode N-2); the tile then goes through LDS transposed, and thread
// t writes 16 K values of the last mode's row c0 + t/4.  Mode N-3 (cm.stage,
// whose rows follow h) keeps its chunks of the four h in LDS and writes
// them at the end: its rows h .. h+3 are neighbours, so each l gives one
// 256-byte run instead of four scattered 64-byte pieces.
struct CopyModes {
  int n;                          // leading modes with a copy
  int stage;                      // index (< n) of mode N-3's copy, or -1
  int64_t I[7], Bh[7], ipad[7], nbt[7];
  char* out[7];
  unsigned char* sc[7];
  char* last;                     // the last mode's copy (nullable)
  unsigned char* last_sc;
  int64_t last_ipad;
};

template <class IT, int KT>
__device__ inline int64_t lead_rowid(const CopyModes& cm, int m, IT r, IT col, IT INp, IT& kk) {
  const IT Bh = (IT)cm.Bh[m], Im = (IT)cm.I[m];
  const IT tt = r / Bh, bh = r - tt * Bh;
  const IT a = tt / Im, i = tt - a * Im;
  const IT bp = bh * INp + col;
  const IT kt = a * (IT)cm.nbt[m] + bp / KT;
  kk = bp - (bp / KT) * KT;
  return (int64_t)kt * cm.ipad[m] + i;
}

constexpr int COPY_HG = 64;      // h blocks (of 4) per 256 rows of mode N-3

// Workgroup ids of the copy: whole runs of 8 (one per XCD) x COPY_HG slots.
__host__ __device__ inline int64_t copy_ids(int64_t ngroups) { return (ngroups + 7) / 8 * 8 * COPY_HG; }

template <class T, int E, class IT>
__global__ void __launch_bounds__(256) block_copy_kernel(const T* X, int64_t H_, int64_t L_, int64_t IN_,
                                                         int64_t INp_, bool vec, CopyModes cm, bf16_t* xpad) {
  constexpr int VPC = E == E_FP8 ? 16 : 8;     // values per 16-byte chunk
  constexpr int KT = 4 * VPC;
  constexpr int ES = E == E_FP8 ? 1 : 2;
  constexpr int NCH = 16 / VPC;                // chunks per thread and tile row
  constexpr int HB = 4;                        // h per workgroup step
  __shared__ float tile[64][65];
  __shared__ uint4 stg[HB][64][4 * NCH];       // mode N-3's chunks: [h][l][chunk]
  const IT H = (IT)H_, L = (IT)L_, IN = (IT)IN_, INp = (IT)INp_;
  const IT Lp = (L + 63) / 64 * 64;
  const IT nlb = Lp / 64, nlead = INp / 64;
  const IT ncb = (IT)((cm.last ? cm.last_ipad : INp_) / 64);
  const IT nhb = (H + HB - 1) / HB;
  const int t = threadIdx.x, rr = t >> 2, q = t & 3;
  // Tile order.  Workgroups go to the chip's XCDs in turn by id (8 of them).
  // A line of mode N-3's e4m3 scales holds bytes of the 64 h blocks of one
  // 256-row tile (at one K tile); those 64 tiles take consecutive slots on
  // one XCD, so that the line is completed in one L2 and written back whole.
  // Ids past the tiles (a short last group of h blocks) do nothing.
  const int64_t nhg = ((int64_t)nhb + COPY_HG - 1) / COPY_HG;
  const int64_t ngroups = nhg * nlb * ncb;
  const int64_t nids = copy_ids(ngroups);
  for (int64_t id = blockIdx.x; id < nids; id += gridDim.x) {
    const int64_t slot = id >> 3, grp = (slot / COPY_HG) * 8 + (id & 7);
    if (grp >= ngroups) continue;                // the same for the whole workgroup
    const IT cb = (IT)(grp % ncb), rest = (IT)(grp / ncb);
    const IT lb = rest % nlb, hb = (rest / nlb) * (IT)COPY_HG + (IT)(slot % COPY_HG);
    if (hb >= nhb) continue;
    const IT l = lb * 64 + (IT)rr, c = cb * 64 + (IT)q * 16;
    const bool ok = l < L;
    const bool lead = cb < nlead;              // the tile holds leading-mode columns
    for (int hh = 0; hh < HB; ++hh) {
      const IT h = hb * HB + (IT)hh;
      if (h >= H) break;                         // the same for the whole workgroup
      const IT r = h * L + l;
      float v[16];
      if (vec && (cb + 1) * 64 <= IN && (lb + 1) * 64 <= L) {
        // interior tile (the same for the whole workgroup): unconditional loads
        load16(X + (int64_t)r * IN + c, v);
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = 0.f;
        if (ok && c < IN) {
#pragma unroll
          for (int k = 0; k < 16; k += 4) load4(X, (int64_t)r * IN + c + k, IN_ - (int64_t)c - k, vec, v + k);
        }
      }
      if (lead) {
        for (int m = 0; m < cm.n; ++m) {
          // every lane takes part (the e4m3 scale pairs lanes q, q ^ 1); only
          // rows inside X store
#pragma unroll
          for (int u = 0; u < NCH; ++u) {
            IT kk;
            const int64_t rowid = lead_rowid<IT, KT>(cm, m, r, c + (IT)(u * VPC), INp, kk);
            int sc;
            const uint4 w = encode_chunk<E>(v + u * VPC, sc);
            if (m == cm.stage) stg[hh][rr][q * NCH + u] = w;
            else if (ok) *(uint4*)(cm.out[m] + rowid * 64 + kk * ES) = w;
            if (ok && E == E_FP8 && ((kk >> 4) & 1) == 0)
              cm.sc[m][scale_pos(rowid, (int)(kk >> 5))] = (unsigned char)sc;
          }
        }
        if (xpad && ok) {
          bf16_t* dst = xpad + (int64_t)r * INp + c;
#pragma unroll
          for (int k = 0; k < 16; k += 4) *(uint2*)(dst + k) = pack_bf16(v + k);
        }
      }
      if (cm.last) {
        __syncthreads();                           // the previous tile's readers are done
#pragma unroll
        for (int k = 0; k < 16; ++k) tile[q * 16 + k][rr] = v[k];
        __syncthreads();
        float w[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) w[k] = tile[rr][q * 16 + k];
        const int64_t crow = (int64_t)cb * 64 + rr;
        const int64_t k0 = (int64_t)h * Lp + (int64_t)lb * 64 + q * 16;
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          const int64_t kk0 = k0 + u * VPC, kt = kk0 / KT, kk = kk0 - kt * KT;
          const int64_t rowid = kt * cm.last_ipad + crow;
          const int sc = store_chunk<E>(w + u * VPC, cm.last + rowid * 64 + kk * ES);
          if (E == E_FP8 && ((kk >> 4) & 1) == 0) cm.last_sc[scale_pos(rowid, (int)(kk >> 5))] = (unsigned char)sc;
        }
      }
    }
    if (cm.stage >= 0 && lead) {
      // mode N-3's chunks: piece e = (l, h, chunk) with the chunk fastest, so
      // that a wave writes the chunks of neighbouring rows h together
      __syncthreads();
      constexpr int PIECES = HB * 64 * 4 * NCH;
#pragma unroll
      for (int it = 0; it < PIECES / 256; ++it) {
        const int e = it * 256 + t;
        const int ch = e % (4 * NCH), hh = (e / (4 * NCH)) % HB, rl = e / (4 * NCH * HB);
        const IT h = hb * HB + (IT)hh, l2 = lb * 64 + (IT)rl;
        if (h < H && l2 < L) {
          IT kk;
          const IT col = cb * 64 + (IT)((ch / NCH) * 16 + (ch % NCH) * VPC);
          const int64_t rowid = lead_rowid<IT, KT>(cm, cm.stage, h * L + l2, col, INp, kk);
          *(uint4*)(cm.out[cm.stage] + rowid * 64 + kk * ES) = stg[hh][rl][ch];
        }
      }
      __syncthreads();                             // stg is rewritten by the next tile
    }
  }
}

// Zero the padding rows I..ipad-1 of every K tile of a blocked copy (and of
// its e4m3 scales).
__global__ void zero_pad_rows_kernel(char* out, unsigned char* scales, int64_t nkt, int64_t I, int64_t ipad) {
  const int64_t rows = ipad - I;
  const int64_t total = nkt * rows * 4;           // 16-byte chunks
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e & 3, rr = e >> 2;
    const int64_t kt = rr / rows, i = I + (rr - kt * rows);
    const int64_t rowid = kt * ipad + i;
    *(uint4*)(out + rowid * 64 + q * 16) = make_uint4(0, 0, 0, 0);
    if (scales && q < 2) scales[scale_pos(rowid, (int)q)] = 0;
  }
}

// The e4m3 sketch in one pass.  Row r = (K tile kt, sketch row sv) of the
// blocked Omega^T holds the values at padded columns jp = kt KT + kk, drawn
// from the sketch stream at L = sv J + j (j the unpadded column; zero in
// padded columns and rows past S; gauss_pair_e4m3), rounded to bf16 and then
// to e4m3 (the scale of each run of 32 in the layout the Gram kernel reads).  A wave takes two rows,
// a lane two neighbouring columns (one draw of a Gaussian pair when L is even).
template <class IT>
__global__ void omega_fp8_kernel(uint64_t seed, uint32_t mode, int64_t S_, int64_t J_, int64_t B_, int64_t IN_,
                                 int64_t INp_, int64_t nrows, fp8_t* q, unsigned char* scales) {
  const IT S = (IT)S_, J = (IT)J_, B = (IT)B_, IN = (IT)IN_, INp = (IT)INp_;
  const IT Bp = B > 1 ? (B / IN) * INp : 1;
  const int lane = threadIdx.x & 63, pl = lane & 31;
  for (int64_t r2 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); 2 * r2 < nrows;
       r2 += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    const int64_t r = 2 * r2 + (lane >> 5);
    const IT kt = (IT)(r >> 6), sv = (IT)(r & 63);
    const IT jp = kt * 64 + (IT)(2 * pl);             // even: jp and jp + 1 share a and bh
    IT j = jp, cols_left = J > jp ? J - jp : 0;
    bool rowok = sv < S;
    if (B > 1) {
      const IT a = jp / Bp, bp = jp - a * Bp;
      const IT bh = bp / INp, bl = bp - bh * INp;
      j = a * B + bh * IN + bl;
      cols_left = bl < IN ? IN - bl : 0;               // valid columns from jp on within this run of I_N
    }
    float v[2] = {0.f, 0.f};
    if (rowok && cols_left > 0) {
      const int64_t L = (int64_t)sv * J_ + (int64_t)j;
      float z0, z1;
      gauss_pair_e4m3((uint64_t)(L >> 1), mode, 0u, seed, z0, z1);
      if ((L & 1) == 0) {
        v[0] = z0;
        v[1] = z1;
      } else {
        v[0] = z1;
        float w0, w1;
        gauss_pair_e4m3((uint64_t)((L + 1) >> 1), mode, 0u, seed, w0, w1);
        v[1] = w0;
      }
      if (cols_left < 2) v[1] = 0.f;
      v[0] = bf16_to_f32(f32_to_bf16(v[0]));
      v[1] = bf16_to_f32(f32_to_bf16(v[1]));
    }
    // runs of 32 values: 16 lanes
    float m = fmaxf(fabsf(v[0]), fabsf(v[1]));
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    const int sc = e8m0_for(m);
    const float mul = pow2_neg(sc - 127);
    *(unsigned short*)(q + r * 64 + 2 * pl) = (unsigned short)e4m3x2(v[0] * mul, v[1] * mul);
    if ((pl & 15) == 0) {
      const int h = pl >> 4;
      scales[(int64_t)kt * 256 + (h * 32 + (int)(sv & 31)) * 4 + (int)(sv >> 5)] = (unsigned char)sc;
    }
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
  g.grid = (int)(g.ntiles * g.splits);
  g.xbase = g.splits / 8;
  g.xleft = 0;
  if (g.xcd_map && g.ntiles * best <= cu) {
    // one round, whole splits per XCD: the spare slots of the 8 XCDs take
    // as many further splits as they hold whole (their tiles on several
    // XCDs), when the cost above prefers it
    const int64_t per_xcd = cu / 8;
    const int64_t left = per_xcd - (int64_t)g.xbase * g.ntiles;
    const int64_t extra = left > 0 ? 8 * left / g.ntiles : 0;
    const int64_t s = best + extra;
    if (extra > 0 && s <= g.nkt &&
        (double)g.nkt / (double)s + 8.0 + 0.12 * (double)(g.ntiles * s) < best_cost) {
      g.splits = (int)s;
      g.xleft = (int)left;
      g.grid = (int)(8 * per_xcd);
    }
  }
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
    hipLaunchKernelGGL(gram_pipe_kernel<E_FP8>, dim3((unsigned)g.grid), dim3(256), 0, s, g);
  } else {
    hipLaunchKernelGGL(gram_pipe_kernel<E_BF16>, dim3((unsigned)g.grid), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

namespace {
bool vec_ok(const void* X, int64_t L, int es) { return (L % 4) == 0 && ((uintptr_t)X % (4 * es)) == 0; }
}  // namespace

hipError_t launch_pad_copies(int src_elem, const void* X, int64_t R, int64_t L, void* Xpad, void* Xt, hipStream_t s) {
  if (!Xpad && !Xt) return hipSuccess;
  const int64_t Lp = pad64(L), Rp = pad64(R);
  const int64_t blocks = (Rp / 64) * (Lp / 64);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  const int es = src_elem == E_F64 ? 8 : src_elem == E_F32 ? 4 : 2;
  const bool vec = vec_ok(X, L, es);
#define PC(T)                                                                                                    \
  hipLaunchKernelGGL(pad_copies_kernel<T>, grid, dim3(256), 0, s, (const T*)X, R, L, vec, (bf16_t*)Xpad, Lp,     \
                     (bf16_t*)Xt, Rp)
  switch (src_elem) {
    case E_F64: PC(double); break;
    case E_F32: PC(float); break;
    default: PC(bf16_t); break;
  }
#undef PC
  return hipGetLastError();
}

int64_t block_rows(int64_t I) { return ceil_div(I, PT) * PT; }

size_t block_copy_bytes(int64_t nkt, int64_t I) { return (size_t)nkt * block_rows(I) * PROW; }

hipError_t launch_block_copies(int src_elem, int elem, const void* X, int order, const int64_t* dims,
                               const bool* want, void* const* out, void* const* scales, void* xpad, hipStream_t s) {
  if (elem != E_FP8 && elem != E_BF16) return hipErrorInvalidValue;
  if (order < 2 || order > 8) return hipErrorInvalidValue;
  const int64_t IN = dims[order - 1], INp = pad64(IN), KT = elem == E_FP8 ? 64 : 32;
  const int64_t L = dims[order - 2], Lp = pad64(L);
  int64_t H = 1;
  for (int k = 0; k + 2 < order; ++k) H *= dims[k];
  CopyModes cm = {};
  cm.stage = -1;
  hipError_t e;
  for (int n = 0; n < order; ++n) {
    if (!want[n]) continue;
    if (!out[n] || (elem == E_FP8 && !scales[n])) return hipErrorInvalidValue;
    if (n == order - 1) {
      cm.last = (char*)out[n];
      cm.last_sc = (unsigned char*)scales[n];
      cm.last_ipad = block_rows(IN);
      continue;
    }
    int64_t A = 1, B = 1;
    for (int k = 0; k < n; ++k) A *= dims[k];
    for (int k = n + 1; k < order; ++k) B *= dims[k];
    const int m = cm.n++;
    if (n == order - 3) cm.stage = m;
    cm.I[m] = dims[n];
    cm.Bh[m] = B / IN;
    cm.ipad[m] = block_rows(dims[n]);
    cm.nbt[m] = (B / IN) * INp / KT;
    cm.out[m] = (char*)out[n];
    cm.sc[m] = (unsigned char*)scales[n];
    const int64_t nkt = A * cm.nbt[m];
    if (cm.ipad[m] > dims[n]) {
      const int64_t total = nkt * (cm.ipad[m] - dims[n]) * 4;
      const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 16384);
      hipLaunchKernelGGL(zero_pad_rows_kernel, dim3(grid), dim3(256), 0, s, (char*)out[n],
                         elem == E_FP8 ? (unsigned char*)scales[n] : nullptr, nkt, dims[n], cm.ipad[m]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (cm.n == 0 && !cm.last && !xpad) return hipSuccess;
  const int64_t ncols = cm.last ? cm.last_ipad : INp;
  const int64_t ntile = copy_ids(ceil_div(ceil_div(H, 4), COPY_HG) * (Lp / 64) * (ncols / 64));
  if (ntile <= 0) return hipSuccess;
  const int es = src_elem == E_F64 ? 8 : src_elem == E_F32 ? 4 : 2;
  const bool vec = vec_ok(X, IN, es);
  const unsigned grid = (unsigned)std::min<int64_t>(ntile, (int64_t)1 << 20);
  // 32-bit index arithmetic when every row, padded column and K index fits
  const bool small = (H + 1) * Lp * std::max(INp, ncols) < ((int64_t)1 << 31);
#define BC(T, EE, IT)                                                                                           \
  hipLaunchKernelGGL((block_copy_kernel<T, EE, IT>), dim3(grid), dim3(256), 0, s, (const T*)X, H, L, IN, INp, vec, \
                     cm, (bf16_t*)xpad)
#define BC_E(T)                                                                  \
  if (elem == E_FP8) { if (small) BC(T, E_FP8, uint32_t); else BC(T, E_FP8, uint64_t); } \
  else { if (small) BC(T, E_BF16, uint32_t); else BC(T, E_BF16, uint64_t); }
  switch (src_elem) {
    case E_F64: BC_E(double); break;
    case E_F32: BC_E(float); break;
    default: BC_E(bf16_t); break;
  }
#undef BC_E
#undef BC
  return hipGetLastError();
}

hipError_t launch_omega_fp8(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t nkt,
                            void* q, void* scales, hipStream_t s) {
  if (S > PW) return hipErrorInvalidValue;
  if (nkt <= 0) return hipSuccess;
  hipError_t e = fill_zero(scales, (size_t)nkt * 256, s);   // the bytes no row writes stay zero
  if (e != hipSuccess) return e;
  const int64_t nrows = nkt * 64;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(nrows, 8), 65535);
  if (nrows * 64 < ((int64_t)1 << 31) && S * J < ((int64_t)1 << 31))
    hipLaunchKernelGGL(omega_fp8_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), nrows, (fp8_t*)q, (unsigned char*)scales);
  else
    hipLaunchKernelGGL(omega_fp8_kernel<uint64_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), nrows, (fp8_t*)q, (unsigned char*)scales);
  return hipGetLastError();
}

hipError_t launch_gram_pipe_reduce(const GramArgs& g, double* C, double* Wt, hipStream_t s) {
  const int64_t total = (int64_t)g.ntri * PT * PT + (int64_t)g.nt * PT * PW;
  unsigned rgrid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096);
  hipLaunchKernelGGL(gram_pipe_reduce_kernel, dim3(rgrid), dim3(256), 0, s, g, C, Wt);
  return hipGetLastError();
}

hipError_t launch_omega_pad(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t Jp,
                            void* out, hipStream_t s) {
  // the row-major S x Jp layout is the blocked one with a single K tile of Jp
  // columns: [0][s][jp]
  if (Jp >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  hipError_t e = fill_zero(out, (size_t)S * Jp * 2, s);
  if (e != hipSuccess) return e;
  const int64_t npairs = (S * J + 1) / 2;
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(npairs, 256), 16384);
  if (grid == 0) return hipSuccess;
  if (S * J < ((int64_t)1 << 31) && S * Jp < ((int64_t)1 << 31))
    hipLaunchKernelGGL(omega_block_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), (int)Jp, (bf16_t*)out);
  else
    hipLaunchKernelGGL(omega_block_kernel<uint64_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), (int)Jp, (bf16_t*)out);
  return hipGetLastError();
}

hipError_t launch_omega_block(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t nkt,
                              int KT, void* out, hipStream_t s) {
  if (S > PW || (KT != 32 && KT != 64)) return hipErrorInvalidValue;
  hipError_t e = fill_zero(out, (size_t)nkt * PW * KT * 2, s);
  if (e != hipSuccess) return e;
  const int64_t npairs = (S * J + 1) / 2;
  unsigned grid = (unsigned)std::min<int64_t>(ceil_div(npairs, 256), 16384);
  if (grid == 0) return hipSuccess;
  if (S * J < ((int64_t)1 << 31) && nkt * KT < ((int64_t)1 << 31))
    hipLaunchKernelGGL(omega_block_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), KT, (bf16_t*)out);
  else
    hipLaunchKernelGGL(omega_block_kernel<uint64_t>, dim3(grid), dim3(256), 0, s, seed, (uint32_t)mode, S, J, B, IN,
                       pad64(IN), KT, (bf16_t*)out);
  return hipGetLastError();
}

}  // namespace rbki
