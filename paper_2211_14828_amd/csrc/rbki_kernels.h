// Host-side launchers of the device kernels (internal to the library).
#pragma once
#include <algorithm>
#include "rbki_common.h"

namespace rbki {

// ------------------------------------------------------------ gram.hip
struct GramArgs {
  const void* X;            // mode view source (element type of the product)
  const void* omegaT;       // S x J sketch rows (same element type), may be null if S == 0
  const unsigned char* xexp;     // fp8 pipelined form: E8M0 scales of X, [K tile][row pad][2]
  const unsigned char* xexp_om;  // fp8 pipelined form: E8M0 scales of Omega^T, [K tile][64][2]
  int64_t A, I, B, J;
  int S;
  int nt, ntri, nw, ntiles;
  int64_t nkt, nbt;
  int splits, xcd_map, vec_ok;
  int xbase, xleft, grid;    // pipelined XCD map: whole splits per XCD, spare slots per XCD, workgroups
  int thin;                 // float32, I <= 64, S <= 64: one 128 x 64 tile [C; W^T] (gram.hip)
  void* partial;            // [splits][ntiles][128*128] float (double for fp64)
  int64_t part_stride;      // elements per split (pipelined bf16 form)
  int64_t wpart_off;        // pipelined form: offset of the sketch partials within a split
  // fp8 block-exponent geometry (blocks of 32 per dimension)
  int order, mode;
  int64_t pdims[8];         // (padded) tensor dims
  int64_t nblk[8];          // blocks per dim
};

int elem_size(int elem);
int gram_bk(int elem);
GramArgs gram_plan(int elem, int64_t A, int64_t I, int64_t B, int S, int cu_count);
size_t gram_partial_bytes(const GramArgs& g, int elem);
hipError_t launch_gram_main(int elem, const GramArgs& g, hipStream_t s);
hipError_t launch_gram_reduce(int elem, const GramArgs& g, double* C, double* Wt, hipStream_t s);
hipError_t launch_omega(int elem, uint64_t seed, int mode, int64_t total, void* out, hipStream_t s);
// Pipelined bf16 / e4m3 form (gram_pipe.hip): 256 x 256 lower-triangle tiles,
// the sketch (S <= 64) computed by the spare wave of each diagonal tile.
// Operands are K-blocked copies of the mode's zero-padded unfolding (view
// [A, I, Bp], Bp a multiple of 64): [K tile][block_rows(I) rows][64 bytes],
// and the sketch [K tile][64][64 bytes]; e4m3 scales per K tile: 512 bytes per
// 256-row tile ([half][row % 32][row / 32]), the sketch's 256 ([half][row % 32][4]).
int64_t pad64(int64_t v);
bool gram_pipe_ok(int64_t I, int S);
int64_t block_rows(int64_t I);                       // I rounded up to whole 256-row tiles
size_t block_copy_bytes(int64_t nkt, int64_t I);     // nkt K tiles of block_rows(I) rows
// elem: E_BF16 or E_FP8 (K tiles of 32 or 64 values)
GramArgs gram_plan_pipe(int elem, int64_t A, int64_t I, int64_t Bp, int S, int cu_count);
size_t gram_pipe_partial_bytes(const GramArgs& g);
hipError_t launch_gram_pipe(int elem, const GramArgs& g, hipStream_t s);
hipError_t launch_gram_pipe_reduce(const GramArgs& g, double* C, double* Wt, hipStream_t s);
// X viewed as R rows of length L -> Xpad (R x pad64(L)) and Xt (L x pad64(R)),
// bf16 with zero padding (either output may be null).
hipError_t launch_pad_copies(int src_elem, const void* X, int64_t R, int64_t L, void* Xpad, void* Xt, hipStream_t s);
// Blocked copies (elem E_BF16 or E_FP8, with scales) of every mode n with
// want[n] in one pass over X (out[n], scales[n] per mode).  Leading modes
// take their K index along [A_n, (B_n / I_N) pad64(I_N)]; the last mode
// along [H, pad64(I_{N-1})] with H the product of the other leading dims.
// xpad (nullable): the row-major padded bf16 copy as well.
hipError_t launch_block_copies(int src_elem, int elem, const void* X, int order, const int64_t* dims,
                               const bool* want, void* const* out, void* const* scales, void* xpad, hipStream_t s);
// The e4m3 blocked sketch of one mode in one pass (the bf16-rounded sketch,
// quantised per run of 32 columns).
hipError_t launch_omega_fp8(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t nkt,
                            void* q, void* scales, hipStream_t s);
// Omega^T (S x J) of one mode as bf16 in the padded column layout S x Jp
// (row-major; the Gram fallback of the mixed forms).
hipError_t launch_omega_pad(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t Jp,
                            void* out, hipStream_t s);
// Omega^T (S x J, S <= 64) of one mode as bf16, blocked [nkt][64][KT] in the
// padded column order (B: the mode's trailing size, IN: the last dimension;
// B = 1 for the last mode); zero in padded columns and rows past S.
hipError_t launch_omega_block(uint64_t seed, int mode, int64_t S, int64_t J, int64_t B, int64_t IN, int64_t nkt,
                              int KT, void* out, hipStream_t s);
hipError_t launch_philox(const uint32_t* ctr, int64_t count, uint64_t seed, uint32_t* out, hipStream_t s);

// ------------------------------------------------------------ sample.hip
// Partial-column sampling (Sec. 3.1): m = round(rate J) columns of a J-column
// unfolding (all of them for rate >= 1), one per stratum
// [floor(k J / m), floor((k+1) J / m)) at a Philox-drawn offset (tag 1).
int64_t sample_count(int64_t J, double rate);
hipError_t launch_sample_columns(uint64_t seed, int mode, int64_t J, int64_t m, int64_t* cols, hipStream_t s);
// Y (I x m row-major, y_elem: x_elem, or E_BF16 rounded to nearest even)
// = the columns cols[0..m) of the view [A, I, B] of X (column j = a B + b).
hipError_t launch_gather_columns(int x_elem, const void* X, int64_t I, int64_t B, const int64_t* cols, int64_t m,
                                 int y_elem, void* Y, hipStream_t s);

// ------------------------------------------------------------ linalg.hip (float64)
// C[m x n] = alpha * op(A) op(B) + beta * C, all row-major with leading dims.
// opA: 0 -> A is m x k (lda), 1 -> A is k x m (A^T used).
// opB: 0 -> B is k x n (ldb), 1 -> B is n x k (B^T used).
hipError_t dgemm(int opA, int opB, int64_t m, int64_t n, int64_t k, double alpha, const double* A,
                 int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                 hipStream_t s);

// Orthonormalise the rows of Y (s x n, row-major: s vectors of length n) by
// CholeskyQR with column dropping, writing the result to Yout (which must not
// alias Y; Y is clobbered when s exceeds the in-LDS variant).  A pivot is
// dropped (its vector set to zero) when it falls below tau_rel times its own
// Gram diagonal or below tau_abs^2 times the largest ref2 entry.  G and Lm
// are s x s scratch; flags (int[s]) receives 1 for kept vectors; ref2
// (device, s doubles, nullable) holds squared reference norms.
//
// DimBudget caps the kept directions of a basis built block by block at the
// dimension of the space: `used_in` (device int) holds the count kept by
// the earlier blocks, at most `limit - *used_in` vectors of this block are
// kept (in order), and `*used_out = *used_in + kept` is written for the next
// block (a different slot, so every workgroup reads the same count).  The
// default (used_in == nullptr) keeps no count.
struct DimBudget {
  const int* used_in = nullptr;
  int* used_out = nullptr;
  int64_t limit = 0;
  __device__ int64_t allowed() const { return used_in ? limit - *used_in : (int64_t)1 << 62; }
  __device__ void record(int64_t kept) const {
    if (used_out) *used_out = (int)((used_in ? *used_in : 0) + kept);
  }
};
hipError_t chol_orth(double* Y, double* Yout, int64_t s, int64_t n, double* G, double* Lm, int* flags,
                     const double* ref2, double tau_rel, double tau_abs, hipStream_t st, DimBudget bud = {});

// Scratch for split-K float64 GEMMs (nullptr disables split-K).
void dgemm_set_scratch(double* p, size_t bytes);

// Row norms squared of Y (s x n) -> out[s].
hipError_t row_norms2(const double* Y, int64_t s, int64_t n, double* out, hipStream_t st);

// One-sided Jacobi on the columns of symmetric PSD Z (n x n, row-major
// input); writes the eigenvalues (descending) to lam[n] and the matching unit
// eigenvectors as the rows of Vt (n x n row-major).  work: scratch of
// jacobi_work_bytes(n).  info (device int): 0 ok, >0 sweep limit reached.
size_t jacobi_work_bytes(int64_t n);
hipError_t jacobi_eig(const double* Z, int64_t n, double* lam, double* Vt, void* work, int* info,
                      int max_sweeps, hipStream_t st);
// The same for up to 8 matrices in one launch (each with its own scratch;
// info[k] points at two ints per matrix).  per_matrix: one workgroup per
// matrix in an ordinary launch instead of the cooperative grid (same
// results; lets solves on other streams run beside it).
hipError_t jacobi_eig_batched(int nmat, const double* const* Z, const int64_t* n, double* const* lam,
                              double* const* Vt, void* const* work, int* const* info, int max_sweeps,
                              hipStream_t st, bool per_matrix = false);

// The R largest eigenpairs of symmetric PSD n x n matrices (eig_top.hip):
// Householder tridiagonalisation (one or more workgroups per matrix),
// multisection and inverse iteration.  lam[k] receives R eigenvalues
// (descending), rows 0..R-1 of Vt[k] (leading dimension n) the unit
// eigenvectors.  Only the upper triangle of Z is read.  info[k] (nullable)
// gets {0, 0}, or info[k][0] = 1 when the workgroups of a reduction did not
// meet within the barrier's spin limit.  coop: a cooperative launch for the
// multi-workgroup reduction; false gives an ordinary launch, for a solve
// enqueued beside other work.
bool eig_top_ok(int64_t n, int64_t R);                  // 1 <= R <= n <= 512
size_t eig_top_work_bytes(int64_t n, int64_t R);
hipError_t eig_top_batched(int nmat, const double* const* Z, const int64_t* n, const int64_t* R,
                           double* const* lam, double* const* Vt, void* const* work, int* const* info,
                           hipStream_t st, bool coop = true);

// Copy / convert helpers.
hipError_t copy_rows_f64(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows,
                         int64_t cols, hipStream_t st);
hipError_t store_factor(const double* Ut /* R x I */, int64_t R, int64_t I, void* out /* I x R */,
                        int out_elem, hipStream_t st);
hipError_t fill_zero(void* p, size_t bytes, hipStream_t st);
// Flip each row of V (rows x n) so its largest-magnitude entry is positive.
hipError_t canonical_sign_rows(double* V, int64_t rows, int64_t n, hipStream_t st);

// ------------------------------------------------------------ ttm.hip
// Y[a, r, b] = sum_i U[i, r] X[a, i, b] for the view [A, I, B] of X;
// U given as Ut (R x I row-major, element type of the product).
// X element type elem; Y written as float (F32/BF16 products) or double (F64).
hipError_t launch_ttm(int elem, const void* X, int64_t A, int64_t I, int64_t B, const void* Ut,
                      int64_t R, void* Y, void* work, size_t work_bytes, hipStream_t s);
size_t ttm_work_bytes(int elem, int64_t A, int64_t I, int64_t B, int64_t R);
// The same product in bf16 on the zero-padded copy Xpad (rows of the last
// dimension IN padded to pad64(IN)); Y is written in the unpadded layout.
hipError_t launch_ttm_padded(const void* Xpad, int64_t A, int64_t I, int64_t B, int64_t IN, const void* Ut,
                             int64_t R, void* Y, hipStream_t s);

// First mode product of the precision forms from a leading mode's blocked
// copy xb (E_FP8 with its scales, or E_BF16), view [A, I, B] of X with last
// dimension IN: Y[a, r, b] = sum_i U[i, r] X[a, i, b] as float, R <= 64.
// Ut: R x I float64; U16: scratch of 64 x block_rows(I) bfloat16.
hipError_t launch_ttm_first_blocked(int elem, const void* xb, const void* scales, int64_t A, int64_t I,
                                    int64_t B, int64_t IN, const double* Ut, int64_t R, void* U16, void* Y,
                                    hipStream_t s);

// Sum over all entries of (X - Uh)^2 and X^2 where Uh[i, j] = sum_r U[i, r] H[r, j]
// (X viewed as I x J row-major, the mode-0 unfolding); partial sums in
// float64, returned in out[0] (residual) and out[1] (norm), reduced in a fixed order.
// bf16_products: the streaming form forms U H from split bfloat16 operands
// (hi + lo parts, relative error about 2^-16).
hipError_t launch_residual(int x_elem, const void* X, int op_elem, const void* Ut, const void* H,
                           int64_t I, int64_t J, int64_t R, double* out, void* work,
                           size_t work_bytes, hipStream_t s, bool bf16_products = false);
size_t residual_work_bytes(int64_t I, int64_t J);

// ------------------------------------------------------------ chain.hip
// The Krylov chain of one mode (blocks j0..j1 of Alg. 1 by the Gram route,
// then Z over the first zr basis rows) run by one workgroup; one launch runs
// up to kChainJobs such instances.  Every pointer is the instance's own
// (float64, row-major): C (I x I) and, for block 0, W^T in Yt (S x I) as left
// by the Gram pass; scratch Yt, Ytmp (S x I), Pm (S x Sp), G (S x S); outputs
// Qt and CQ (rows j S .. (j+1) S - 1 of block j, I wide; CQ holds Q_j C) and
// Z (zr x zr); used: the q + 2 direction counters.
constexpr int kChainJobs = 8;
struct ChainJob {
  const double* C;
  double* Yt;
  double* Ytmp;
  double* Pm;
  double* G;
  double* CQ;
  double* Qt;
  double* Z;
  int* used;
  int I, S, zr;
};
struct ChainArgs {
  ChainJob job[kChainJobs];
  int j0, j1;
  int power;                 // power iteration: one block, replaced at every step
  double tau_rel, tau_abs;
};
bool krylov_chain_ok(int64_t I, int64_t S);
hipError_t launch_krylov_chain(const ChainArgs& a, int njobs, hipStream_t st);

// Element conversions of the whole tensor.
hipError_t convert_tensor(int src_elem, const void* src, int dst_elem, void* dst, int64_t n,
                          hipStream_t s);

}  // namespace rbki
