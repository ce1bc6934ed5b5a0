// The Krylov chain of small modes in one persistent launch (Alg. 1 with the
// Gram route of Remark 1, and Z of Alg. 2, step 3).
//
// After the Gram pass of mode n has left C = X_(n) X_(n)^T (I x I) and the
// sketch W^T = (X_(n) Omega)^T (S x I) in memory, the rest of the mode's
// Krylov work is a chain of small float64 products and factorisations whose
// cost, run as separate launches, is launch and memory latency.  Here one
// workgroup runs a whole chain, and one launch runs the chains of many
// instances (the modes of one decomposition): workgroup b takes instance b.
// Each block j of the basis is made exactly as by the separate launches:
//
//   block 0:  Y = W^T;
//   block j:  Y = (C Q_{j-1})^T, then twice Y -= (Y Q^T) Q over the earlier
//             blocks (classical Gram-Schmidt, repeated);
//   then CholeskyQR2 of Y: G = Y Y^T = L L^T, Y <- L^{-1} Y, twice, the first
//   pass with the drop rule (a pivot below tau_rel G_kk, below
//   tau_abs^2 max ||y_k||^2 of the block before projection, or past the
//   direction budget I is dropped: its row becomes zero), giving Q_j;
//   then (C Q_j)^T = Q_j C, kept for block j+1 and for Z.
// Finally Z = Q (C Q) over the first zr rows of the basis.  Power iteration
// (Sec. 3.1) runs the same steps on one block, replaced at every step, with
// no projection and no direction budget after block 0.
//
// Products.  All products are formed by the workgroup's four waves on the
// float64 matrix cores (v_mfma_f64_16x16x4f64) with operands read straight
// from memory: the matrices of one instance (at most 256 x 256 for C, and
// blocks of at most 64 x 256) stay in the caches between steps.  On gfx950
// the instruction takes A(i, k) from lane i + 16 k, B(k, j) from lane
// j + 16 k, and returns D(r + 4 v, j) in item v of lane j + 16 r (checked on
// the device).  A wave owns 32 x 32 output blocks (16 x 16 when the output
// has fewer than eight blocks of 32), sums its K loop in a fixed order, and
// loads the next four K steps while it multiplies the current ones.
//
// Factor.  The s x s Gram matrix of a CholeskyQR pass is factored in LDS by
// wave 0 (left-looking: column k is G(i, k) - sum_{j<k} L(i, j) L(k, j),
// subtracted in increasing j, the pivot read from lane k), then each thread
// solves L y = Y(:, c) for its columns c by forward substitution with y in
// registers.
//
// Scratch per instance: Yt, Ytmp (S x I), Pm (S x Sp), G (S x S); the basis
// Qt (Sp x I), its products CQ (Sp x I) and Z (zr x zr) are outputs.  The
// direction counters used[0 .. q+1] are the ones the separate launches keep.
#include "rbki_kernels.h"

namespace rbki {
namespace {

constexpr int CH_THREADS = 512;
constexpr int CH_WAVES = CH_THREADS / 64;

__device__ inline double lane_value(double v, int k) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), k),
                          __builtin_amdgcn_readlane(__double2loint(v), k));
}

__device__ inline double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// C = alpha op(A) op(B) + beta C with op(A)(i, k) = A[i sai + k sak] and
// op(B)(k, j) = B[k sbk + j sbj] (a transpose swaps the two strides).
struct GemmOp {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int64_t sai, sak, sbk, sbj, ldc;
  double alpha, beta;
};

__device__ inline GemmOp op(int M, int N, int K, double alpha, const double* A, int lda, bool ta, const double* B,
                            int ldb, bool tb, double beta, double* C, int ldc) {
  GemmOp g;
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.sai = ta ? 1 : lda;
  g.sak = ta ? lda : 1;
  g.sbk = tb ? 1 : ldb;
  g.sbj = tb ? ldb : 1;
  g.ldc = ldc;
  g.alpha = alpha;
  g.beta = beta;
  return g;
}

typedef double d2u_t __attribute__((ext_vector_type(2), aligned(8)));

// KS consecutive values p[t * stride] (p at k = k0), t < KS, zero past K.
template <int KS>
__device__ inline void load_run(const double* p, int64_t stride, int k0, int K, bool in, double (&out)[KS]) {
  if (in && stride == 1 && k0 + KS <= K) {
#pragma unroll
    for (int t = 0; t < KS; t += 2) {
      const d2u_t v = *(const d2u_t*)(p + t);
      out[t] = v.x;
      out[t + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < KS; ++t) out[t] = (in && k0 + t < K) ? p[t * stride] : 0.0;
  }
}

// One wave's output block of (16 RB) x (16 CB) at (r0, c0); sub-blocks past
// M or N are skipped (a wave-uniform test, so the MFMAs run with every lane).
// A stage covers 4 KS values of k: lane group g = lane / 16 holds
// k = k0 + KS g + t, t < KS, of its row of op(A) and column of op(B), and
// MFMA step t multiplies the four values k0 + KS g + t, g < 4 (the same
// order of k for both operands, so the sum is the product; an operand that
// is contiguous along k is read KS values at a time).  The next stage is
// loaded while the current one is multiplied.
template <int RB, int CB, int KS>
__device__ inline void wave_block(const GemmOp& g, int r0, int c0, int lane) {
  const int li = lane & 15, lg = lane >> 4;
  bool rv[RB], cv[CB];
#pragma unroll
  for (int u = 0; u < RB; ++u) rv[u] = r0 + 16 * u < g.M;
#pragma unroll
  for (int v = 0; v < CB; ++v) cv[v] = c0 + 16 * v < g.N;
  f64x4_t acc[RB][CB];
#pragma unroll
  for (int u = 0; u < RB; ++u)
#pragma unroll
    for (int v = 0; v < CB; ++v) acc[u][v] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  const double* pa[RB];
  const double* pb[CB];
  bool ia[RB], jb[CB];
#pragma unroll
  for (int u = 0; u < RB; ++u) {
    const int i = r0 + 16 * u + li;
    ia[u] = i < g.M;
    pa[u] = g.A + (int64_t)(ia[u] ? i : 0) * g.sai;
  }
#pragma unroll
  for (int v = 0; v < CB; ++v) {
    const int j = c0 + 16 * v + li;
    jb[v] = j < g.N;
    pb[v] = g.B + (int64_t)(jb[v] ? j : 0) * g.sbj;
  }
  constexpr int KST = 4 * KS;
  // the lane's first k, and the pointer steps of a stage
#pragma unroll
  for (int u = 0; u < RB; ++u) pa[u] += (int64_t)(KS * lg) * g.sak;
#pragma unroll
  for (int v = 0; v < CB; ++v) pb[v] += (int64_t)(KS * lg) * g.sbk;
  const int64_t da = (int64_t)KST * g.sak, db = (int64_t)KST * g.sbk;
  double a0[RB][KS], b0[CB][KS], a1[RB][KS], b1[CB][KS];
  auto load = [&](double (&aa)[RB][KS], double (&bb)[CB][KS], int k0) {
    const int kb = k0 + KS * lg;
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      load_run<KS>(pa[u], g.sak, kb, g.K, ia[u], aa[u]);
      pa[u] += da;
    }
#pragma unroll
    for (int v = 0; v < CB; ++v) {
      load_run<KS>(pb[v], g.sbk, kb, g.K, jb[v], bb[v]);
      pb[v] += db;
    }
  };
  auto mul = [&](const double (&aa)[RB][KS], const double (&bb)[CB][KS]) {
#pragma unroll
    for (int t = 0; t < KS; ++t)
#pragma unroll
      for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int v = 0; v < CB; ++v)
          if (rv[u] && cv[v]) acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[u][t], bb[v][t], acc[u][v], 0, 0, 0);
  };
  const int nst = (g.K + KST - 1) / KST;
  if (nst > 0) load(a0, b0, 0);
  int st = 0;
  for (; st + 2 <= nst; st += 2) {
    load(a1, b1, KST * (st + 1));
    mul(a0, b0);
    if (st + 2 < nst) load(a0, b0, KST * (st + 2));
    mul(a1, b1);
  }
  if (st < nst) mul(a0, b0);
#pragma unroll
  for (int u = 0; u < RB; ++u)
#pragma unroll
    for (int v = 0; v < CB; ++v) {
      const int col = c0 + 16 * v + li;
      if (!rv[u] || !cv[v] || col >= g.N) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = r0 + 16 * u + lg + 4 * t;
        if (row < g.M) {
          double* p = g.C + (int64_t)row * g.ldc + col;
          *p = g.beta == 0.0 ? g.alpha * acc[u][v][t] : g.alpha * acc[u][v][t] + g.beta * *p;
        }
      }
    }
}

// The whole workgroup's product; the caller synchronises before the result
// is read.  32 x 32 blocks (16 values of k a stage) when there is at least
// one per wave, else 16 x 16 blocks (32 values of k a stage).
__device__ __noinline__ void wg_gemm(GemmOp g) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int mb = (g.M + 31) / 32, nb = (g.N + 31) / 32;
  if (mb * nb >= CH_WAVES) {
    for (int blk = wave; blk < mb * nb; blk += CH_WAVES)
      wave_block<2, 2, 4>(g, (blk / nb) * 32, (blk % nb) * 32, lane);
  } else {
    const int mb16 = (g.M + 15) / 16, nb16 = (g.N + 15) / 16;
    for (int blk = wave; blk < mb16 * nb16; blk += CH_WAVES)
      wave_block<1, 1, 8>(g, (blk / nb16) * 16, (blk % nb16) * 16, lane);
  }
}

constexpr int CH_SMAX = 64;
__shared__ double ch_L[CH_SMAX][CH_SMAX + 1];
__shared__ double ch_dinv[CH_SMAX];
__shared__ double ch_ref2[CH_SMAX];

// Squared norms of the s rows of Y (s x n) into ch_ref2.
__device__ __noinline__ void wg_row_norms2(const double* Y, int s, int n) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int r = wave; r < s; r += CH_WAVES) {
    double acc = 0.0;
    for (int c = lane; c < n; c += 64) {
      const double v = Y[(int64_t)r * n + c];
      acc = fma(v, v, acc);
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) ch_ref2[r] = acc;
  }
  __syncthreads();
}

// The factor of one CholeskyQR pass: G (s x s, symmetric) = L L^T by wave 0,
// lane i holding row i in registers (left-looking: column k is
// G(i, k) - sum_{j<k} L(i, j) L(k, j), with row k of L read from LDS, where
// lane k left it, and the pivot from lane k), with the drop rule (use_ref:
// the absolute floor from ch_ref2, the squared row norms of the block before
// projection); then L^{-1} by forward substitution on the unit vectors, lane
// c taking column c.  A dropped pivot gives a zero row and column of L and a
// zero row of L^{-1}.  L^{-1} overwrites G (s x s, row-major).
template <int SMAX>
__device__ __noinline__ void wg_chol_inv(double* G, int s, bool use_ref, double tau_rel, double tau_abs,
                                         DimBudget bud) {
  const int tid = threadIdx.x;
  for (int e = tid; e < s * s; e += CH_THREADS) {
    const int i = e / s, j = e - i * s;
    ch_L[i][j] = G[e];
  }
  __syncthreads();
  if (tid < 64) {
    const int i = tid;
    const bool row_ok = i < s;
    double mx = (use_ref && row_ok) ? ch_ref2[i] : 0.0;
    mx = warp_max(mx);
    const double abs_floor = tau_abs * tau_abs * mx;
    double row[SMAX];
#pragma unroll
    for (int j = 0; j < SMAX; ++j) row[j] = (row_ok && j < s) ? ch_L[i][j] : 0.0;
    const double d0 = row_ok ? ch_L[i][i] : 0.0;
    const int64_t allowed = bud.allowed();
    int64_t nkept = 0;
#pragma unroll
    for (int k = 0; k < SMAX; ++k) {
      if (k < s) {
        double v0 = row[k], v1 = 0.0;
#pragma unroll
        for (int j = 0; j + 1 < k; j += 2) {
          v0 -= row[j] * ch_L[k][j];
          v1 -= row[j + 1] * ch_L[k][j + 1];
        }
        if (k & 1) v0 -= row[k - 1] * ch_L[k][k - 1];
        const double v = v0 + v1;
        const double d = lane_value(v, k), dk0 = lane_value(d0, k);
        const bool kp = (dk0 > 0.0) && (d > tau_rel * dk0) && (d > abs_floor) && nkept < allowed;
        nkept += kp;
        const double piv = kp ? sqrt(d) : 0.0;
        const double inv = kp ? 1.0 / piv : 0.0;
        const double lik = (i > k && row_ok) ? v * inv : (i == k ? piv : 0.0);
        row[k] = lik;
        if (row_ok) ch_L[i][k] = lik;
        if (i == k) ch_dinv[k] = inv;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    if (i == 0) bud.record(nkept);
    // column c = i of L^{-1}
    double x[SMAX];
#pragma unroll
    for (int k = 0; k < SMAX; ++k) {
      if (k < s) {
        double a0 = i == k ? 1.0 : 0.0, a1 = 0.0;
#pragma unroll
        for (int j = 0; j + 1 < k; j += 2) {
          a0 -= ch_L[k][j] * x[j];
          a1 -= ch_L[k][j + 1] * x[j + 1];
        }
        if (k & 1) a0 -= ch_L[k][k - 1] * x[k - 1];
        x[k] = (a0 + a1) * ch_dinv[k];
        if (row_ok) G[(int64_t)k * s + i] = x[k];
      }
    }
  }
  __syncthreads();
}

template <int SMAX>
__global__ void __launch_bounds__(CH_THREADS) krylov_chain_kernel(ChainArgs a) {
  const ChainJob jb = a.job[blockIdx.x];
  const int I = jb.I, S = jb.S;
  const int64_t blk = (int64_t)S * I;
  for (int j = a.j0; j <= a.j1; ++j) {
    // power iteration keeps one block, replaced at every step
    const int64_t off = a.power ? 0 : j * blk;
    double* Qj = jb.Qt + off;
    if (j == 0) {
      wg_row_norms2(jb.Yt, S, I);
    } else {
      // Y = (C Q_{j-1})^T, kept from the previous block
      const double* prev = jb.CQ + (a.power ? 0 : (j - 1) * blk);
      for (int64_t e = threadIdx.x; e < blk; e += CH_THREADS) jb.Yt[e] = prev[e];
      __syncthreads();
      wg_row_norms2(jb.Yt, S, I);
      const int m = S * j;
      for (int pass = 0; pass < 2 && !a.power; ++pass) {
        wg_gemm(op(S, m, I, 1.0, jb.Yt, I, false, jb.Qt, I, true, 0.0, jb.Pm, m));
        __syncthreads();
        wg_gemm(op(S, I, m, -1.0, jb.Pm, m, false, jb.Qt, I, false, 1.0, jb.Yt, I));
        __syncthreads();
      }
    }
    // CholeskyQR2: Ytmp = L^{-1} Y with the drop rule, then Q_j = L^{-1} Ytmp
    wg_gemm(op(S, S, I, 1.0, jb.Yt, I, false, jb.Yt, I, true, 0.0, jb.G, S));
    __syncthreads();
    wg_chol_inv<SMAX>(jb.G, S, true, a.tau_rel, a.tau_abs,
                      (a.power && j > 0) ? DimBudget{} : DimBudget{jb.used + j, jb.used + j + 1, I});
    wg_gemm(op(S, I, S, 1.0, jb.G, S, false, jb.Yt, I, false, 0.0, jb.Ytmp, I));
    __syncthreads();
    wg_gemm(op(S, S, I, 1.0, jb.Ytmp, I, false, jb.Ytmp, I, true, 0.0, jb.G, S));
    __syncthreads();
    wg_chol_inv<SMAX>(jb.G, S, false, a.tau_rel, 0.0, DimBudget{});
    wg_gemm(op(S, I, S, 1.0, jb.G, S, false, jb.Ytmp, I, false, 0.0, Qj, I));
    __syncthreads();
    // (C Q_j)^T = Q_j C (C symmetric)
    wg_gemm(op(S, I, I, 1.0, Qj, I, false, jb.C, I, false, 0.0, jb.CQ + off, I));
    __syncthreads();
  }
  if (jb.zr > 0) wg_gemm(op(jb.zr, jb.zr, I, 1.0, jb.Qt, I, false, jb.CQ, I, true, 0.0, jb.Z, jb.zr));
}

}  // namespace

bool krylov_chain_ok(int64_t I, int64_t S) { return I >= 1 && I <= 256 && S >= 1 && S <= CH_SMAX; }

hipError_t launch_krylov_chain(const ChainArgs& a, int njobs, hipStream_t st) {
  if (njobs < 1 || njobs > kChainJobs) return hipErrorInvalidValue;
  int smax = 0;
  for (int i = 0; i < njobs; ++i) {
    if (!krylov_chain_ok(a.job[i].I, a.job[i].S)) return hipErrorInvalidValue;
    smax = std::max(smax, a.job[i].S);
  }
  if (smax <= 16)
    hipLaunchKernelGGL(krylov_chain_kernel<16>, dim3(njobs), dim3(CH_THREADS), 0, st, a);
  else if (smax <= 32)
    hipLaunchKernelGGL(krylov_chain_kernel<32>, dim3(njobs), dim3(CH_THREADS), 0, st, a);
  else if (smax <= 48)
    hipLaunchKernelGGL(krylov_chain_kernel<48>, dim3(njobs), dim3(CH_THREADS), 0, st, a);
  else
    hipLaunchKernelGGL(krylov_chain_kernel<64>, dim3(njobs), dim3(CH_THREADS), 0, st, a);
  return hipGetLastError();
}

}  // namespace rbki
