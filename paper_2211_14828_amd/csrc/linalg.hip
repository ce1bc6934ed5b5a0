// Float64 dense linear algebra on small matrices (the Krylov basis, the
// projected matrix Z and its eigenvectors).  Every routine here works on
// matrices of at most a few thousand rows/columns and runs entirely on the
// device.
#include <hip/hip_cooperative_groups.h>
#include <cstdlib>

#include "rbki_kernels.h"

namespace cg = cooperative_groups;

namespace rbki {

namespace {

// ------------------------------------------------------------------ DGEMM
// 64 x 64 output tile per 256-thread workgroup, 4 x 4 outputs per thread,
// K staged through LDS in steps of 16.
constexpr int GT = 64, GK = 16;

__global__ void __launch_bounds__(256) dgemm_kernel(int opA, int opB, int64_t m, int64_t n, int64_t k,
                                                    double alpha, const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb, double beta,
                                                    double* __restrict__ C, int64_t ldc, double* __restrict__ part,
                                                    int64_t kchunk) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t row0 = (int64_t)blockIdx.y * GT, col0 = (int64_t)blockIdx.x * GT;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = kb + kchunk < k ? kb + kchunk : k;
  // this thread's four elements of each staged tile: A (i, kk), B (kk, j)
  int ai[4], ak[4], bk[4], bj[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = threadIdx.x + 256 * t;
    if (opA == 0) { ai[t] = e / GK; ak[t] = e % GK; } else { ak[t] = e / GT; ai[t] = e % GT; }
    if (opB == 0) { bk[t] = e / GT; bj[t] = e % GT; } else { bj[t] = e / GK; bk[t] = e % GK; }
  }
  // the next K tile is loaded into registers while the current one is
  // multiplied, so only the first tile's memory latency is exposed
  double ra[4], rb[4];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t r = row0 + ai[t], c = k0 + ak[t];
      ra[t] = (r < m && c < ke) ? (opA == 0 ? A[r * lda + c] : A[c * lda + r]) : 0.0;
      const int64_t r2 = k0 + bk[t], c2 = col0 + bj[t];
      rb[t] = (r2 < ke && c2 < n) ? (opB == 0 ? B[r2 * ldb + c2] : B[c2 * ldb + r2]) : 0.0;
    }
  };
  double acc[4][4] = {};
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      As[ak[t]][ai[t]] = ra[t];
      Bs[bk[t]][bj[t]] = rb[t];
    }
    __syncthreads();
    if (k0 + GK < ke) fetch(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty + 16 * u];
        b[u] = Bs[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = row0 + ty + 16 * u, c = col0 + tx + 16 * v;
      if (r < m && c < n) {
        if (part) {
          part[(int64_t)blockIdx.z * m * n + r * n + c] = acc[u][v];
        } else {
          double* p = C + r * ldc + c;
          *p = beta == 0.0 ? alpha * acc[u][v] : alpha * acc[u][v] + beta * *p;
        }
      }
    }
}

// C = alpha * sum_z part[z] + beta * C, summed in a fixed order.
__global__ void dgemm_reduce_kernel(int64_t m, int64_t n, int splits, const double* part, double alpha, double beta,
                                    double* C, int64_t ldc) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m * n; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int z = 0; z < splits; ++z) acc += part[(int64_t)z * m * n + e];
    const int64_t r = e / n, c = e - r * n;
    double* p = C + r * ldc + c;
    *p = beta == 0.0 ? alpha * acc : alpha * acc + beta * *p;
  }
}

// ------------------------------------------------------------ Cholesky QR
// Right-looking Cholesky of the s x s Gram matrix G in LDS with column
// dropping, then the inverse of the (reduced) factor, one workgroup.  A pivot
// d_k (the Schur-complement diagonal) is dropped, with its row and column of
// the factor set to zero, when d_k <= tau_rel * G_kk (the vector lies within
// the span of the earlier kept ones to working accuracy) or
// d_k <= tau_abs^2 * max_k ref2[k] (it is at round-off level relative to the
// block before projection).  Writes Linv (s x s, zero rows/columns for dropped
// vectors) and flags[k] = 1 for kept vectors.
constexpr int CHOL_MAX = 96;

__global__ void __launch_bounds__(1024) chol_inv_kernel(const double* G, int64_t s, double* Linv, int* flags,
                                                        const double* ref2, double tau_rel, double tau_abs,
                                                        DimBudget bud) {
  __shared__ double Ls[CHOL_MAX][CHOL_MAX + 1];
  __shared__ double Xs[CHOL_MAX][CHOL_MAX + 1];
  __shared__ double d0[CHOL_MAX];
  __shared__ int keep[CHOL_MAX];
  __shared__ double red[16];
  __shared__ double sh_ref;
  const int tid = threadIdx.x;
  double mx = 0.0;
  if (ref2)
    for (int64_t i = tid; i < s; i += blockDim.x) mx = fmax(mx, ref2[i]);
  mx = warp_max(mx);
  if ((tid & 63) == 0) red[tid >> 6] = mx;
  for (int e = tid; e < (int)(s * s); e += blockDim.x) {
    const int i = e / (int)s, j = e - i * (int)s;
    Ls[i][j] = G[e];
    if (i == j) d0[i] = G[e];
  }
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
    sh_ref = v;
  }
  __syncthreads();
  const double abs_floor = tau_abs * tau_abs * sh_ref;
  const int64_t allowed = bud.allowed();
  int64_t nkept = 0;
  for (int k = 0; k < s; ++k) {
    const double d = Ls[k][k];
    const int kp = (d0[k] > 0.0) && (d > tau_rel * d0[k]) && (d > abs_floor) && nkept < allowed;
    nkept += kp;
    const double piv = kp ? sqrt(d) : 0.0;
    __syncthreads();
    for (int i = k + tid; i < s; i += blockDim.x) Ls[i][k] = kp ? (i == k ? piv : Ls[i][k] / piv) : 0.0;
    if (tid == 0) keep[k] = kp;
    __syncthreads();
    if (kp) {
      const int t = s - k - 1;
      for (int e = tid; e < t * t; e += blockDim.x) {
        const int i = k + 1 + e / t, j = k + 1 + e % t;
        if (j <= i) Ls[i][j] -= Ls[i][k] * Ls[j][k];
      }
    }
    __syncthreads();
  }
  // X = L^{-1} restricted to kept rows/columns, right-looking: starting from
  // the identity, row k is scaled by 1 / L_kk and then removed from the rows
  // below it.  Only columns c <= k of a row are nonzero at step k.  A dropped
  // k has a zero factor column, so its row and column of X stay zero.
  const int sn = (int)s;
  for (int e = tid; e < sn * sn; e += blockDim.x) {
    const int i = e / sn, j = e - i * sn;
    Xs[i][j] = (i == j && keep[i]) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < sn; ++k) {
    if (keep[k]) {
      const double inv = 1.0 / Ls[k][k];
      for (int c = tid; c <= k; c += blockDim.x) Xs[k][c] *= inv;
    }
    __syncthreads();
    if (keep[k]) {
      const int w = k + 1, t = sn - k - 1;
      for (int e = tid; e < t * w; e += blockDim.x) {
        const int i = k + 1 + e / w, c = e - (e / w) * w;
        Xs[i][c] -= Ls[i][k] * Xs[k][c];
      }
    }
    __syncthreads();
  }
  // a dropped row k of L still holds its entries left of the diagonal, which
  // reached row k of X above: dropped vectors get a zero row
  for (int e = tid; e < sn * sn; e += blockDim.x) {
    const int i = e / sn, j = e - i * sn;
    Linv[e] = keep[i] ? Xs[i][j] : 0.0;
  }
  for (int64_t i = tid; i < s; i += blockDim.x) flags[i] = keep[i];
  if (tid == 0) bud.record(nkept);
}

// CholeskyQR step for s <= 64 in one launch: Yout = L^{-1} Y where G = L L^T
// (same drop rule as above: a dropped vector gets a zero row of Yout).
// One wave per workgroup, 64 columns of Y each; every workgroup factors G
// itself, so no workgroup waits for another.  G is zero-padded to SMAX in LDS
// (a padded pivot is dropped and changes nothing), and the factor runs in
// panels of 16 columns: lane i holds row i of the panel in registers and
// reads the finished column k from the lane that holds it (v_readlane), then
// the wave applies the panel to the trailing rows and columns in 4 x 4 tiles.
// Every entry receives its updates in column order, one FMA each, as in the
// unblocked right-looking form.  The pivot is d * rsqrt(d) and its reciprocal
// the Newton-refined rsqrt itself.  Then each lane solves L y = Y(:, c) for
// its column c by forward substitution, with y in registers and L read by LDS
// broadcast, four rows per branch.  Loads of G and Y are clamped into range
// so they are all issued before the first wait.  flags is written by
// workgroup 0.
constexpr int CS_MAX = 64;
constexpr int CS_NB = 16;

__device__ inline double lane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

template <int SMAX>
__global__ void __launch_bounds__(64) chol_solve_kernel(const double* G, int s, const double* Y, int64_t n,
                                                        double* Yout, int* flags, const double* ref2,
                                                        double tau_rel, double tau_abs, DimBudget bud) {
  static_assert(SMAX % CS_NB == 0, "panels of 16 columns");
  __shared__ double Ls[SMAX][SMAX + 1];
  __shared__ double dinv[SMAX];
  __shared__ int keep[SMAX];
  const int lane = threadIdx.x;
  {
    double gv[SMAX * SMAX / 64];
#pragma unroll
    for (int q = 0; q < SMAX * SMAX / 64; ++q) {
      const int e = lane + 64 * q, i = e / SMAX, j = e - i * SMAX;
      gv[q] = G[(i < s ? i : s - 1) * s + (j < s ? j : s - 1)];
    }
#pragma unroll
    for (int q = 0; q < SMAX * SMAX / 64; ++q) {
      const int e = lane + 64 * q, i = e / SMAX, j = e - i * SMAX;
      Ls[i][j] = (i < s && j < s) ? gv[q] : 0.0;
    }
  }
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  const int64_t cc = c < n ? c : n - 1;
  double y[SMAX];
#pragma unroll
  for (int k = 0; k < SMAX; ++k) y[k] = Y[(int64_t)(k < s ? k : s - 1) * n + cc];
  const double mx = warp_max((ref2 && lane < s) ? ref2[lane] : 0.0);
  const double abs_floor = tau_abs * tau_abs * mx;
  const int64_t allowed = bud.allowed();
  __syncthreads();
  const double d0 = lane < SMAX ? Ls[lane][lane] : 0.0;
  int64_t nkept = 0;
#pragma unroll 1
  for (int c0 = 0; c0 < SMAX; c0 += CS_NB) {
    {
      const int i = lane;
      double r[CS_NB];
#pragma unroll
      for (int jj = 0; jj < CS_NB; ++jj) r[jj] = i < SMAX ? Ls[i][c0 + jj] : 0.0;
#pragma unroll
      for (int kk = 0; kk < CS_NB; ++kk) {
        const int k = c0 + kk;
        const double v = r[kk];           // G(i, k) minus the earlier columns' terms
        const double d = lane_f64(v, k), dk0 = lane_f64(d0, k);
        const bool kp = (dk0 > 0.0) && (d > tau_rel * dk0) && (d > abs_floor) && nkept < allowed;
        nkept += kp;
        const double rs = rsq_nr(kp ? d : 1.0);
        const double inv = kp ? rs : 0.0;
        const double lik = i > k ? v * inv : (i == k ? d * inv : 0.0);
        r[kk] = lik;
        if (i == k) {
          keep[k] = kp;
          dinv[k] = inv;
        }
#pragma unroll
        for (int jj = kk + 1; jj < CS_NB; ++jj) r[jj] -= lik * lane_f64(lik, c0 + jj);
      }
      if (i < SMAX) {
#pragma unroll
        for (int jj = 0; jj < CS_NB; ++jj) Ls[i][c0 + jj] = r[jj];
      }
    }
    __syncthreads();
    // trailing rows and columns t0.. of the lower triangle's square, 4 x 4
    // tiles (the upper part is updated too and never read)
    const int t0 = c0 + CS_NB, mt = (SMAX - t0) / 4;
    for (int t = lane; t < mt * mt; t += 64) {
      const int ti = t / mt, tj = t - ti * mt;
      const int i0 = t0 + 4 * ti, j0 = t0 + 4 * tj;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[a][q] = Ls[i0 + a][j0 + q];
#pragma unroll
      for (int kk = 0; kk < CS_NB; ++kk) {
        double li[4], lj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          li[a] = Ls[i0 + a][c0 + kk];
          lj[a] = Ls[j0 + a][c0 + kk];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[a][q] -= li[a] * lj[q];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) Ls[i0 + a][j0 + q] = acc[a][q];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    if (lane < s) flags[lane] = keep[lane];
    // every workgroup reads the count of earlier blocks; one writes the total
    if (lane == 0) bud.record(nkept);
  }
#pragma unroll
  for (int k0 = 0; k0 < SMAX; k0 += 4) {
    if (k0 < s) {
#pragma unroll
      for (int k = k0; k < k0 + 4; ++k) {
        double a0 = y[k], a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int j = 0; j + 3 < k; j += 4) {
          a0 -= Ls[k][j] * y[j];
          a1 -= Ls[k][j + 1] * y[j + 1];
          a2 -= Ls[k][j + 2] * y[j + 2];
          a3 -= Ls[k][j + 3] * y[j + 3];
        }
#pragma unroll
        for (int j = k & ~3; j < k; ++j) a0 -= Ls[k][j] * y[j];
        y[k] = ((a0 + a1) + (a2 + a3)) * dinv[k];   // zero for a dropped or padded vector
      }
      if (c < n) {
#pragma unroll
        for (int k = k0; k < k0 + 4; ++k)
          if (k < s) Yout[(int64_t)k * n + c] = y[k];
      }
    }
  }
}

// Left-looking Cholesky of the s x s Gram matrix G with column dropping, one
// workgroup, for s beyond the LDS variant (same drop rule).
__global__ void __launch_bounds__(1024) chol_drop_kernel(const double* G, int64_t s, double* L, int* flags,
                                                         const double* ref2, double tau_rel, double tau_abs,
                                                         DimBudget bud) {
  __shared__ double red[16];
  __shared__ double sh_ref;
  __shared__ int sh_keep;
  __shared__ double sh_piv;
  const int tid = threadIdx.x;
  double mx = 0.0;
  if (ref2)
    for (int64_t i = tid; i < s; i += blockDim.x) mx = fmax(mx, ref2[i]);
  mx = warp_max(mx);
  if ((tid & 63) == 0) red[tid >> 6] = mx;
  __syncthreads();
  if (tid == 0) {
    double v = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
    sh_ref = v;
  }
  for (int64_t i = tid; i < s * s; i += blockDim.x) L[i] = 0.0;
  __syncthreads();
  const double abs_floor = tau_abs * tau_abs * sh_ref;
  const int64_t allowed = bud.allowed();
  int64_t nkept = 0;                               // meaningful in thread 0
  for (int64_t kc = 0; kc < s; ++kc) {
    if (tid == 0) {
      double d = G[kc * s + kc];
      for (int64_t j = 0; j < kc; ++j) d -= L[kc * s + j] * L[kc * s + j];
      const double gkk = G[kc * s + kc];
      const int keep = (gkk > 0.0) && (d > tau_rel * gkk) && (d > abs_floor) && nkept < allowed;
      nkept += keep;
      sh_keep = keep;
      sh_piv = keep ? sqrt(d) : 0.0;
      flags[kc] = keep;
      if (keep) L[kc * s + kc] = sh_piv;
    }
    __syncthreads();
    if (sh_keep) {
      const double piv = sh_piv;
      for (int64_t i = kc + 1 + tid; i < s; i += blockDim.x) {
        double v = G[i * s + kc];
        for (int64_t j = 0; j < kc; ++j) v -= L[i * s + j] * L[kc * s + j];
        L[i * s + kc] = v / piv;
      }
    }
    __syncthreads();
  }
  if (tid == 0) bud.record(nkept);
}

// Y (s x n rows) <- L^{-1} Y row-wise (forward substitution along the s
// vectors), one thread per column; dropped vectors become zero.
__global__ void trsm_rows_kernel(double* Y, int64_t s, int64_t n, const double* L, const int* flags) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t kc = 0; kc < s; ++kc) {
      if (!flags[kc]) {
        Y[kc * n + c] = 0.0;
        continue;
      }
      double v = Y[kc * n + c];
      for (int64_t j = 0; j < kc; ++j)
        if (flags[j]) v -= L[kc * s + j] * Y[j * n + c];
      Y[kc * n + c] = v / L[kc * s + kc];
    }
  }
}

__global__ void row_norms2_kernel(const double* Y, int64_t s, int64_t n, double* out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= s) return;
  double acc = 0.0;
  for (int64_t c = lane; c < n; c += 64) {
    const double v = Y[row * n + c];
    acc = fma(v, v, acc);
  }
  acc = warp_sum(acc);
  if (lane == 0) out[row] = acc;
}

// ------------------------------------------------------------ Jacobi
// Block one-sided (Hestenes) Jacobi on the columns of symmetric PSD matrices,
// several matrices per launch.  The columns of each matrix are split into
// nblk blocks of nb columns (zero-padded).  Rounds follow the circle method
// over blocks: in each round a workgroup takes one pair of blocks and stages
// their 2 nb columns P in LDS.  It forms the small Gram matrix G = P^T P once,
// diagonalises it by cyclic two-sided Jacobi sweeps on G itself while
// accumulating the rotation V (the rotation angles come from three entries of
// G instead of three length-n dot products), and applies P <- P V once.  The
// nblk - 1 rounds of a sweep are separated by grid barriers.  A matrix is done
// when a whole sweep met no pair of its columns with |cos| above tol.  At
// convergence A = Z V has orthogonal columns a_j = lambda_j v_j: eigenvalues
// are the column norms and eigenvectors the normalised columns.
constexpr int JAC_MAXB = 8;    // matrices per launch
constexpr int JAC_APPLY_MAX = 5;   // 16 x 16 output blocks per wave in the apply phase

struct JacobiArgs {
  double* A[JAC_MAXB];         // npad x n column-major working copies
  int64_t n[JAC_MAXB];
  int nblk[JAC_MAXB];
  int* info[JAC_MAXB];         // info[0]: 0 or sweeps at the limit, info[1]: sweeps used
  int nmat, nb, npos, max_nblk;
  int64_t ld;
  int max_sweeps, inner_sweeps;
  double tol;
  unsigned long long* offmax;  // [3][JAC_MAXB] per-sweep max |cos| bit patterns
  unsigned long long* prof;    // nullable: phase clocks of workgroup 0 (diagnostics)
};

// Circle ordering: position pos (0 <= pos < nblk) holds this element in round
// `round` (0 <= round < nblk - 1); position 0 is fixed, the others rotate.
__device__ inline int circle_block(int pos, int round, int nblk) {
  if (pos == 0) return 0;
  int v = pos - 1 + round;              // < 2 (nblk - 1)
  if (v >= nblk - 1) v -= nblk - 1;
  return 1 + v;
}


// Rotation (c, s) zeroing the (p, q) entry of a 2x2 Gram block
// [al ga; ga be]: new_p = c p - s q, new_q = s p + c q.  Returns false when
// |ga| <= tol sqrt(al be) (the pair is already orthogonal to tolerance).
// The rotation is the standard one: zeta = (be - al) / (2 ga),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t.
__device__ inline bool jacobi_rotation(double al, double be, double ga, double tol, double& c, double& s,
                                       double& cosang) {
  c = 1.0;
  s = 0.0;
  al = fmax(al, 0.0);
  be = fmax(be, 0.0);
  if (!(al > 1e-300 && be > 1e-300)) { cosang = 0.0; return false; }
  cosang = fabs(ga) * rsq_nr(al) * rsq_nr(be);
  if (cosang <= tol) return false;
  const double zeta = (be - al) * rcp_nr(2.0 * ga);
  const double z2 = fma(zeta, zeta, 1.0);
  const double root = z2 < 1e300 ? z2 * rsq_nr(z2) : fabs(zeta);   // sqrt(1 + zeta^2)
  const double tm = rcp_nr(fabs(zeta) + root);
  const double t = zeta >= 0.0 ? tm : -tm;
  c = rsq_nr(fma(t, t, 1.0));
  s = c * t;
  return true;
}

// COOP: one workgroup per (matrix, pair position), rounds separated by grid
// barriers (cooperative launch).  !COOP: one workgroup per matrix walks every
// position of a round itself; an ordinary launch, so that solves on other
// streams can run beside it.  The pairs of a round touch disjoint columns and
// every pair does the same arithmetic in either form, so the two give
// bit-identical results.
template <bool COOP>
__global__ void __launch_bounds__(1024) jacobi_kernel(JacobiArgs J) {
  extern __shared__ double sm[];
  __shared__ double sh_off[16];
  __shared__ int sh_done[JAC_MAXB];
  __shared__ double rot_c[16], rot_s[16];
  __shared__ int rot_p[16], rot_q[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = COOP ? blockIdx.x / J.npos : blockIdx.x;
  const int pos0 = COOP ? blockIdx.x % J.npos : 0;
  const int nb = J.nb, two = 2 * nb;
  const int nbk = (two + 15) / 16;                 // 16-wide MFMA blocks across the pair
  const int64_t n = J.n[m];
  const int64_t ld = J.ld;                         // odd stride >= n: conflict-free column reads
  double* P = sm;                                  // columns-major [two][ld]
  double* G = P + (int64_t)two * ld;               // [two][two + 1]
  double* V = G + two * (two + 1);
  double* S = V + two * (two + 1);                 // Gram partials [16][256]
  const int gs = two + 1;
  if (tid < JAC_MAXB) sh_done[tid] = 0;
  __syncthreads();
  int sweep;
  for (sweep = 0; sweep < J.max_sweeps; ++sweep) {
    if (COOP && blockIdx.x == 0 && tid < J.nmat) J.offmax[((sweep + 1) % 3) * JAC_MAXB + tid] = 0ull;
    double local_off = 0.0;
    const int npos_m = J.nblk[m] / 2;
    const bool mine = !sh_done[m] && pos0 < npos_m;
    const int pos_end = COOP ? pos0 + 1 : npos_m;
    for (int round = 0; round < (COOP ? J.max_nblk : J.nblk[m]) - 1; ++round) {
      for (int pos = pos0; pos < pos_end; ++pos) {
      unsigned long long t0 = wall_clock64();
      if (mine && round < J.nblk[m] - 1) {
        const int bp = circle_block(pos, round, J.nblk[m]);
        const int bq = circle_block(J.nblk[m] - 1 - pos, round, J.nblk[m]);
        double* A = J.A[m];
        for (int c = wave; c < two; c += 16) {
          const int gc = c < nb ? bp * nb + c : bq * nb + (c - nb);
          const double* src = A + (int64_t)gc * n;
          for (int64_t r = lane; r < n; r += 64) P[c * ld + r] = src[r];
        }
        __syncthreads();
        unsigned long long t1 = wall_clock64();
        // G = P^T P on fp64 MFMA 16x16x4: wave w takes output block (w % nbk^2)
        // and K slice (w / nbk^2); slices are summed through LDS.
        {
          const int nblk2 = nbk * nbk;
          const int nslice = 16 / nblk2;
          const int blk = wave % nblk2, sl = wave / nblk2;
          const int bi = blk / nbk, bj = blk % nbk;
          const int i = bi * 16 + (lane & 15), j = bj * 16 + (lane & 15);
          const int64_t ksteps = (n + 3) / 4;
          const int64_t k0 = ksteps * sl / nslice, k1 = ksteps * (sl + 1) / nslice;
          f64x4_t d = {0.0, 0.0, 0.0, 0.0};
          for (int64_t kt = k0; kt < k1; ++kt) {
            const int64_t r = kt * 4 + (lane >> 4);
            const double a = (i < two && r < n) ? P[i * ld + r] : 0.0;
            const double b = (j < two && r < n) ? P[j * ld + r] : 0.0;
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) S[(sl * nblk2 + blk) * 256 + (4 * v + (lane >> 4)) * 16 + (lane & 15)] = d[v];
          __syncthreads();
          for (int e = tid; e < two * two; e += blockDim.x) {
            const int ii = e / two, jj = e % two;
            const int b2 = (ii >> 4) * nbk + (jj >> 4);
            double acc = 0.0;
            for (int q = 0; q < nslice; ++q) acc += S[(q * nblk2 + b2) * 256 + (ii & 15) * 16 + (jj & 15)];
            G[ii * gs + jj] = acc;
            V[ii * gs + jj] = ii == jj ? 1.0 : 0.0;
          }
          __syncthreads();
        }
        unsigned long long t2 = wall_clock64();
        // inner cyclic sweep on G (two-sided), accumulating V.  In each step
        // lanes k < nb of wave 0 form the rotation of pair k once and publish
        // it in LDS; then, in one phase, thread t < nb^2 applies both
        // rotations of its 2 x 2 block of G (rows of pair t / nb, columns of
        // pair t % nb: G' = J^T G J restricted to that block), and the next
        // 2 nb^2 threads apply the column rotations to V.  The pairs partition
        // the indices, so every entry has exactly one writer.
        {
          for (int isw = 0; isw < J.inner_sweeps; ++isw) {
            double inner_off = 0.0;
            for (int ir = 0; ir < two - 1; ++ir) {
              if (tid < nb) {
                const int p = circle_block(tid, ir, two);
                const int q = circle_block(two - 1 - tid, ir, two);
                double c, s, ca;
                jacobi_rotation(G[p * gs + p], G[q * gs + q], G[p * gs + q], J.tol, c, s, ca);
                inner_off = fmax(inner_off, ca);
                rot_c[tid] = c;
                rot_s[tid] = s;
                rot_p[tid] = p;
                rot_q[tid] = q;
              }
              __syncthreads();
              if (tid < nb * nb) {
                const int k1 = tid / nb, k2 = tid - k1 * nb;
                const double c1 = rot_c[k1], s1 = rot_s[k1], c2 = rot_c[k2], s2 = rot_s[k2];
                if (s1 != 0.0 || s2 != 0.0) {
                  const int a0 = rot_p[k1], a1 = rot_q[k1], b0 = rot_p[k2], b1 = rot_q[k2];
                  const double g00 = G[a0 * gs + b0], g01 = G[a0 * gs + b1];
                  const double g10 = G[a1 * gs + b0], g11 = G[a1 * gs + b1];
                  // rows: p' = c1 p - s1 q, q' = s1 p + c1 q
                  const double h00 = c1 * g00 - s1 * g10, h01 = c1 * g01 - s1 * g11;
                  const double h10 = s1 * g00 + c1 * g10, h11 = s1 * g01 + c1 * g11;
                  // columns: p' = c2 p - s2 q, q' = s2 p + c2 q
                  G[a0 * gs + b0] = c2 * h00 - s2 * h01;
                  G[a0 * gs + b1] = s2 * h00 + c2 * h01;
                  G[a1 * gs + b0] = c2 * h10 - s2 * h11;
                  G[a1 * gs + b1] = s2 * h10 + c2 * h11;
                }
              } else if (tid < nb * nb + two * nb) {
                const int e = tid - nb * nb;
                const int i = e / nb, k = e - i * nb;
                const double c = rot_c[k], sn = rot_s[k];
                if (sn != 0.0) {
                  const int p = rot_p[k], q = rot_q[k];
                  const double vp = V[i * gs + p], vq = V[i * gs + q];
                  V[i * gs + p] = c * vp - sn * vq;
                  V[i * gs + q] = sn * vp + c * vq;
                }
              }
              __syncthreads();
            }
            if (wave == 0) {
              const double w = warp_max(inner_off);
              if (lane == 0) sh_off[0] = w;
            }
            __syncthreads();
            const double mx = sh_off[0];
            __syncthreads();
            if (isw == 0) local_off = fmax(local_off, mx);
            if (mx <= J.tol) break;
          }
        }
        unsigned long long t3 = wall_clock64();
        // A(:, pair) <- P V on fp64 MFMA: 16 x 16 output blocks over
        // (row block, column block), K = two.  The blocks are held in
        // registers until every wave has finished reading P, written back
        // into P, and then copied out column by column (coalesced).
        {
          const int64_t rblocks = (n + 15) / 16;
          const int64_t nblocks = rblocks * nbk;   // <= 16 * JAC_APPLY_MAX (host check)
          f64x4_t d[JAC_APPLY_MAX];
#pragma unroll
          for (int it = 0; it < JAC_APPLY_MAX; ++it) {
            d[it] = f64x4_t{0.0, 0.0, 0.0, 0.0};
            const int64_t ob = wave + 16 * it;
            if (ob < nblocks) {
              const int64_t rb = ob / nbk;
              const int cb = (int)(ob % nbk);
              const int64_t r = rb * 16 + (lane & 15);
              const int j = cb * 16 + (lane & 15);
              for (int kt = 0; kt < (two + 3) / 4; ++kt) {
                const int k = kt * 4 + (lane >> 4);
                const double a = (r < n && k < two) ? P[k * ld + r] : 0.0;
                const double b = (j < two && k < two) ? V[k * gs + j] : 0.0;
                d[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d[it], 0, 0, 0);
              }
            }
          }
          __syncthreads();
#pragma unroll
          for (int it = 0; it < JAC_APPLY_MAX; ++it) {
            const int64_t ob = wave + 16 * it;
            if (ob < nblocks) {
              const int64_t rb = ob / nbk;
              const int cb = (int)(ob % nbk);
              const int jo = cb * 16 + (lane & 15);
              if (jo < two) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                  const int64_t ro = rb * 16 + 4 * v + (lane >> 4);
                  if (ro < n) P[jo * ld + ro] = d[it][v];
                }
              }
            }
          }
          __syncthreads();
          for (int c = wave; c < two; c += 16) {
            const int gc = c < nb ? bp * nb + c : bq * nb + (c - nb);
            double* dst = A + (int64_t)gc * n;
            for (int64_t r = lane; r < n; r += 64) dst[r] = P[c * ld + r];
          }
        }
        __threadfence();
        if (J.prof && blockIdx.x == 0 && tid == 0) {
          unsigned long long t4 = wall_clock64();
          J.prof[0] += t1 - t0;
          J.prof[1] += t2 - t1;
          J.prof[2] += t3 - t2;
          J.prof[3] += t4 - t3;
          J.prof[5] += 1;
        }
        if (!COOP) __syncthreads();               // P, G and V are reused by the next position
      }
      }
      if constexpr (COOP) {
        unsigned long long tg = wall_clock64();
        cg::this_grid().sync();
        if (J.prof && blockIdx.x == 0 && tid == 0) J.prof[4] += wall_clock64() - tg;
      }
    }
    if constexpr (!COOP) {
      // local_off is uniform across the workgroup: the sweep's largest |cos|
      // over every pair of this matrix
      if (!sh_done[m] && local_off <= J.tol && tid == 0) {
        J.info[m][0] = 0;
        J.info[m][1] = sweep + 1;
      }
      __syncthreads();
      if (local_off <= J.tol) {
        if (tid == 0) sh_done[m] = 1;
        break;
      }
      continue;
    }
    // publish this workgroup's largest |cos| of the sweep (first inner sweep of
    // each round: the state before any rotation of that round)
    if (tid == 0 && mine)
      atomicMax(&J.offmax[(sweep % 3) * JAC_MAXB + m], (unsigned long long)__double_as_longlong(local_off));
    __threadfence();
    cg::this_grid().sync();
    if (tid < J.nmat && !sh_done[tid]) {
      const double v = __longlong_as_double(
          (long long)__atomic_load_n(&J.offmax[(sweep % 3) * JAC_MAXB + tid], __ATOMIC_RELAXED));
      if (v <= J.tol) {
        sh_done[tid] = 1;
        if (blockIdx.x == 0) {
          J.info[tid][0] = 0;
          J.info[tid][1] = sweep + 1;
        }
      }
    }
    __syncthreads();
    bool all = true;
    for (int k = 0; k < J.nmat; ++k) all = all && sh_done[k];
    if (all) break;
  }
  if (COOP && blockIdx.x == 0 && tid < J.nmat && !sh_done[tid]) {
    J.info[tid][0] = sweep;
    J.info[tid][1] = sweep;
  }
  if (!COOP && tid == 0 && !sh_done[m]) {
    J.info[m][0] = sweep;
    J.info[m][1] = sweep;
  }
}

// Column norms of the converged A, then a rank sort (descending, ties by
// index) and normalised columns as rows of Vt.  One workgroup per matrix.
struct FinishArgs {
  const double* A[JAC_MAXB];
  int64_t n[JAC_MAXB];
  double* lam[JAC_MAXB];
  double* Vt[JAC_MAXB];
  double* norms[JAC_MAXB];
};

__global__ void jacobi_finish_kernel(FinishArgs F) {
  const int m = blockIdx.x;
  const double* A = F.A[m];
  const int64_t n = F.n[m];
  double* lam = F.lam[m];
  double* Vt = F.Vt[m];
  double* norms = F.norms[m];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  for (int64_t j = wave; j < n; j += nwaves) {
    double acc = 0.0;
    for (int64_t r = lane; r < n; r += 64) acc = fma(A[j * n + r], A[j * n + r], acc);
    acc = warp_sum(acc);
    if (lane == 0) norms[j] = sqrt(acc);
  }
  __syncthreads();
  for (int64_t j = tid; j < n; j += blockDim.x) {
    const double v = norms[j];
    int64_t rank = 0;
    for (int64_t i = 0; i < n; ++i) {
      const double w = norms[i];
      rank += (w > v) || (w == v && i < j);
    }
    lam[rank] = v;
    norms[n + j] = (double)rank;
  }
  __syncthreads();
  for (int64_t e = tid; e < n * n; e += blockDim.x) {
    const int64_t j = e / n, r = e - j * n;
    const int64_t dst = (int64_t)norms[n + j];
    const double nv = norms[j];
    Vt[dst * n + r] = nv > 0.0 ? A[j * n + r] / nv : 0.0;
  }
}

__global__ void pad_copy_kernel(const double* Z, int64_t n, int64_t npad, double* A) {
  // A column-major n x npad: column j = row j of Z (Z symmetric), zero beyond n
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npad * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / n, r = e - j * n;
    A[e] = j < n ? Z[j * n + r] : 0.0;
  }
}

__global__ void copy_rows_kernel(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows,
                                 int64_t cols) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

template <class T>
__global__ void store_factor_kernel(const double* Ut, int64_t R, int64_t I, T* out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < R * I;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R, r = e - i * R;
    out[e] = (T)Ut[r * I + i];
  }
}

// Sign rule for singular/eigen vectors: flip each row of V (rows x n) so that
// its largest-magnitude entry (lowest index on ties) is positive.  One wave per row.
__global__ void canonical_sign_rows_kernel(double* V, int64_t rows, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= rows) return;
  double* v = V + row * n;
  double best = -1.0;
  int64_t bi = n;
  for (int64_t c = lane; c < n; c += 64) {
    const double a = fabs(v[c]);
    if (a > best) { best = a; bi = c; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if (best <= 0.0 || bi >= n) return;
  const double sgn = v[bi] < 0.0 ? -1.0 : 1.0;
  if (sgn < 0.0)
    for (int64_t c = lane; c < n; c += 64) v[c] = -v[c];
}

__global__ void fill_zero_kernel(unsigned* p, size_t words) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < words; e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

inline unsigned grid_for(int64_t work, int64_t per = 256, int64_t cap = 8192) {
  int64_t g = ceil_div(work, per);
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

}  // namespace

// per host thread: the scratch of the call being enqueued by that thread
static thread_local double* g_dgemm_scratch = nullptr;
static thread_local size_t g_dgemm_scratch_bytes = 0;

void dgemm_set_scratch(double* p, size_t bytes) {
  g_dgemm_scratch = p;
  g_dgemm_scratch_bytes = bytes;
}

hipError_t dgemm(int opA, int opB, int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t tiles = ceil_div(m, GT) * ceil_div(n, GT);
  int64_t splits = ceil_div(256, tiles);
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, k / 64));
  splits = std::min<int64_t>(splits, 64);
  if (g_dgemm_scratch == nullptr) splits = 1;
  while (splits > 1 && (size_t)splits * m * n * 8 > g_dgemm_scratch_bytes) --splits;
  const int64_t kchunk = splits > 1 ? ceil_div(ceil_div(k, splits), GK) * GK : std::max<int64_t>(k, 1);
  splits = splits > 1 ? ceil_div(k, kchunk) : 1;
  dim3 grid((unsigned)ceil_div(n, GT), (unsigned)ceil_div(m, GT), (unsigned)splits);
  double* part = splits > 1 ? g_dgemm_scratch : nullptr;
  hipLaunchKernelGGL(dgemm_kernel, grid, dim3(256), 0, s, opA, opB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                     part, kchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  hipLaunchKernelGGL(dgemm_reduce_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(m * n, 256), 4096)), dim3(256), 0, s,
                     m, n, (int)splits, part, alpha, beta, C, ldc);
  return hipGetLastError();
}

hipError_t row_norms2(const double* Y, int64_t s, int64_t n, double* out, hipStream_t st) {
  if (s <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_norms2_kernel, dim3((unsigned)ceil_div(s, 4)), dim3(256), 0, st, Y, s, n, out);
  return hipGetLastError();
}

hipError_t chol_orth(double* Y, double* Yout, int64_t s, int64_t n, double* G, double* Lm, int* flags,
                     const double* ref2, double tau_rel, double tau_abs, hipStream_t st, DimBudget bud) {
  if (s <= 0) return hipSuccess;
  hipError_t e = dgemm(0, 1, s, s, n, 1.0, Y, n, Y, n, 0.0, G, s, st);
  if (e != hipSuccess) return e;
  if (s <= CS_MAX) {
    const dim3 grid((unsigned)ceil_div(n, 64));
    if (s <= 16)
      hipLaunchKernelGGL(chol_solve_kernel<16>, grid, dim3(64), 0, st, G, (int)s, Y, n, Yout, flags, ref2, tau_rel,
                         tau_abs, bud);
    else if (s <= 32)
      hipLaunchKernelGGL(chol_solve_kernel<32>, grid, dim3(64), 0, st, G, (int)s, Y, n, Yout, flags, ref2, tau_rel,
                         tau_abs, bud);
    else if (s <= 48)
      hipLaunchKernelGGL(chol_solve_kernel<48>, grid, dim3(64), 0, st, G, (int)s, Y, n, Yout, flags, ref2, tau_rel,
                         tau_abs, bud);
    else
      hipLaunchKernelGGL(chol_solve_kernel<64>, grid, dim3(64), 0, st, G, (int)s, Y, n, Yout, flags, ref2, tau_rel,
                         tau_abs, bud);
    return hipGetLastError();
  }
  if (s <= CHOL_MAX) {
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), 0, st, G, s, Lm, flags, ref2, tau_rel, tau_abs, bud);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return dgemm(0, 0, s, n, s, 1.0, Lm, s, Y, n, 0.0, Yout, n, st);
  }
  hipLaunchKernelGGL(chol_drop_kernel, dim3(1), dim3(1024), 0, st, G, s, Lm, flags, ref2, tau_rel, tau_abs, bud);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(trsm_rows_kernel, dim3(grid_for(n)), dim3(256), 0, st, Y, s, n, Lm, flags);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return copy_rows_f64(Yout, n, Y, n, s, n, st);
}

// Block width: the staged pair (2 nb columns of length n), G, V and the
// Gram partials (16 x 256 doubles) must fit in 160 KB of LDS.
static size_t jacobi_lds_bytes(int64_t n, int nb) {
  const int two = 2 * nb;
  const int64_t ld = (n & 1) ? n : n + 1;
  return (size_t)(two * ld + 2 * two * (two + 1) + 16 * 256) * 8;
}

static void jacobi_geometry(int64_t n, int& nb, int& nblk) {
  nb = 16;
  while (nb > 2 && jacobi_lds_bytes(n, nb) > 160 * 1024 - 1024) nb /= 2;
  if (n <= 2 * nb) nb = (int)std::max<int64_t>(1, (n + 1) / 2);
  nblk = (int)ceil_div(n, nb);
  if (nblk < 2) nblk = 2;
  if (nblk & 1) ++nblk;
}

size_t jacobi_work_bytes(int64_t n) {
  // npad <= n + 2 * nb <= n + 32, so this bound grows with n and covers every
  // smaller matrix that reuses the same scratch
  return (size_t)((n + 32) * n * 8 + 2 * n * 8 + 256);  // A, norms/ranks, offmax
}

hipError_t jacobi_eig_batched(int nmat, const double* const* Z, const int64_t* ns, double* const* lam,
                              double* const* Vt, void* const* work, int* const* info, int max_sweeps, hipStream_t st,
                              bool per_matrix) {
  if (nmat <= 0) return hipSuccess;
  if (nmat > JAC_MAXB) return hipErrorInvalidValue;
  int64_t nmax = 0;
  for (int k = 0; k < nmat; ++k) nmax = std::max(nmax, ns[k]);
  int nb, nblk_dummy;
  jacobi_geometry(nmax, nb, nblk_dummy);
  if (ceil_div(nmax, 16) * ceil_div(2 * nb, 16) > 16 * JAC_APPLY_MAX) return hipErrorInvalidValue;
  JacobiArgs ja = {};
  FinishArgs fa = {};
  ja.nmat = nmat;
  ja.nb = nb;
  ja.max_sweeps = max_sweeps;
  ja.inner_sweeps = 1;
  if (const char* e = getenv("RBKI_JACOBI_INNER")) ja.inner_sweeps = std::max(1, atoi(e));
  ja.tol = 1e-12;
  ja.max_nblk = 2;
  hipError_t e;
  for (int k = 0; k < nmat; ++k) {
    const int64_t n = ns[k];
    int nbk = (int)ceil_div(n, nb);
    if (nbk < 2) nbk = 2;
    if (nbk & 1) ++nbk;
    const int64_t npad = (int64_t)nb * nbk;
    char* w = (char*)work[k];
    ja.A[k] = (double*)w;
    ja.n[k] = n;
    ja.nblk[k] = nbk;
    ja.info[k] = info[k];
    ja.max_nblk = std::max(ja.max_nblk, nbk);
    fa.A[k] = ja.A[k];
    fa.n[k] = n;
    fa.lam[k] = lam[k];
    fa.Vt[k] = Vt[k];
    fa.norms[k] = (double*)(w + npad * n * 8);
    hipLaunchKernelGGL(pad_copy_kernel, dim3(grid_for(npad * n)), dim3(256), 0, st, Z[k], n, npad, ja.A[k]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // the convergence slots live after matrix 0's scratch
  {
    int nb0 = (int)ceil_div(ns[0], nb);
    if (nb0 < 2) nb0 = 2;
    if (nb0 & 1) ++nb0;
    (void)nb0;
  }
  ja.offmax = (unsigned long long*)((char*)work[0] + jacobi_work_bytes(ns[0]) - 256);
  ja.prof = getenv("RBKI_JACOBI_PROF") ? ja.offmax + 3 * JAC_MAXB : nullptr;   // 6 slots after offmax
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, st, (unsigned*)ja.offmax, (size_t)(3 * JAC_MAXB * 2 + 12));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  ja.npos = ja.max_nblk / 2;
  ja.ld = (nmax & 1) ? nmax : nmax + 1;
  const size_t shmem = jacobi_lds_bytes(nmax, nb);
  if (per_matrix) {
    e = hipFuncSetAttribute((const void*)jacobi_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shmem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(jacobi_kernel<false>, dim3(nmat), dim3(1024), shmem, st, ja);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else {
    e = hipFuncSetAttribute((const void*)jacobi_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shmem);
    if (e != hipSuccess) return e;
    void* args[] = {&ja};
    e = hipLaunchCooperativeKernel((const void*)jacobi_kernel<true>, dim3(ja.npos * nmat), dim3(1024), args, shmem,
                                   st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(nmat), dim3(1024), 0, st, fa);
  return hipGetLastError();
}

hipError_t jacobi_eig(const double* Z, int64_t n, double* lam, double* Vt, void* work, int* info, int max_sweeps,
                      hipStream_t st) {
  const double* Zs[1] = {Z};
  int64_t ns[1] = {n};
  double* ls[1] = {lam};
  double* vs[1] = {Vt};
  void* ws[1] = {work};
  int* is[1] = {info};
  return jacobi_eig_batched(1, Zs, ns, ls, vs, ws, is, max_sweeps, st);
}

hipError_t copy_rows_f64(double* dst, int64_t ldd, const double* src, int64_t lds, int64_t rows, int64_t cols,
                         hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_rows_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, st, dst, ldd, src, lds, rows, cols);
  return hipGetLastError();
}

hipError_t store_factor(const double* Ut, int64_t R, int64_t I, void* out, int out_elem, hipStream_t st) {
  if (out_elem == E_F64)
    hipLaunchKernelGGL(store_factor_kernel<double>, dim3(grid_for(R * I)), dim3(256), 0, st, Ut, R, I, (double*)out);
  else
    hipLaunchKernelGGL(store_factor_kernel<float>, dim3(grid_for(R * I)), dim3(256), 0, st, Ut, R, I, (float*)out);
  return hipGetLastError();
}

hipError_t canonical_sign_rows(double* V, int64_t rows, int64_t n, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(canonical_sign_rows_kernel, dim3((unsigned)ceil_div(rows, 4)), dim3(256), 0, st, V, rows, n);
  return hipGetLastError();
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for((int64_t)(bytes / 4))), dim3(256), 0, st, (unsigned*)p, bytes / 4);
  return hipGetLastError();
}

}  // namespace rbki
