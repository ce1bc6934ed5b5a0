// The R leading eigenpairs of small symmetric positive semidefinite float64
// matrices: the small eigenproblem of Alg. 2, steps 4-5, where only the R
// eigenvectors of Z = Q^T X_(n) X_(n)^T Q that become factor columns are
// needed.  The method is the textbook dense one for a few eigenpairs:
//
//  1. Householder reduction Z = H T H^T to a symmetric tridiagonal T.  The
//     upper triangle is held in LDS, its rows dealt round-robin to G
//     workgroups (G = 1 up to n of about 165).  The rank-2 update of step k
//     is fused with the matrix-vector product of step k+1; with G > 1 the
//     workgroups exchange their partial products and the next reflector's row
//     through a small global buffer once per step.
//  2. The R largest eigenvalues of T by multisection on Sturm counts (the
//     number of negative pivots of the LDL^T factorisation of T - x I equals
//     the number of eigenvalues below x), one wave per eigenvalue testing
//     128 points a round, in a kernel of its own.
//  3. Their eigenvectors of T by inverse iteration: a pivoted LU of
//     T - lambda I per eigenvalue, one thread each, three solves.  Eigenvalues
//     closer than 1e-3 ||T|| form a cluster whose vectors are
//     re-orthogonalised (modified Gram-Schmidt) after every solve.
//  4. Back-transformation by the Householder reflectors, one wave per vector.
//
// Results are deterministic: every sum is taken in a fixed order.
#include <cfloat>
#include <cstdlib>

#include "rbki_kernels.h"

namespace rbki {
namespace {

constexpr int EIG_MAXB = 8;
constexpr int EIG_NS_MAX = 8;                // n <= 64 * EIG_NS_MAX
constexpr int SOLVE_THREADS = 512;          // eigenvalue / eigenvector workgroup (R <= 512)
constexpr int SOLVE_WAVES = SOLVE_THREADS / 64;
constexpr int EIG_ITERS = 3;                 // inverse-iteration solves
constexpr int RED_THREADS = 1024;            // reduction workgroup
constexpr int RED_WAVES = RED_THREADS / 64;
constexpr int RED_GMAX = 32;                 // workgroups per matrix at most
constexpr size_t LDS_BYTES = 160 * 1024;
constexpr unsigned SPIN_LIMIT = 1u << 20;    // barrier polls before giving up (default)
constexpr double EPS = 0x1p-53;              // unit roundoff of float64

struct EigArgs {
  const double* Z[EIG_MAXB];
  int n[EIG_MAXB], R[EIG_MAXB];
  double* A[EIG_MAXB];       // n x n working copy; row k holds reflector k after the reduction
  double* d[EIG_MAXB];       // diagonal of T (n)
  double* e[EIG_MAXB];       // off-diagonal of T (n, last entry 0)
  double* tau[EIG_MAXB];     // reflector scalars (n)
  double* X[EIG_MAXB];       // eigenvectors of T, [r][i] (R x n)
  double* Y[EIG_MAXB];       // forward-substitution results, [r][i]
  double* ainv[EIG_MAXB];    // LU of T - lambda I per eigenvalue, [i][R]: 1 / U(i,i)
  double* bu[EIG_MAXB];      //   U(i, i+1)
  double* du[EIG_MAXB];      //   U(i, i+2)
  double* cm[EIG_MAXB];      //   multiplier of L at step i
  unsigned char* piv[EIG_MAXB];  // row interchange at step i
  double* lam[EIG_MAXB];
  double* Vt[EIG_MAXB];
  int* info[EIG_MAXB];
  int G[EIG_MAXB];           // workgroups sharing the reduction
  double* P[EIG_MAXB];       // exchange of partial products, [2][G][n]
  double* RB[EIG_MAXB];      // exchange of the next reflector's row, [2][n]
  unsigned* cnt[EIG_MAXB];   // barrier counter (zero at launch)
  unsigned spin_limit;       // barrier polls before giving up; 0: give up at the first barrier
};

// Value of element idx of a vector spread as x[t] = v[64 t + lane].
template <int NS>
__device__ inline double pick(const double (&x)[NS], int idx) {
  double v = 0.0;
#pragma unroll
  for (int t = 0; t < NS; ++t)
    if (t == (idx >> 6)) v = x[t];
  return __shfl(v, idx & 63, 64);
}

// Lane permutation of a float64 by DPP (both 32-bit halves moved alike).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double lane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
// Sum over the 64 lanes, the same in every lane: exchanges within 16-lane
// rows by DPP (lane xor 1, xor 2, half-row mirror, row mirror), then the four
// row sums read from lanes 0, 16, 32, 48; a fixed order throughout.
__device__ inline double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

template <class T> __device__ inline T warp_min(T v) {
  for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, 64); v = v < w ? v : w; }
  return v;
}

// Number of eigenvalues of T (diagonal dl, squared off-diagonal e2l) below
// x0 and x1, evaluated together.  A pivot smaller than pivmin in magnitude is
// replaced by -pivmin, which keeps the recurrence finite.
// 1/x from the hardware estimate and one Newton-Raphson step (relative
// error about 2^-50, which perturbs the counts as a change of e^2 in the last
// bits would)
__device__ inline double rcp_nr1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ inline void sturm2(const double* dl, const double* e2l, int n, double pivmin, double x0, double x1,
                              int& c0, int& c1) {
  double q0 = dl[0] - x0, q1 = dl[0] - x1;
  if (fabs(q0) < pivmin) q0 = -pivmin;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  c0 = q0 < 0.0;
  c1 = q1 < 0.0;
  for (int i = 1; i < n; ++i) {
    const double di = dl[i], ee = e2l[i - 1];
    q0 = (di - x0) - ee * rcp_nr1(q0);
    q1 = (di - x1) - ee * rcp_nr1(q1);
    if (fabs(q0) < pivmin) q0 = -pivmin;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    c0 += q0 < 0.0;
    c1 += q1 < 0.0;
  }
}

__device__ inline double start_entry(int i, int r) {
  // fixed pseudo-random start vector entry in (-1, 1) (an integer hash)
  uint32_t h = (uint32_t)i * 0x9E3779B1u ^ ((uint32_t)r + 1u) * 0x85EBCA77u;
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  return ((double)h + 0.5) * 0x1p-31 - 1.0;
}

__device__ inline double away_from_zero(double u, double tol) {
  return fabs(u) < tol ? (u < 0.0 ? -tol : tol) : u;
}

// Barrier of the G workgroups of one matrix: arrive on a counter (release),
// poll it (acquire) until all have arrived for this step.  The polling is
// bounded: on time-out *failed (LDS, read by thread 0 only) is raised and
// later barriers no longer wait, so a lost arrival ends the launch with an
// error flag instead of a hang.
__device__ inline void group_barrier(unsigned* cnt, unsigned target, int* failed, unsigned limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    if (limit == 0) *failed = 1;
    while (!*failed && __hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > limit) *failed = 1;
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

// Step 1.  Workgroup gi of matrix m holds rows i = gi, gi + G, ... of the
// upper triangle, packed in LDS (row i from column i on).  Row i is walked by
// wave (local row) % 16, column j by lane j % 64.
template <int NS>
__global__ void __launch_bounds__(RED_THREADS) eig_reduce_kernel(EigArgs g) {
  constexpr int NM = 64 * NS;
  extern __shared__ __attribute__((aligned(16))) double sm[];
  double* Vb = sm;                 // [2][NM] reflectors of this and the previous step
  double* Wb = Vb + 2 * NM;        // [2][NM] their rank-2 partners
  double* cacc = Wb + 2 * NM;      // [16][NM] per-wave column sums of the product
  double* rowsum = cacc + RED_WAVES * NM;   // row sums of the product (own rows)
  double* rowbuf = rowsum + NM;    // the next reflector's row
  double* dsh = rowbuf + NM;       // diagonal, off-diagonal and tau of T, written out at the end
  double* esh = dsh + NM;
  double* tsh = esh + NM;
  double* red = tsh + NM;          // scalars
  double* rows = red + 128;        // packed rows; reflector k replaces row k once used

  const int m = blockIdx.y, gi = blockIdx.x;
  const int n = g.n[m], G = g.G[m];
  if (gi >= G) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Z = g.Z[m];
  double* H = g.A[m];              // reflector k is written to row k (columns k+2..)
  const int nr = (n - gi + G - 1) / G;
  auto roff = [&](int r) { return r * (n - gi) - G * (r * (r - 1) / 2); };   // start of local row r

  for (int r = wave; r < nr; r += RED_WAVES) {
    const int i = gi + r * G, base = roff(r) - i;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      if (j >= i && j < n) rows[base + j] = Z[i * n + j];
    }
  }
  for (int j = tid; j < 4 * NM; j += RED_THREADS) Vb[j] = 0.0;   // Vb and Wb
  if (wave == 0) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      rowbuf[j] = j < n ? Z[j] : 0.0;
    }
  }
  int* failed = (int*)(red + 63);
  if (tid == 0) *failed = 0;
  __syncthreads();

  // Reflector k (wave 0, identical in every workgroup) from rowbuf = row k
  // after the updates of steps up to k-2, minus the update of step k-1:
  // v = x - beta e_{k+1} scaled so that v_{k+1} = 1, tau = (beta - alpha) / beta,
  // beta = -sign(alpha) ||x||, x the part of the row beyond the diagonal.
  auto reflector = [&](int k, const double* Vp, const double* Wp, double* Vn) {
    const double vpk = Vp[k], wpk = Wp[k];
    double x[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      x[t] = (j >= k && j < n) ? fma(-vpk, Wp[j], fma(-wpk, Vp[j], rowbuf[j])) : 0.0;
    }
    const double dk = pick(x, k), alpha = pick(x, k + 1);
    double s2 = 0.0;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      if (j >= k + 2 && j < n) s2 = fma(x[t], x[t], s2);
    }
    s2 = wave_sum(s2);
    double tk = 0.0, beta = alpha, scal = 0.0;
    if (s2 > 0.0) {
      const double r = sqrt(fma(alpha, alpha, s2));
      beta = alpha >= 0.0 ? -r : r;
      tk = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const bool own = k % G == gi;
    const int kbase = roff((k - gi) / G) - k;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      const double v = j == k + 1 ? 1.0 : (j >= k + 2 && j < n ? x[t] * scal : 0.0);
      Vn[j] = v;
      if (own && j >= k + 2 && j < n) rows[kbase + j] = v;
    }
    if (lane == 0) {
      dsh[k] = dk;
      esh[k] = beta;
      tsh[k] = tk;
      red[0] = tk;
    }
  };

  if (wave == 0 && n >= 3) reflector(0, Vb + NM, Wb + NM, Vb);   // the other buffers are still zero
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int cur = k & 1;
    double* Vc = Vb + cur * NM;
    double* Wc = Wb + cur * NM;
    double* Vp = Vb + (cur ^ 1) * NM;
    double* Wp = Wb + (cur ^ 1) * NM;
    const double tk = red[0];

    // own rows i >= k+1: apply the previous step's update A -= v w^T + w v^T
    // and accumulate y = A v (row sums across lanes, column sums per lane)
    double vcj[NS], vpj[NS], wpj[NS], csum[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      vcj[t] = Vc[64 * t + lane];
      vpj[t] = Vp[64 * t + lane];
      wpj[t] = Wp[64 * t + lane];
      csum[t] = 0.0;
    }
    const int r0 = k + 1 > gi ? (k + 1 - gi + G - 1) / G : 0;
    for (int r = r0 + wave; r < nr; r += RED_WAVES) {
      const int i = gi + r * G, base = roff(r) - i;
      const double vci = Vc[i], vpi = Vp[i], wpi = Wp[i];
      double rs = 0.0;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int j = 64 * t + lane;
        if (j >= i && j < n) {
          const double a = fma(-vpi, wpj[t], fma(-wpi, vpj[t], rows[base + j]));
          rows[base + j] = a;
          rs = fma(a, vcj[t], rs);
          if (j > i) csum[t] = fma(a, vci, csum[t]);
          if (i == k + 1) rowbuf[j] = a;
        }
      }
      rs = wave_sum(rs);
      if (lane == 0) rowsum[i] = rs;
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) cacc[wave * NM + 64 * t + lane] = csum[t];
    __syncthreads();

    // y = A v for j > k into rowsum: this workgroup's row and column sums,
    // plus (G > 1) the other workgroups' parts and row k+1 from its owner,
    // exchanged through global memory, added in a fixed order
    const int par = k & 1;
    double* Pp = g.P[m] + (size_t)par * G * n;
    double* RBp = g.RB[m] + (size_t)par * n;
    for (int j = tid; j < n; j += RED_THREADS) {
      if (j > k) {
        double y = (j - gi) % G == 0 ? rowsum[j] : 0.0;
#pragma unroll
        for (int w = 0; w < RED_WAVES; ++w) y += cacc[w * NM + j];
        if (G > 1) {
          Pp[gi * n + j] = y;
          if ((k + 1) % G == gi) RBp[j] = rowbuf[j];
        } else {
          rowsum[j] = y;
        }
      }
    }
    if (G > 1) {
      group_barrier(g.cnt[m], (unsigned)(k + 1) * (unsigned)G, failed, g.spin_limit);
      for (int j = tid; j < n; j += RED_THREADS) {
        if (j > k) {
          double y = 0.0;
#pragma unroll 4
          for (int q = 0; q < G; ++q) y += Pp[q * n + j];
          rowsum[j] = y;
          rowbuf[j] = RBp[j];
        }
      }
    }
    __syncthreads();

    if (wave == 0) {
      // p = tau y, K = tau p^T v / 2, w = p - K v; then the next reflector
      // from row k+1
      double pj[NS], pv = 0.0;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int j = 64 * t + lane;
        pj[t] = (j > k && j < n) ? tk * rowsum[j] : 0.0;
        pv = fma(pj[t], vcj[t], pv);
      }
      const double K = 0.5 * tk * wave_sum(pv);
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int j = 64 * t + lane;
        Wc[j] = (j > k && j < n) ? fma(-K, vcj[t], pj[t]) : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
      if (k + 3 < n) reflector(k + 1, Vc, Wc, Vp);
    }
    __syncthreads();
  }

  // the last 2 x 2 block: row n-2 (rowbuf) and entry (n-1, n-1) (its owner)
  // after the last update; then T and the reflectors go out
  if (tid == 0) {
    if (n <= 2) {
      dsh[0] = Z[0];
      esh[0] = n == 2 ? Z[1] : 0.0;
      if (n == 2) dsh[1] = Z[3];
    } else {
      const int c = (n - 3) & 1, p = n - 2, q = n - 1;
      const double* Vc = Vb + c * NM;
      const double* Wc = Wb + c * NM;
      dsh[p] = fma(-Vc[p], Wc[p], fma(-Wc[p], Vc[p], rowbuf[p]));
      esh[p] = fma(-Vc[p], Wc[q], fma(-Wc[p], Vc[q], rowbuf[q]));
      if (q % G == gi) g.d[m][q] = fma(-Vc[q], Wc[q], fma(-Wc[q], Vc[q], rows[roff((q - gi) / G)]));
    }
    if (*failed && g.info[m]) g.info[m][0] = 1;
  }
  __syncthreads();
  if (gi == 0) {
    for (int i = tid; i < n; i += RED_THREADS) {
      if (i < n - 1 || n <= 2) g.d[m][i] = dsh[i];
      g.e[m][i] = i < n - 1 ? esh[i] : 0.0;
      g.tau[m][i] = i + 2 < n ? tsh[i] : 0.0;
    }
  }
  for (int r = wave; r < nr; r += RED_WAVES) {
    const int k = gi + r * G, base = roff(r) - k;
    if (k + 2 >= n) continue;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      if (j >= k + 2 && j < n) H[k * n + j] = rows[base + j];
    }
  }
}

// Bounds of the spectrum of T (wave 0 of a workgroup, from d and e in
// global memory): out[0] = ||T|| (max row sum), out[1] = the pivot floor of
// the Sturm counts, out[2], out[3] = Gershgorin lower and upper bounds;
// e2l[i] = e_i^2.
template <int NS>
__device__ inline void spectrum_bounds(const double* d, const double* e, int n, int lane, double* e2l,
                                       double* out) {
  double rmax = 0.0, e2max = 0.0, lo = DBL_MAX, hi = -DBL_MAX;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int i = 64 * t + lane;
    if (i < n) {
      const double ei = e[i], off = fabs(ei) + (i > 0 ? fabs(e[i - 1]) : 0.0);
      rmax = fmax(rmax, fabs(d[i]) + off);
      e2max = fmax(e2max, ei * ei);
      lo = fmin(lo, d[i] - off);
      hi = fmax(hi, d[i] + off);
      e2l[i] = ei * ei;
    }
  }
  rmax = warp_max(rmax);
  e2max = warp_max(e2max);
  lo = warp_min(lo);
  hi = warp_max(hi);
  if (lane == 0) {
    out[0] = rmax;
    out[1] = DBL_MIN * fmax(1.0, e2max);
    out[2] = lo;
    out[3] = hi;
  }
}

// Step 2: the R largest eigenvalues of T by multisection on Sturm counts
// (the number of negative pivots of the LDL^T factorisation of T - x I is
// the number of eigenvalues below x).  A workgroup of BIS_WAVES waves takes
// one eigenvalue and tests 128 points per wave a round (P = 128 BIS_WAVES),
// so the interval shrinks P + 1-fold per round: 6 rounds to float64 accuracy
// with four waves, against 8 with one (each round is a sequential Sturm
// count, the cost).  The waves add their counts in LDS; every wave then holds
// the same interval, so all take the same exits.  Grid (R, matrices).
constexpr int BIS_WAVES = 4;

template <int NS>
__global__ void __launch_bounds__(64 * BIS_WAVES) eig_bisect_kernel(EigArgs g) {
  constexpr int NM = 64 * NS;
  __shared__ double dl[NM], e2l[NM], bnd[4];
  __shared__ int cnt[2][BIS_WAVES];
  const int m = blockIdx.y;
  const int n = g.n[m], R = g.R[m];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = (int)blockIdx.x;
  if (r >= R) return;                              // the same for the whole workgroup
  for (int i = tid; i < n; i += blockDim.x) dl[i] = g.d[m][i];
  if (wave == 0) spectrum_bounds<NS>(g.d[m], g.e[m], n, lane, e2l, bnd);
  __syncthreads();
  const double tnorm = bnd[0], pivmin = bnd[1];
  const double margin = 2.0 * n * EPS * tnorm + 2.0 * pivmin;
  const double atol = EPS * tnorm;
  constexpr int P = 128 * BIS_WAVES;               // points a round
  const int kk = n - 1 - r;                        // ascending index of the eigenvalue
  double lo = bnd[2] - margin, hi = bnd[3] + margin;
  // lo and hi are the same in every thread, so the loop is uniform
  for (int it = 0; it < 96; ++it) {
    if (hi - lo <= fmax(atol, 2.0 * EPS * fmax(fabs(lo), fabs(hi)))) break;
    const double wd = hi - lo;
    const int q = 128 * wave + lane;               // this lane's points q and q + 64
    const double x0 = lo + wd * ((double)(q + 1) / (double)(P + 1));
    const double x1 = lo + wd * ((double)(q + 65) / (double)(P + 1));
    int c0, c1;
    sturm2(dl, e2l, n, pivmin, x0, x1, c0, c1);
    const int nw = __popcll(__ballot(c0 <= kk)) + __popcll(__ballot(c1 <= kk));
    if (lane == 0) cnt[it & 1][wave] = nw;
    __syncthreads();
    int nb = 0;
#pragma unroll
    for (int w = 0; w < BIS_WAVES; ++w) nb += cnt[it & 1][w];
    const double nlo = nb > 0 ? lo + wd * ((double)nb / (double)(P + 1)) : lo;
    const double nhi = nb < P ? lo + wd * ((double)(nb + 1) / (double)(P + 1)) : hi;
    const bool progress = nhi - nlo < wd;          // false once float64 cannot split further
    lo = nlo;
    hi = nhi;
    if (!progress) break;
  }
  if (tid == 0) g.lam[m][r] = 0.5 * (lo + hi);
}

// Step 3 for one matrix per workgroup, from d and e of T and the eigenvalues.
template <int NS>
__global__ void __launch_bounds__(SOLVE_THREADS) eig_solve_kernel(EigArgs g) {
  constexpr int NM = 64 * NS;
  extern __shared__ __attribute__((aligned(16))) double sm[];
  double* dl = sm;
  double* el = dl + NM;
  double* e2l = el + NM;
  double* laml = e2l + NM;
  double* shl = laml + NM;
  double* red = shl + NM;          // 64 scalars
  int* cl = (int*)(red + 64);      // cluster starts (NM + 1)

  const int m = blockIdx.x;
  const int n = g.n[m], R = g.R[m];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < n; i += SOLVE_THREADS) {
    dl[i] = g.d[m][i];
    el[i] = g.e[m][i];
  }
  __syncthreads();

  // the spectrum's bounds, and the eigenvalues from eig_bisect_kernel
  if (wave == 0) spectrum_bounds<NS>(g.d[m], g.e[m], n, lane, e2l, red + 32);
  for (int r = tid; r < R; r += SOLVE_THREADS) laml[r] = g.lam[m][r];
  __syncthreads();
  const double tnorm = red[32];

  // ---- 3. eigenvectors of T by inverse iteration
  if (tid == 0) {
    // clusters of close eigenvalues; equal shifts within a cluster are
    // separated by a few ulps so that the factorisations differ
    const double ortol = 1e-3 * tnorm;
    int ncl = 0;
    for (int r = 0; r < R; ++r) {
      double s = laml[r];
      if (r == 0 || laml[r - 1] - laml[r] > ortol) {
        cl[ncl++] = r;
      } else {
        const double pt = 10.0 * EPS * fmax(fabs(s), EPS * tnorm);
        if (shl[r - 1] - s < pt) s = shl[r - 1] - pt;
      }
      shl[r] = s;
    }
    cl[ncl] = R;
    red[36] = (double)ncl;
  }
  __syncthreads();
  const int ncl = (int)red[36];
  const double ptol = tnorm > 0.0 ? EPS * tnorm : DBL_MIN;
  double* __restrict__ X = g.X[m];
  double* __restrict__ Y = g.Y[m];
  double* __restrict__ ainv = g.ainv[m];
  double* __restrict__ bu = g.bu[m];
  double* __restrict__ du = g.du[m];
  double* __restrict__ cm = g.cm[m];
  unsigned char* __restrict__ piv = g.piv[m];
  if (tid < R) {
    // pivoted LU of T - s I (U with two superdiagonals), and the start vector
    const int r = tid;
    const double s = shl[r];
    double* xr = X + r * n;
    double acur = dl[0] - s, bcur = n > 1 ? el[0] : 0.0;
    // branch-free: the pivot choice only selects operands
    for (int k = 0; k + 1 < n; ++k) {
      const double ck = el[k], an = dl[k + 1] - s, bn = k + 2 < n ? el[k + 1] : 0.0;
      const int o = k * R + r;
      const bool swap = fabs(acur) < fabs(ck);
      const double piv_v = swap ? ck : acur;          // U(k, k)
      const double other = swap ? acur : ck;          // entry eliminated below it
      const double mult = piv_v != 0.0 ? other * rcp_nr(piv_v) : 0.0;
      ainv[o] = rcp_nr(away_from_zero(piv_v, ptol));
      bu[o] = swap ? an : bcur;
      du[o] = swap ? bn : 0.0;
      cm[o] = mult;
      piv[o] = swap ? 1 : 0;
      const double na = swap ? fma(-mult, an, bcur) : fma(-mult, bcur, an);
      bcur = swap ? -mult * bn : bn;
      acur = na;
      xr[k] = start_entry(k, r);
    }
    const int o = (n - 1) * R + r;
    ainv[o] = rcp_nr(away_from_zero(acur, ptol));
    bu[o] = 0.0;
    du[o] = 0.0;
    xr[n - 1] = start_entry(n - 1, r);
  }
  for (int it = 0; it < EIG_ITERS; ++it) {
    if (tid < R) {
      // entries of x are at most 1 (start vector, then unit vectors); y =
      // ptol x keeps the solve finite: x <- U^-1 L^-1 P y
      const int r = tid;
      double* xr = X + r * n;
      double* yr = Y + r * n;
      // blocks of steps: all inputs of a block are loaded before any of its
      // results is stored, so that the loads overlap; each block waits about
      // one memory latency, so the blocks are as long as the registers allow
      // (32 steps forward, 24 backward)
      constexpr int B = 32;
      double yk = xr[0] * ptol;
      for (int k0 = 0; k0 + 1 < n; k0 += B) {
        double xv[B], mv[B];
        bool sv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          const int k = k0 + u < n - 1 ? k0 + u : n - 2;
          xv[u] = xr[k + 1];
          mv[u] = cm[k * R + r];
          sv[u] = piv[k * R + r] != 0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
          if (k0 + u + 1 < n) {
            // rows k and k+1 exchanged when piv: (top, bottom) = (y_{k+1}, y_k)
            const double yn = xv[u] * ptol;
            const double top = sv[u] ? yn : yk, bot = sv[u] ? yk : yn;
            yr[k0 + u] = top;
            yk = fma(-mv[u], top, bot);
          }
        }
      }
      yr[n - 1] = yk;
      double x1 = 0.0, x2 = 0.0;
      constexpr int BB = 24;
      for (int k0 = n - 1; k0 >= 0; k0 -= BB) {
        double yv[BB], dv[BB], bv[BB], av[BB];
#pragma unroll
        for (int u = 0; u < BB; ++u) {
          const int k = k0 - u >= 0 ? k0 - u : 0;
          yv[u] = yr[k];
          dv[u] = du[k * R + r];
          bv[u] = bu[k * R + r];
          av[u] = ainv[k * R + r];
        }
#pragma unroll
        for (int u = 0; u < BB; ++u) {
          if (k0 - u >= 0) {
            const double xk = fma(-dv[u], x2, fma(-bv[u], x1, yv[u])) * av[u];
            xr[k0 - u] = xk;
            x2 = x1;
            x1 = xk;
          }
        }
      }
    }
    __syncthreads();
    // modified Gram-Schmidt inside each cluster, then unit 2-norm
    for (int c = wave; c < ncl; c += SOLVE_WAVES) {
      const int s0 = cl[c], s1 = cl[c + 1];
      for (int j = s0; j < s1; ++j) {
        double xj[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const int i = 64 * t + lane;
          const double v = X[j * n + (i < n ? i : n - 1)];
          xj[t] = i < n ? v : 0.0;
        }
        for (int p = s0; p < j; ++p) {
          double xp[NS], dot = 0.0;
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            const int i = 64 * t + lane;
            const double v = X[p * n + (i < n ? i : n - 1)];
            xp[t] = i < n ? v : 0.0;
            dot = fma(xp[t], xj[t], dot);
          }
          dot = wave_sum(dot);
#pragma unroll
          for (int t = 0; t < NS; ++t) xj[t] = fma(-dot, xp[t], xj[t]);
        }
        double nn = 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) nn = fma(xj[t], xj[t], nn);
        nn = wave_sum(nn);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const int i = 64 * t + lane;
          if (i < n) X[j * n + i] = xj[t] * inv;
        }
      }
    }
    __syncthreads();
  }
}

// Step 4: x <- H_0 H_1 ... H_{n-3} x for eigenvector r of matrix m (one wave),
// written as row r of Vt.
template <int NS>
__global__ void __launch_bounds__(64) eig_back_kernel(EigArgs g) {
  const int r = blockIdx.x, m = blockIdx.y, lane = threadIdx.x;
  const int n = g.n[m], R = g.R[m];
  if (r >= R) return;
  __shared__ double taus[64 * NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int i = 64 * t + lane;
    taus[i] = i < n ? g.tau[m][i] : 0.0;
  }
  __syncthreads();
  const double* A = g.A[m];
  const double* X = g.X[m];
  double x[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int i = 64 * t + lane;
    x[t] = i < n ? X[r * n + i] : 0.0;
  }
  // row k of A from a clamped address, and tau_k; the reflector (1 at k+1,
  // zero before) is formed from the row at use, so that the loads stay in
  // flight.  A zero tau gives a zero update, so no branch waits on it.
  auto load_v = [&](int k, double (&v)[NS], double& tk) {
    const int kc = k >= 0 ? k : 0;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      v[t] = A[kc * n + (j < n ? j : n - 1)];
    }
    tk = taus[kc];
  };
  auto apply = [&](int k, const double (&a)[NS], double tk) {
    if (k < 0) return;                             // uniform: past the last reflector
    double v[NS], dot = 0.0;
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int j = 64 * t + lane;
      v[t] = j == k + 1 ? 1.0 : (j >= k + 2 && j < n ? a[t] : 0.0);
      dot = fma(v[t], x[t], dot);
    }
    const double f = tk * wave_sum(dot);
#pragma unroll
    for (int t = 0; t < NS; ++t) x[t] = fma(-f, v[t], x[t]);
  };
  // reflectors n-3 down to 0, BD in flight: each waits on its row about a
  // memory latency after the request, so the ring holds enough rows to
  // cover it (one wave per workgroup, registers to spare)
  constexpr int BD = 16;
  double vr[BD][NS], tr[BD];
  int k = n - 3;
#pragma unroll
  for (int u = 0; u < BD; ++u) load_v(k - u, vr[u], tr[u]);
  for (; k >= 0; k -= BD) {
#pragma unroll
    for (int u = 0; u < BD; ++u) {
      apply(k - u, vr[u], tr[u]);
      load_v(k - u - BD, vr[u], tr[u]);
    }
  }
  double* out = g.Vt[m] + (size_t)r * n;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int j = 64 * t + lane;
    if (j < n) out[j] = x[t];
  }
}

size_t solve_lds_bytes(int ns) {
  const int nm = 64 * ns;
  return (size_t)(5 * nm + 64) * 8 + (size_t)(nm + 1) * 4;
}
size_t reduce_fixed_bytes(int ns) { return (size_t)((9 + RED_WAVES) * 64 * ns + 128) * 8; }

// Smallest G whose largest share of packed rows fits in LDS beside the rest
// (0: none up to RED_GMAX); rows_cap receives that share in doubles.
int reduce_groups(int64_t n, int64_t& rows_cap) {
  const int ns = (int)ceil_div(n, 64);
  for (int G = 1; G <= RED_GMAX && G <= n; ++G) {
    int64_t rows = 0;
    for (int64_t i = 0; i < n; i += G) rows += n - i;   // group 0 holds the most
    if (reduce_fixed_bytes(ns) + (size_t)rows * 8 <= LDS_BYTES) {
      rows_cap = rows;
      return G;
    }
  }
  return 0;
}

struct Layout {
  size_t A, d, e, tau, X, Y, ainv, bu, du, cm, piv, P, RB, cnt, total;
};
inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
Layout layout(int64_t n, int64_t R) {
  Layout L;
  size_t o = 0;
  int64_t cap = 0;
  const int G = std::max(1, reduce_groups(n, cap));
  auto take = [&](size_t bytes) { const size_t at = o; o = al256(o + bytes); return at; };
  L.A = take((size_t)n * n * 8);
  L.d = take((size_t)n * 8);
  L.e = take((size_t)n * 8);
  L.tau = take((size_t)n * 8);
  L.X = take((size_t)n * R * 8);
  L.Y = take((size_t)n * R * 8);
  L.ainv = take((size_t)n * R * 8);
  L.bu = take((size_t)n * R * 8);
  L.du = take((size_t)n * R * 8);
  L.cm = take((size_t)n * R * 8);
  L.piv = take((size_t)n * R);
  L.P = take((size_t)2 * G * n * 8);
  L.RB = take((size_t)2 * n * 8);
  L.cnt = take(64);
  L.total = o;
  return L;
}

template <int NS>
hipError_t launch_ns(EigArgs& a, int nmat, int gmax, int64_t rows_cap, int rmax, bool coop, hipStream_t st) {
  hipError_t e;
  const size_t rshm = reduce_fixed_bytes(NS) + (size_t)rows_cap * 8;
  if ((e = hipFuncSetAttribute((const void*)eig_reduce_kernel<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)rshm)) != hipSuccess)
    return e;
  if (gmax > 1) {
    // the workgroups of a matrix wait for each other: a cooperative launch
    // guarantees that they are all resident.  An ordinary launch (coop false,
    // for a solve that runs beside other work) relies on the few workgroups
    // becoming resident as the device frees room; the barrier's bounded spin
    // reports a failure rather than waiting for ever.
    for (int k = 0; k < nmat; ++k)
      if (a.G[k] > 1 && (e = fill_zero(a.cnt[k], 64, st)) != hipSuccess) return e;
    if (coop) {
      void* args[] = {&a};
      e = hipLaunchCooperativeKernel((const void*)eig_reduce_kernel<NS>, dim3(gmax, nmat), dim3(RED_THREADS), args,
                                     rshm, st);
      if (e != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(eig_reduce_kernel<NS>, dim3(gmax, nmat), dim3(RED_THREADS), rshm, st, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  } else {
    hipLaunchKernelGGL(eig_reduce_kernel<NS>, dim3(1, nmat), dim3(RED_THREADS), rshm, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const size_t sshm = solve_lds_bytes(NS);
  if ((e = hipFuncSetAttribute((const void*)eig_solve_kernel<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sshm)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(eig_bisect_kernel<NS>, dim3((unsigned)rmax, nmat), dim3(64 * BIS_WAVES), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(eig_solve_kernel<NS>, dim3(nmat), dim3(SOLVE_THREADS), sshm, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(eig_back_kernel<NS>, dim3(rmax, nmat), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace

bool eig_top_ok(int64_t n, int64_t R) {
  int64_t cap;
  return n >= 1 && n <= 64 * EIG_NS_MAX && R >= 1 && R <= n && reduce_groups(n, cap) > 0;
}

size_t eig_top_work_bytes(int64_t n, int64_t R) { return layout(n, R).total; }

hipError_t eig_top_batched(int nmat, const double* const* Z, const int64_t* ns, const int64_t* Rs,
                           double* const* lam, double* const* Vt, void* const* work, int* const* info,
                           hipStream_t st, bool coop) {
  if (nmat <= 0) return hipSuccess;
  if (nmat > EIG_MAXB) return hipErrorInvalidValue;
  EigArgs a = {};
  // RBKI_EIG_SPIN_LIMIT: barrier polls of a multi-workgroup reduction before
  // it gives up and reports failure (0: at once), to test the error path
  a.spin_limit = SPIN_LIMIT;
  if (const char* lim = getenv("RBKI_EIG_SPIN_LIMIT")) a.spin_limit = (unsigned)strtoul(lim, nullptr, 10);
  int64_t nmax = 0, rmax = 0, rows_cap = 0;
  int gmax = 1;
  for (int k = 0; k < nmat; ++k) {
    if (!eig_top_ok(ns[k], Rs[k])) return hipErrorInvalidValue;
    const Layout L = layout(ns[k], Rs[k]);
    char* w = (char*)work[k];
    a.Z[k] = Z[k];
    a.n[k] = (int)ns[k];
    a.R[k] = (int)Rs[k];
    a.A[k] = (double*)(w + L.A);
    a.d[k] = (double*)(w + L.d);
    a.e[k] = (double*)(w + L.e);
    a.tau[k] = (double*)(w + L.tau);
    a.X[k] = (double*)(w + L.X);
    a.Y[k] = (double*)(w + L.Y);
    a.ainv[k] = (double*)(w + L.ainv);
    a.bu[k] = (double*)(w + L.bu);
    a.du[k] = (double*)(w + L.du);
    a.cm[k] = (double*)(w + L.cm);
    a.piv[k] = (unsigned char*)(w + L.piv);
    a.lam[k] = lam[k];
    a.Vt[k] = Vt[k];
    a.info[k] = info ? info[k] : nullptr;
    int64_t cap = 0;
    a.G[k] = reduce_groups(ns[k], cap);
    a.P[k] = (double*)(w + L.P);
    a.RB[k] = (double*)(w + L.RB);
    a.cnt[k] = (unsigned*)(w + L.cnt);
    gmax = std::max(gmax, a.G[k]);
    rows_cap = std::max(rows_cap, cap);
    nmax = std::max(nmax, ns[k]);
    rmax = std::max(rmax, Rs[k]);
  }
  switch ((int)ceil_div(nmax, 64)) {
    case 1: return launch_ns<1>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
    case 2: return launch_ns<2>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
    case 3: return launch_ns<3>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
    case 4: return launch_ns<4>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
    case 5: return launch_ns<5>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
    case 6: return launch_ns<6>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
    case 7: return launch_ns<7>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
    default: return launch_ns<8>(a, nmat, gmax, rows_cap, (int)rmax, coop, st);
  }
}

}  // namespace rbki
